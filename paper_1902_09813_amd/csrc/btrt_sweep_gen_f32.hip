// Sweep kernels of the general node model (power-law flux, phi-dependent source, wall table)
// with plain FP32 storage (all source kinds, K1 modes and launch shapes), instantiated in
// this translation unit alone.

#include "btrt_device.h"

namespace btrtk {

hipError_t sweep_gen_f32(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s)
{
    return sweep_with_gen<Plain<float>>(a, src_kind, kmode, cfg, s);
}

LaunchCfg resolve_gen_f32(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg)
{
    return resolve_with_gen<Plain<float>>(a, src_kind, kmode, cfg);
}

}  // namespace btrtk
