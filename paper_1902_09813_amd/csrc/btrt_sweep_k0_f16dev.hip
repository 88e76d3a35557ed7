// Sweep kernels of the FP16 scaled-deviation storage format for k0 = 1 (kK0One: the collision drops
// its (1 - k0) f_i term), all source kinds, K1 modes and launch shapes, instantiated in this
// translation unit alone.

#include "btrt_device.h"

namespace btrtk {

hipError_t sweep_k0_f16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s)
{
    return sweep_with_k0<Dev<F16Codec>>(a, src_kind, kmode, cfg, s);
}

LaunchCfg resolve_k0_f16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg)
{
    return resolve_with_k0<Dev<F16Codec>>(a, src_kind, kmode, cfg);
}

}  // namespace btrtk
