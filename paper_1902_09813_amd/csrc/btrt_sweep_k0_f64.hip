// Sweep kernels of the F64 populations storage format for k0 = 1 (kK0One: the collision
// drops its (1 - k0) f_i term), all source kinds, K1 modes and launch shapes, instantiated in
// this translation unit alone.

#include "btrt_device.h"

namespace btrtk {

hipError_t sweep_k0_f64(const SweepArgs<double>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s)
{
    return sweep_with_k0<Plain<double>>(a, src_kind, kmode, cfg, s);
}

LaunchCfg resolve_k0_f64(const SweepArgs<double>& a, int src_kind, int kmode, const LaunchCfg& cfg)
{
    return resolve_with_k0<Plain<double>>(a, src_kind, kmode, cfg);
}

}  // namespace btrtk
