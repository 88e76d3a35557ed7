// Sweep kernels of the FP64 populations storage format (all source kinds, K1 modes and launch
// shapes), instantiated in this translation unit alone.

#include "btrt_device.h"

namespace btrtk {

hipError_t sweep_f64(const SweepArgs<double>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s)
{
    return sweep_with<Plain<double>>(a, src_kind, kmode, cfg, s);
}

LaunchCfg resolve_f64(const SweepArgs<double>& a, int src_kind, int kmode, const LaunchCfg& cfg)
{
    return resolve_with<Plain<double>>(a, src_kind, kmode, cfg);
}

}  // namespace btrtk
