// Sweep kernels of the FP16 scaled deviations storage format (all source kinds, K1 modes and launch
// shapes), instantiated in this translation unit alone.

#include "btrt_device.h"

namespace btrtk {

hipError_t sweep_f16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s)
{
    return sweep_with<Dev<F16Codec>>(a, src_kind, kmode, cfg, s);
}

LaunchCfg resolve_f16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg)
{
    return resolve_with<Dev<F16Codec>>(a, src_kind, kmode, cfg);
}

}  // namespace btrtk
