// Sweep kernels of the BF16 scaled deviations storage format (all source kinds, K1 modes and launch
// shapes), instantiated in this translation unit alone.

#include "btrt_device.h"

namespace btrtk {

hipError_t sweep_bf16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s)
{
    return sweep_with<Dev<BF16Codec>>(a, src_kind, kmode, cfg, s);
}

LaunchCfg resolve_bf16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg)
{
    return resolve_with<Dev<BF16Codec>>(a, src_kind, kmode, cfg);
}

}  // namespace btrtk
