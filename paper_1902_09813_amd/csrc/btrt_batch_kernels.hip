// Launchers of the batched kernels (one persistent launch over the tiles or strips of every
// instance of a batch or server round).

#include "btrt_device.h"

namespace btrtk {

template <typename T, int K0>
hipError_t launch_batch_sweep_k0(const BatchEntry<T>* ent, const int* begin, const int* par, int ninst, int total_tiles,
                                 int flip, int steps, int grid, int rows, bool nts, hipStream_t s)
{
    if (batch_walks(steps)) {
        // Several resident strips per CU: a persistent grid of `grid` blocks covers the list.
        const unsigned g = static_cast<unsigned>(grid > 0 ? std::min(grid * kWalkGroup, total_tiles) : total_tiles);
        if (steps == 4)
            hipLaunchKernelGGL((batchw_kernel<T, 4, K0>), dim3(g), dim3(kWave), 0, s, ent, begin, par, ninst,
                               total_tiles, flip, rows);
        else if (steps == 6)
            hipLaunchKernelGGL((batchw_kernel<T, 6, K0>), dim3(g), dim3(kWave), 0, s, ent, begin, par, ninst,
                               total_tiles, flip, rows);
        else
            hipLaunchKernelGGL((batchw_kernel<T, 7, K0>), dim3(g), dim3(kWave), 0, s, ent, begin, par, ninst,
                               total_tiles, flip, rows);
        return hipGetLastError();
    }
    const unsigned g = static_cast<unsigned>(grid > 0 ? std::min(grid, total_tiles) : total_tiles);
    if (steps == 2 && nts)
        hipLaunchKernelGGL((batch2_kernel<T, K0, true>), dim3(g), dim3(kBlock2), 0, s, ent, begin, par, ninst,
                           total_tiles, flip);
    else if (steps == 2)
        hipLaunchKernelGGL((batch2_kernel<T, K0, false>), dim3(g), dim3(kBlock2), 0, s, ent, begin, par, ninst,
                           total_tiles, flip);
    else if (nts)
        hipLaunchKernelGGL((batch1_kernel<T, K0, true>), dim3(g), dim3(kBlock), 0, s, ent, begin, par, ninst,
                           total_tiles, flip);
    else
        hipLaunchKernelGGL((batch1_kernel<T, K0, false>), dim3(g), dim3(kBlock), 0, s, ent, begin, par, ninst,
                           total_tiles, flip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_sweep(const BatchEntry<T>* ent, const int* begin, const int* par, int ninst, int total_tiles,
                              int flip, int steps, int grid, int rows, bool k0one, bool nts, hipStream_t s)
{
    if (total_tiles <= 0 || ninst <= 0) return hipSuccess;
    return k0one ? launch_batch_sweep_k0<T, kK0One>(ent, begin, par, ninst, total_tiles, flip, steps, grid, rows, nts, s)
                 : launch_batch_sweep_k0<T, 0>(ent, begin, par, ninst, total_tiles, flip, steps, grid, rows, nts, s);
}

int batch_strip_columns(int steps)
{
    return steps == 4 ? Walk<4>::W : (steps == 6 ? Walk<6>::W : Walk<7>::W);
}

int tile_rows(int steps, int precision_bytes)
{
    if (steps == 2) return precision_bytes == 8 ? Tile2<double>::TY : Tile2<float>::TY;
    return kTileY;
}

template hipError_t launch_batch_sweep<double>(const BatchEntry<double>*, const int*, const int*, int, int, int, int,
                                               int, int, bool, bool, hipStream_t);
template hipError_t launch_batch_sweep<float>(const BatchEntry<float>*, const int*, const int*, int, int, int, int,
                                              int, int, bool, bool, hipStream_t);

}  // namespace btrtk
