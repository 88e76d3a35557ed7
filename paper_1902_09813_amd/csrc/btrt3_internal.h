// Internal interface between the host runtime of the D3Q19 solver (btrt3_api.cpp) and its
// gfx950 kernels (btrt3_kernels.hip). Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace btrt3k {

constexpr int kQ = 19;

// Everything one D3Q19 sweep needs, by value in the kernel argument segment.
template <typename T>
struct Sweep3 {
    const T* fin;       // 19 planes of f+(t-1); plane stride `plane`
    T* fout;            // 19 planes receiving f+(t)
    const T* phi_prev;  // phi(t-1)
    T* phi_out;         // phi(t)
    const T* src;       // source plane (null: none)
    int64_t plane;      // elements per plane: pitch * ny * nz
    int nx, ny, nz, pitch;
    int slab;           // pitch * ny
    int per[3];         // 1 when the axis is periodic
    T wall[6];          // phi_w of faces x-, x+, y-, y+, z-, z+
    T a[3], b[3];       // B(phi) = a phi + b phi^2 / 2
    T A0[6];            // (a11, a12, a13, a22, a23, a33) of A0, per-node K1 when beta > 0
    T beta;
    T K1[6];            // constant K1 (symmetric) in the same order
    T k0;
    T cq[6];            // the collision's constants 3/2, -9/2, 3, -3, 9, -9 (from the arguments the
                        // kernels keep them in scalar registers, so a multiply-add needs no copy of
                        // its accumulator)
    T q2[6];            // K2 rates (k2_11, k2_12s, k2_13s, k2_22, k2_23s, k2_33), off-diagonals
                        // symmetrised (Eq. (100))
    int tiles_x, tiles_y;
    int nts;            // 1: the one-step kernel stores non-temporally (the launcher picks it)
    int zc;             // two-step kernel: output planes per workgroup
};

// Gather-reduce arguments: the sweep arguments of the current state plus the buffers.
template <typename T>
struct Gather3 {
    Sweep3<T> s;
    double* snap;       // residual: FP64 phi snapshot (dense), updated in place
    const double* ref;  // error: reference (dense)
    double* out;        // dense output of field and population reads
    double* partial;    // per-block partial sums
    int population;     // -1: phi
};

constexpr int kPartials = 6;
constexpr int kReduceBlocks3 = 1024;

template <typename T>
hipError_t launch3_sweep(const Sweep3<T>& a, bool src, bool k1_per_node, hipStream_t s);
// Two time steps in one launch (f+(t-1), phi(t-1) -> f+(t+1), phi(t+1)); the same bits as two
// launch3_sweep calls. tile 1: 64 x 8 threads per workgroup, 2: 32 x 16, 3: 32 x 8, 4: 16 x 16;
// zc output planes per workgroup (>= 1).
constexpr int kTiles2 = 5;  // tile values 0 (automatic) .. 4
template <typename T>
hipError_t launch3_sweep2(const Sweep3<T>& a, bool src, bool k1_per_node, int tile, int zc, hipStream_t s);
// Workgroups of a two-step launch for the grid (tile shape and z chunk as above).
int64_t sweep2_workgroups(int nx, int ny, int nz, int tile, int zc);
// Workgroups of the two-step kernel that one compute unit holds at once (its LDS and registers),
// for the variant a launch with these arguments takes; 1 if the runtime cannot tell.
template <typename T>
int sweep2_blocks_per_cu(bool walls, bool src, bool k1_per_node, int tile);
// f+(-1) and phi(-1) := phi0 (FP64 values converted to T) into a.fout / a.phi_out.
template <typename T>
hipError_t launch3_init(const Sweep3<T>& a, const double* phi0, hipStream_t s);
template <typename T>
hipError_t launch3_gather(const Gather3<T>& a, hipStream_t s);
// mode 0: residual (Eq. (64)); 1: error norms against ref (Eq. (63)); result: kPartials doubles.
template <typename T>
hipError_t launch3_reduce(const Gather3<T>& a, int mode, double* result, hipStream_t s);
template <typename T>
hipError_t launch3_convert(const double* in, T* out, int nx, int ny, int nz, int pitch, hipStream_t s);

}  // namespace btrt3k
