// Device helpers shared by the kernel translation units (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"
#include "vsr_internal.h"

namespace vsr {
namespace dev {

constexpr int QOF(int P) { return (3 * (P + 1) + 1) / 2; }

__device__ __forceinline__ bool is_free(const Dims &d, int K, int J, int I) {
    return K >= 1 && K <= d.Lz && J >= 1 && J <= d.Ly && I >= 1 && I <= d.Lx;
}
__device__ __forceinline__ int64_t free_index(const Dims &d, int K, int J, int I) {
    return ((int64_t)(K - 1) * d.Ly + (J - 1)) * d.Lx + (I - 1);
}

// Element vectors hold (p+1)^3 values per cell laid out across cells row by row: row
// ((ez ny + ey)(p+1) + k)(p+1) + j holds the x-rows (local i) of the cells ex = 0 .. nx-1
// one after another, so the lattice nodes of one x-line read one contiguous run.  Slot s
// of a general-operator split starts at s ncell (p+1)^3.
template <int N1>
__device__ __forceinline__ int64_t elem_index(const Dims &d, int ex, int ey, int ez, int k, int j, int i) {
    return ((((int64_t)ez * d.ny + ey) * N1 + k) * N1 + j) * ((int64_t)d.nx * N1) + (int64_t)ex * N1 + i;
}

// Above degree kFusedScatterMaxP the patch solutions (star boxes of (2p-1)^3 nodes around
// each mesh vertex) are kept as 8 lattice vectors, one per vertex-parity class (vx mod 2,
// vy mod 2, vz mod 2): boxes of stars of one class do not overlap (their vertices are two
// cells apart along some axis), so a star writes its box into its class's vector, and nodes
// no star of the class covers stay zero.  The scatter-add of the boxes (Sec. 2.5) at a
// lattice node is then the sum of the 8 vectors' entries there.
__device__ __forceinline__ int64_t star_class(int vx, int vy, int vz) { return (vx & 1) + 2 * (vy & 1) + 4 * (vz & 1); }

template <typename T>
__device__ __forceinline__ T star_box_sum(const T *__restrict__ U, int64_t n, int64_t idx) {
    T v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = U[c * n + idx];
    return ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
}

template <typename T>
__device__ __forceinline__ void atomic_add_global(T *p, T v) {
    unsafeAtomicAdd(p, v);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// A kernel launched under a gate returns at once, in every workgroup and before any
// barrier, when the flag it points to is nonzero (a converged member of a batched solve).
__device__ __forceinline__ bool gated(const double *gate) { return gate != nullptr && *gate != 0.0; }

inline unsigned grid_for(int64_t n, int block = 256) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

inline unsigned round64(int n) { return (unsigned)((n + 63) / 64 * 64); }

}  // namespace dev
}  // namespace vsr

#define VSR_P_SWITCH(p, CALL)                                  \
    switch (p) {                                               \
        case 2: CALL(2); break;                                \
        case 3: CALL(3); break;                                \
        case 4: CALL(4); break;                                \
        case 5: CALL(5); break;                                \
        case 6: CALL(6); break;                                \
        case 7: CALL(7); break;                                \
        case 8: CALL(8); break;                                \
        case 9: CALL(9); break;                                \
        case 10: CALL(10); break;                              \
        case 11: CALL(11); break;                              \
        case 12: CALL(12); break;                              \
        case 13: CALL(13); break;                              \
        case 14: CALL(14); break;                              \
        case 15: CALL(15); break;                              \
        default: throw Error(VSR_EINVAL, "unsupported degree"); \
    }
