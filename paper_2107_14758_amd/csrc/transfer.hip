// Lattice transfers in one launch each: the FDM change of basis z = T z~ and its transpose
// r~ = T^T r (Sec. 2.4), and the Q1 coarse transfer P and P^T (Sec. 2.5).
//
// On a structured hexahedral mesh each of these maps is a Kronecker product M x M x M of
// one 1D lattice map, and the 1D map is block-structured by cell: the outputs that cell e
// owns along an axis depend on a short window of inputs that starts at a fixed offset from
// the cell.  One workgroup handles one cell: it stages the cell's input window in LDS
// (zero outside the lattice), contracts x, then y, then z, and writes its own outputs.
// Windows overlap between neighbouring cells; the overlap is read through the caches,
// each lattice value once from HBM.
#include "device_common.h"

namespace vsr {

namespace {
using namespace dev;

constexpr int XFER_THREADS = 256;
constexpr int XFER_LDS_BUDGET = 48 * 1024;

// Per axis, cell e maps inputs e*in_step + in_off + s (s < K) to outputs e*out_step + a
// (a < OA) with the OA x K row-major matrix M.  out = alpha * (M x M x M) in + beta * out.
// The z inputs are taken UC planes at a time so that the window fits the LDS budget.
template <typename Tin, typename T, int OA, int K>
__global__ void __launch_bounds__(XFER_THREADS)
    k_transfer(const double *__restrict__ gate, const T *__restrict__ M, int ncx, int ncy, int ncz, int in_step,
               int in_off, int out_step, int ix, int iy, int iz, int ox, int oy, int oz, const Tin *__restrict__ in,
               T *__restrict__ out, T alpha, T beta) {
    if (gated(gate)) return;
    constexpr int KP = K | 1;   // odd row pitch: rows read with a lane stride of KP hit distinct banks
    constexpr int PLANE = K * KP + OA * KP + OA * OA;   // LDS per input plane
    // planes per chunk: within the LDS budget and at most about 12 window loads per thread
    constexpr int UCL = XFER_LDS_BUDGET / (int)sizeof(T) / PLANE, UCR = 12 * XFER_THREADS / (K * K);
    constexpr int UCB = UCL < UCR ? UCL : UCR;
    constexpr int UC = UCB < 1 ? 1 : (UCB > K ? K : UCB);
    static_assert(OA * OA <= XFER_THREADS, "one thread per (x, y) output column");
    // M is read at wave-uniform addresses (scalar loads, SGPR operands of the FMAs); only
    // the lattice data goes through LDS
    __shared__ T I[UC * K * KP];      // [u][t][s]: input window, s along x
    __shared__ T A[UC * OA * KP];     // [u][a][t]: after the x contraction
    __shared__ T Bc[UC * OA * OA];    // [u][b][a]: after the y contraction

    // consecutive workgroups land on different XCDs: give each XCD a contiguous run of
    // cells so that the overlapping windows meet in the same L2
    const int nc = ncx * ncy * ncz, per = (nc + 7) / 8;
    const int cell = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (cell >= nc) return;
    const int ex = cell % ncx, ey = (cell / ncx) % ncy, ez = cell / (ncx * ncy);
    const int tid = threadIdx.x;
    const int x0 = ex * in_step + in_off, y0 = ey * in_step + in_off, z0 = ez * in_step + in_off;
    const int za = tid % OA, zb = tid / OA;   // z-stage owner of output column (a, b)
    T acc[OA];
#pragma unroll
    for (int c = 0; c < OA; ++c) acc[c] = T(0);

    constexpr int NW = UC * K * K, NL = (NW + XFER_THREADS - 1) / XFER_THREADS;   // window loads per thread
    for (int u0 = 0; u0 < K; u0 += UC) {
        const int uc = K - u0 < UC ? K - u0 : UC;
        // every load of the chunk in flight before the first LDS store
        T wv[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int i = tid + l * XFER_THREADS;
            const int s = i % K, t = (i / K) % K, u = i / (K * K);
            const int xi = x0 + s, yi = y0 + t, zi = z0 + u0 + u;
            wv[l] = (i < NW && u < uc && xi >= 0 && xi < ix && yi >= 0 && yi < iy && zi >= 0 && zi < iz)
                        ? (T)in[((int64_t)zi * iy + yi) * ix + xi]
                        : T(0);
        }
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int i = tid + l * XFER_THREADS;
            if (i < NW) I[(i / K) * KP + i % K] = wv[l];
        }
        __syncthreads();
        // x: A[u][a][t] = sum_s M[a][s] I[u][t][s], one input row per thread
        for (int r = tid; r < uc * K; r += XFER_THREADS) {
            const int u = r / K, t = r % K;
            T v[K];
#pragma unroll
            for (int s = 0; s < K; ++s) v[s] = I[r * KP + s];
#pragma unroll
            for (int a = 0; a < OA; ++a) {
                T sum = T(0);
#pragma unroll
                for (int s = 0; s < K; ++s) sum += M[a * K + s] * v[s];
                A[(u * OA + a) * KP + t] = sum;
            }
        }
        __syncthreads();
        // y: Bc[u][b][a] = sum_t M[b][t] A[u][a][t]
        for (int r = tid; r < uc * OA; r += XFER_THREADS) {
            const int u = r / OA, a = r % OA;
            T v[K];
#pragma unroll
            for (int t = 0; t < K; ++t) v[t] = A[r * KP + t];
#pragma unroll
            for (int b = 0; b < OA; ++b) {
                T sum = T(0);
#pragma unroll
                for (int t = 0; t < K; ++t) sum += M[b * K + t] * v[t];
                Bc[(u * OA + b) * OA + a] = sum;
            }
        }
        __syncthreads();
        // z: acc[c] += sum_u M[c][u0 + u] Bc[u][b][a]
        if (tid < OA * OA) {
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                if (u < uc) {
                    const T v = Bc[(u * OA + zb) * OA + za];
#pragma unroll
                    for (int c = 0; c < OA; ++c) acc[c] += M[c * K + u0 + u] * v;
                }
            }
        }
        __syncthreads();
    }
    if (tid < OA * OA) {
        const int xo = ex * out_step + za, yo = ey * out_step + zb;
        if (xo < ox && yo < oy) {
#pragma unroll
            for (int c = 0; c < OA; ++c) {
                const int zo = ez * out_step + c;
                if (zo < oz) {
                    const int64_t q = ((int64_t)zo * oy + yo) * ox + xo;
                    out[q] = beta == T(0) ? alpha * acc[c] : alpha * acc[c] + beta * out[q];
                }
            }
        }
    }
}

}  // namespace

template <typename Tin, typename T>
void launch_transfer(int kind, int p, const int ncell[3], const int in_dims[3], const int out_dims[3], const T *M,
                     const Tin *in, T *out, T alpha, T beta, const Exec &e) {
    const int nc = ncell[0] * ncell[1] * ncell[2];
    if (nc == 0 || (int64_t)out_dims[0] * out_dims[1] * out_dims[2] == 0) return;
    const unsigned grid = 8u * (unsigned)((nc + 7) / 8);
#define GO(OA, K, IS, IO, OS)                                                                                          \
    hipLaunchKernelGGL((k_transfer<Tin, T, OA, K>), dim3(grid), dim3(XFER_THREADS), 0, e.s, e.gate, M, ncell[0],      \
                       ncell[1], ncell[2], IS, IO, OS, in_dims[0], in_dims[1], in_dims[2], out_dims[0], out_dims[1], \
                       out_dims[2], in, out, alpha, beta)
#define CALL(P)                                                               \
    switch (kind) {                                                           \
        case XFER_FDM_RESTRICT: GO(P, 2 * P - 1, P, 0, P); break;             \
        case XFER_FDM_PROLONG: GO(P, P + 1, P, -1, P); break;                 \
        case XFER_COARSE_RESTRICT: GO(1, 2 * P - 1, P, 0, 1); break;          \
        case XFER_COARSE_PROLONG: GO(P, 2, 1, -1, P); break;                  \
        default: throw Error(VSR_EINVAL, "unknown transfer kind");            \
    }
    VSR_P_SWITCH(p, CALL)
#undef CALL
#undef GO
}

template void launch_transfer<double, double>(int, int, const int *, const int *, const int *, const double *,
                                              const double *, double *, double, double, const Exec &);
template void launch_transfer<float, float>(int, int, const int *, const int *, const int *, const float *,
                                            const float *, float *, float, float, const Exec &);
template void launch_transfer<double, float>(int, int, const int *, const int *, const int *, const float *,
                                             const double *, float *, float, float, const Exec &);

}  // namespace vsr
