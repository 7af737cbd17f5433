// Lattice transfers in one launch each: the FDM change of basis z = T z~ and its transpose
// r~ = T^T r (Sec. 2.4), and the Q1 coarse transfer P and P^T (Sec. 2.5).
//
// On a structured hexahedral mesh each of these maps is a Kronecker product M x M x M of
// one 1D lattice map, and the 1D map is block-structured by cell: the outputs that cell e
// owns along an axis depend on a short window of inputs that starts at a fixed offset from
// the cell.  One workgroup handles one cell: it stages the cell's input window in LDS
// (zero outside the lattice), contracts x, then y, then z, and writes its own outputs;
// for three of the four maps small cells are taken 2 x 2 (or 2 x 1) at a time to share
// their windows.
// Windows overlap between neighbouring cells; the overlap is read through the caches,
// each lattice value once from HBM.
#include "device_common.h"

namespace vsr {

namespace {
using namespace dev;

constexpr int XFER_THREADS = 256;
constexpr int XFER_LDS_BUDGET = 48 * 1024;

// Sum over the workgroup, valid in thread 0 (fixed order: waves by index).
__device__ __forceinline__ double xfer_block_sum(double v) {
    __shared__ double part[XFER_THREADS / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) part[wv] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < XFER_THREADS / 64; ++i) s += part[i];
    return s;
}

// Value of the assembled star boxes (sum over the stars whose boxes hold it, Sec. 2.5) at free
// lattice node (I, J, K), 1-based, with the boxes stored per mesh vertex ((2p-1)^3 each, x
// fastest; the layout up to degree kFusedScatterMaxP): the patch scatter-add evaluated where
// the prolongation needs it; interior_only drops the stars of boundary vertices.  Every
// candidate load is issued before the fixed-order sum.
template <typename T, int P>
__device__ __forceinline__ T star_box_gather(const T *__restrict__ U, int nx, int ny, int nz, int interior_only, int I, int J,
                                          int K) {
    constexpr int m = P - 1, w = 2 * m + 1, w3 = w * w * w;
    const int P3[3] = {I, J, K}, ncell[3] = {nx, ny, nz};
    int v[3][2], a[3][2], nc[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int Pp = P3[ax], e = Pp / P, al = Pp - e * P;
        if (al == 0) {
            v[ax][0] = e; a[ax][0] = m; v[ax][1] = e; a[ax][1] = m; nc[ax] = 1;
        } else {
            v[ax][0] = e; a[ax][0] = m + al; v[ax][1] = e + 1; a[ax][1] = al - 1; nc[ax] = 2;
        }
        if (interior_only) {
            int k = 0;
            for (int t = 0; t < nc[ax]; ++t)
                if (v[ax][t] >= 1 && v[ax][t] <= ncell[ax] - 1) { v[ax][k] = v[ax][t]; a[ax][k] = a[ax][t]; ++k; }
            nc[ax] = k;
        }
    }
    T val[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int tz = t >> 2, ty = (t >> 1) & 1, tx = t & 1;
        const bool ok = tz < nc[2] && ty < nc[1] && tx < nc[0];
        const int64_t vid = ((int64_t)v[2][tz] * (ny + 1) + v[1][ty]) * (nx + 1) + v[0][tx];
        val[t] = ok ? U[vid * w3 + (a[2][tz] * w + a[1][ty]) * w + a[0][tx]] : T(0);
    }
    T sum = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) sum += val[t];
    return sum;
}

// Per axis, cell e maps inputs e*IS + in_off + s (s < K) to outputs e*out_step + a (a < OA)
// with the OA x K row-major matrix M.  out = alpha * (M x M x M) in + beta * out.
// A workgroup takes a brick of CX x CY x 1 cells: their windows along x and y overlap and
// are staged once (KX = K + (CX-1) IS by KY = K + (CY-1) IS values per z-plane).  The z
// inputs are taken UC planes at a time so that the window fits the LDS budget.
// BOXES (the FDM prolongation up to degree kFusedScatterMaxP): in holds the star boxes of the
// patch solves, and the window is their assembled sum (star_box_gather; box_mode 2 = interior
// stars only) instead of a lattice vector, so the scatter-add needs no pass of its own.
template <typename Tin, typename T, int OA, int K, int IS, int CX, int CY, bool BOXES = false>
__global__ void __launch_bounds__(XFER_THREADS)
    k_transfer(const double *__restrict__ gate, const T *__restrict__ M, int ncx, int ncy, int ncz, int in_off,
               int out_step, int ix, int iy, int iz, int ox, int oy, int oz, const Tin *__restrict__ in,
               T *__restrict__ out, T alpha, T beta, double *__restrict__ out64, const double *__restrict__ dotv,
               double *__restrict__ partials, int box_mode, int64_t in_cstride) {
    if (gated(gate)) return;
    if (gridDim.y > 1) {   // independent components (no dot): blockIdx.y selects one
        in += blockIdx.y * in_cstride;
        out += blockIdx.y * (int64_t)ox * oy * oz;
        if (out64 != nullptr) out64 += blockIdx.y * (int64_t)ox * oy * oz;
    }
    constexpr int KX = K + (CX - 1) * IS, KY = K + (CY - 1) * IS;   // window extents along x and y
    constexpr int AX = CX * OA, AY = CY * OA;                       // outputs along x and y
    constexpr int KXP = KX | 1, KYP = KY | 1;   // odd row pitches: strided LDS reads hit distinct banks
    constexpr int PLANE = KY * KXP + AX * KYP + AY * AX;   // LDS per input plane
    // planes per chunk: within the LDS budget and at most about 12 window loads per thread
    constexpr int UCL = XFER_LDS_BUDGET / (int)sizeof(T) / PLANE, UCR = 12 * XFER_THREADS / (KX * KY);
    constexpr int UCB = UCL < UCR ? UCL : UCR;
    constexpr int UC = UCB < 1 ? 1 : (UCB > K ? K : UCB);
    static_assert(AX * AY <= XFER_THREADS, "one thread per (x, y) output column");
    // M is read at wave-uniform addresses (scalar loads, SGPR operands of the FMAs); only
    // the lattice data goes through LDS
    __shared__ T I[UC * KY * KXP];    // [u][t][s]: input window, s along x
    __shared__ T A[UC * AX * KYP];    // [u][a][t]: after the x contraction
    __shared__ T Bc[UC * AY * AX];    // [u][b][a]: after the y contraction

    // consecutive workgroups land on different XCDs: give each XCD a contiguous run of
    // bricks so that the overlapping windows meet in the same L2
    const int nbx = (ncx + CX - 1) / CX, nby = (ncy + CY - 1) / CY, nb = nbx * nby * ncz, per = (nb + 7) / 8;
    const int brick = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (brick >= nb) {
        if (partials != nullptr && threadIdx.x == 0) partials[blockIdx.x] = 0.0;
        return;
    }
    const int bx = brick % nbx, by = (brick / nbx) % nby, ez = brick / (nbx * nby);
    const int tid = threadIdx.x;
    const int x0 = bx * CX * IS + in_off, y0 = by * CY * IS + in_off, z0 = ez * IS + in_off;
    const int za = tid % AX, zb = tid / AX;   // z-stage owner of output column (a, b) of the brick
    T acc[OA];
#pragma unroll
    for (int c = 0; c < OA; ++c) acc[c] = T(0);

    constexpr int NW = UC * KY * KX, NL = (NW + XFER_THREADS - 1) / XFER_THREADS;   // window loads per thread
    for (int u0 = 0; u0 < K; u0 += UC) {
        const int uc = K - u0 < UC ? K - u0 : UC;
        // every load of the chunk in flight before the first LDS store
        T wv[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int i = tid + l * XFER_THREADS;
            const int s = i % KX, t = (i / KX) % KY, u = i / (KX * KY);
            const int xi = x0 + s, yi = y0 + t, zi = z0 + u0 + u;
            const bool inside = i < NW && u < uc && xi >= 0 && xi < ix && yi >= 0 && yi < iy && zi >= 0 && zi < iz;
            if constexpr (BOXES)
                wv[l] = inside ? star_box_gather<T, OA>((const T *)in, ncx, ncy, ncz, box_mode == 2, xi + 1, yi + 1, zi + 1)
                               : T(0);
            else
                wv[l] = inside ? (T)in[((int64_t)zi * iy + yi) * ix + xi] : T(0);
        }
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int i = tid + l * XFER_THREADS;
            if (i < NW) I[(i / KX) * KXP + i % KX] = wv[l];
        }
        __syncthreads();
        // x: A[u][c OA + a][t] = sum_s M[a][s] I[u][t][c IS + s], one input row per thread
        for (int r = tid; r < uc * KY; r += XFER_THREADS) {
            const int u = r / KY, t = r % KY;
            T v[KX];
#pragma unroll
            for (int s = 0; s < KX; ++s) v[s] = I[r * KXP + s];
#pragma unroll
            for (int c = 0; c < CX; ++c)
#pragma unroll
                for (int a = 0; a < OA; ++a) {
                    T sum = T(0);
#pragma unroll
                    for (int s = 0; s < K; ++s) sum += M[a * K + s] * v[c * IS + s];
                    A[(u * AX + c * OA + a) * KYP + t] = sum;
                }
        }
        __syncthreads();
        // y: Bc[u][d OA + b][a] = sum_t M[b][t] A[u][a][d IS + t]
        for (int r = tid; r < uc * AX; r += XFER_THREADS) {
            const int u = r / AX, a = r % AX;
            T v[KY];
#pragma unroll
            for (int t = 0; t < KY; ++t) v[t] = A[r * KYP + t];
#pragma unroll
            for (int d = 0; d < CY; ++d)
#pragma unroll
                for (int b = 0; b < OA; ++b) {
                    T sum = T(0);
#pragma unroll
                    for (int t = 0; t < K; ++t) sum += M[b * K + t] * v[d * IS + t];
                    Bc[(u * AY + d * OA + b) * AX + a] = sum;
                }
        }
        __syncthreads();
        // z: acc[c] += sum_u M[c][u0 + u] Bc[u][b][a]
        if (tid < AX * AY) {
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                if (u < uc) {
                    const T v = Bc[(u * AY + zb) * AX + za];
#pragma unroll
                    for (int c = 0; c < OA; ++c) acc[c] += M[c * K + u0 + u] * v;
                }
            }
        }
        __syncthreads();
    }
    double prod = 0.0;
    if (tid < AX * AY) {
        const int xo = (bx * CX + za / OA) * out_step + za % OA, yo = (by * CY + zb / OA) * out_step + zb % OA;
        if (xo < ox && yo < oy) {
#pragma unroll
            for (int c = 0; c < OA; ++c) {
                const int zo = ez * out_step + c;
                if (zo < oz) {
                    const int64_t q = ((int64_t)zo * oy + yo) * ox + xo;
                    const T v = beta == T(0) ? alpha * acc[c] : alpha * acc[c] + beta * out[q];
                    out[q] = v;
                    if (out64 != nullptr) {
                        out64[q] = (double)v;
                        if (dotv != nullptr) prod += dotv[q] * (double)v;
                    }
                }
            }
        }
    }
    if (partials != nullptr) {
        prod = xfer_block_sum(prod);
        if (tid == 0) partials[blockIdx.x] = prod;
    }
}

// Cells per brick along x and y: two each while the brick's output columns fit the
// workgroup, except for the FDM restriction (its 2p-1 window per cell makes a brick's
// x stage register-heavy: 2 x 2 bricks measured 24 us against 17 us for single cells at
// 16^3 Q7, while the other three transfers gained 10-30%).
constexpr int brick_x(int kind, int OA) { return kind != XFER_FDM_RESTRICT && 2 * OA * OA <= XFER_THREADS ? 2 : 1; }
constexpr int brick_y(int kind, int OA) { return kind != XFER_FDM_RESTRICT && 4 * OA * OA <= XFER_THREADS ? 2 : 1; }

}  // namespace

int transfer_blocks(int kind, int p, const int ncell[3]) {
    const int OA = kind == XFER_COARSE_RESTRICT ? 1 : p, CX = brick_x(kind, OA), CY = brick_y(kind, OA);
    const int nb = ((ncell[0] + CX - 1) / CX) * ((ncell[1] + CY - 1) / CY) * ncell[2];
    return 8 * ((nb + 7) / 8);
}

template <typename Tin, typename T>
void launch_transfer(int kind, int p, const int ncell[3], const int in_dims[3], const int out_dims[3], const T *M,
                     const Tin *in, T *out, T alpha, T beta, const Exec &e, double *out64, const double *dotv,
                     double *partials, int box_mode, int ncomp) {
    if (ncomp < 1 || (ncomp > 1 && (dotv != nullptr || partials != nullptr)))
        throw Error(VSR_EINVAL, "transfer components: no dot");
    const int nc = ncell[0] * ncell[1] * ncell[2];
    // the input of one component: a lattice vector, or the star boxes of its patch solves
    // ((nx+1)(ny+1)(nz+1) boxes of (2p-1)^3 values)
    const int64_t wb = 2 * p - 1;
    const int64_t in_cstride = box_mode != 0 ? (int64_t)(ncell[0] + 1) * (ncell[1] + 1) * (ncell[2] + 1) * wb * wb * wb
                                             : (int64_t)in_dims[0] * in_dims[1] * in_dims[2];
    if (nc == 0 || (int64_t)out_dims[0] * out_dims[1] * out_dims[2] == 0) {
        const int nb = transfer_blocks(kind, p, ncell);
        if (partials != nullptr && nb > 0) launch_fill<double>(nb, partials, 0.0, e);
        return;
    }
#define GO(KIND, OA, K, IS, IO, OS)                                                                                    \
    {                                                                                                                  \
        constexpr int CX = brick_x(KIND, OA), CY = brick_y(KIND, OA);                                                  \
        const int nb = ((ncell[0] + CX - 1) / CX) * ((ncell[1] + CY - 1) / CY) * ncell[2];                            \
        if (box_mode != 0) {                                                                                           \
            if constexpr (KIND == XFER_FDM_PROLONG && std::is_same<Tin, T>::value)                                     \
                hipLaunchKernelGGL((k_transfer<Tin, T, OA, K, IS, CX, CY, true>),                                      \
                                   dim3(8u * (unsigned)((nb + 7) / 8), (unsigned)ncomp), dim3(XFER_THREADS), 0, e.s,   \
                                   e.gate, M, ncell[0], ncell[1], ncell[2], IO, OS, in_dims[0], in_dims[1], in_dims[2], \
                                   out_dims[0], out_dims[1], out_dims[2], in, out, alpha, beta, out64, dotv, partials, \
                                   box_mode, in_cstride);                                                              \
            else throw Error(VSR_EINVAL, "star-box input is for the FDM prolongation only");                           \
        } else {                                                                                                       \
            hipLaunchKernelGGL((k_transfer<Tin, T, OA, K, IS, CX, CY>), dim3(8u * (unsigned)((nb + 7) / 8), (unsigned)ncomp), \
                               dim3(XFER_THREADS), 0, e.s, e.gate, M, ncell[0], ncell[1], ncell[2], IO, OS, in_dims[0], \
                               in_dims[1], in_dims[2], out_dims[0], out_dims[1], out_dims[2], in, out, alpha, beta,   \
                               out64, dotv, partials, 0, in_cstride);                                                 \
        }                                                                                                              \
    }
#define CALL(P)                                                               \
    switch (kind) {                                                           \
        case XFER_FDM_RESTRICT: GO(XFER_FDM_RESTRICT, P, 2 * P - 1, P, 0, P); break;       \
        case XFER_FDM_PROLONG: GO(XFER_FDM_PROLONG, P, P + 1, P, -1, P); break;            \
        case XFER_COARSE_RESTRICT: GO(XFER_COARSE_RESTRICT, 1, 2 * P - 1, P, 0, 1); break; \
        case XFER_COARSE_PROLONG: GO(XFER_COARSE_PROLONG, P, 2, 1, -1, P); break;          \
        default: throw Error(VSR_EINVAL, "unknown transfer kind");            \
    }
    VSR_P_SWITCH(p, CALL)
#undef CALL
#undef GO
}

template void launch_transfer<double, double>(int, int, const int *, const int *, const int *, const double *,
                                              const double *, double *, double, double, const Exec &, double *,
                                              const double *, double *, int, int);
template void launch_transfer<float, float>(int, int, const int *, const int *, const int *, const float *,
                                            const float *, float *, float, float, const Exec &, double *,
                                            const double *, double *, int, int);
template void launch_transfer<double, float>(int, int, const int *, const int *, const int *, const float *,
                                             const double *, float *, float, float, const Exec &, double *,
                                             const double *, double *, int, int);

}  // namespace vsr
