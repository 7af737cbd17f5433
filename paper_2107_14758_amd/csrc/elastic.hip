// Primal linear elasticity operator on axis-aligned cells (Sec. 3.1), FP64 or FP32.
//
// a(v, u) = int 2 mu eps(v) : eps(u) + lam div v div u.  On a box cell every block A_cd of
// the component blocks is a sum of Kronecker products of the 1-D reference matrices
// A (int phi_a' phi_b'), B (int phi_a phi_b) and C (int phi_a' phi_b, the test function
// differentiated), each taken with the q-point GLL rule of the scalar operator:
//   A_cc = sum_a k_ca (B x B x A placed with A on axis a),  k_ca = (mu + (mu + lam) [a = c]) |J| (2/h_a)^2
//   A_cd = mu s_cd (C^T on axis c, C on axis d, B on the third)
//        + lam s_cd (C on axis c, C^T on axis d, B on the third),      s_cd = |J| (2/h_c) (2/h_d)
// (from mu d_d v_c d_c u_d + lam d_c v_c d_d u_d): 21 terms per cell, 7 per output component.
//
// One workgroup per cell in three groups of whole wavefronts, group c computing output
// component c.  The input components pass through LDS one at a time; on each, every group
// runs up to three of its terms (the diagonal block's three on its own component, the
// coupling block's two on the others).  Up to p = 11 each (j, i) column of a group has two
// threads, each owning half of the z planes: a term's x and y contractions run plane by
// plane through the group's LDS slabs and its z contraction reads the y results of all
// planes back from LDS.  Above p = 11 (three groups of two threads per column would exceed
// 1,024 threads) one thread owns the column and keeps the y and z contractions in registers.
// The cell's results go to three element vectors (one per component) for the gather.
#include "device_common.h"

namespace vsr {
namespace dev {
namespace {

constexpr int MA = 0, MB = 1, MC = 2, MCT = 3;   // the 1-D matrices
constexpr int kElasticCoef = 12;                 // per cell: k[c][a] at 3 c + a (9), then s_xy, s_xz, s_yz

// Whole wavefronts covering t threads.
constexpr int el_waves(int t) { return t < 64 ? 64 : (t + 63) / 64 * 64; }
// Threads per (j, i) column: two while three groups of them fit a workgroup of 1,024.
constexpr int el_halves(int p) { return 3 * el_waves(2 * (p + 1) * (p + 1)) <= 1024 ? 2 : 1; }
// Threads of one output component's group.
constexpr int el_group(int p) { return el_waves(el_halves(p) * (p + 1) * (p + 1)); }
static_assert(3 * el_group(11) <= 1024 && el_halves(11) == 2 && el_halves(12) == 1 && 3 * el_group(15) <= 1024,
              "workgroup sizes");

// The matrix on `axis` (0 = x, 1 = y, 2 = z) of term s of block (C, D): for C == D the
// stiffness A on axis s and B elsewhere; for C != D term 0 is mu's (C^T on axis C, C on axis
// D) and term 1 lam's (C on axis C, C^T on axis D), B on the third axis.
constexpr int term_mat(int axis, int C, int D, int s) {
    if (C == D) return axis == s ? MA : MB;
    const int mc = s == 0 ? MCT : MC, md = s == 0 ? MC : MCT;
    return axis == C ? mc : (axis == D ? md : MB);
}
constexpr bool has_term(int C, int D, int s) { return C == D || s < 2; }

// Planes k0 <= k < k0 + KH (below N1) of X = (I x I x Mx) xs, for column (j, i)
template <typename T, int N1, int KH>
__device__ __forceinline__ void x_half(const T *Mx, const T *xs, T *X, int j, int i, int k0) {
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
        const int k = k0 + kk;
        if (k < N1) {
            T s = 0;
#pragma unroll
            for (int ii = 0; ii < N1; ++ii) s += Mx[i * N1 + ii] * xs[(k * N1 + j) * N1 + ii];
            X[(k * N1 + j) * N1 + i] = s;
        }
    }
}

// The same planes of Yv = (I x My x I) X
template <typename T, int N1, int KH>
__device__ __forceinline__ void y_half(const T *My, const T *X, T *Yv, int j, int i, int k0) {
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
        const int k = k0 + kk;
        if (k < N1) {
            T s = 0;
#pragma unroll
            for (int jj = 0; jj < N1; ++jj) s += My[j * N1 + jj] * X[(k * N1 + jj) * N1 + i];
            Yv[(k * N1 + j) * N1 + i] = s;
        }
    }
}

// y[kk] += w ((Mz x I x I) Yv)[k0 + kk] for column (j, i)
template <typename T, int N1, int KH>
__device__ __forceinline__ void z_half(const T *Mz, const T *Yv, int j, int i, int k0, T w, T (&y)[KH]) {
    T Yc[N1];
#pragma unroll
    for (int kk = 0; kk < N1; ++kk) Yc[kk] = Yv[(kk * N1 + j) * N1 + i];
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
        const int k = k0 + kk;
        if (k < N1) {
            T s = 0;
#pragma unroll
            for (int m = 0; m < N1; ++m) s += Mz[k * N1 + m] * Yc[m];
            y[kk] += w * s;
        }
    }
}

// X = (I x I x Mx) xs for the group's columns
template <typename T, int N1>
__device__ __forceinline__ void x_pass(const T *Mx, const T *xs, T *X, int j, int i) {
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        T s = 0;
#pragma unroll
        for (int ii = 0; ii < N1; ++ii) s += Mx[i * N1 + ii] * xs[(k * N1 + j) * N1 + ii];
        X[(k * N1 + j) * N1 + i] = s;
    }
}

// y += w (Mz x My x I) X for thread (j, i)'s z-column, in registers
template <typename T, int N1>
__device__ __forceinline__ void yz_pass(const T *My, const T *Mz, const T *X, int j, int i, T w, T (&y)[N1]) {
    T Y[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        T s = 0;
#pragma unroll
        for (int jj = 0; jj < N1; ++jj) s += My[j * N1 + jj] * X[(k * N1 + jj) * N1 + i];
        Y[k] = s;
    }
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        T s = 0;
#pragma unroll
        for (int kk = 0; kk < N1; ++kk) s += Mz[k * N1 + kk] * Y[kk];
        y[k] += w * s;
    }
}

template <typename T, int P>
__global__ void __launch_bounds__(3 * el_group(P))
    k_op_elastic_box(const double *__restrict__ gate, Dims d, const T *__restrict__ M1, const T *__restrict__ coef, T mu,
                     T lam, const T *__restrict__ x, T *__restrict__ E) {
    if (gated(gate)) return;
    constexpr int N1 = P + 1, N2 = N1 * N1, N3 = N2 * N1, NG = el_group(P), H = el_halves(P);
    constexpr int KH = (N1 + H - 1) / H;   // z planes per thread
    // A, B, C, C^T: [m][row = test][col = trial], in LDS (at p = 15 with the cell blocks 139 KB)
    __shared__ T sM[4 * N2];
    __shared__ T xs[N3];                        // the input component's cell block [k][j][i]
    __shared__ T Xs[(H == 2 ? 6 : 3) * N3];     // per group: after the x (and the y) contraction
    const int tid = threadIdx.x;
    const int g = tid / NG, lt = tid - g * NG;
    const int64_t e = blockIdx.x;
    const int ex = (int)(e % d.nx), ey = (int)((e / d.nx) % d.ny), ez = (int)(e / ((int64_t)d.nx * d.ny));
    for (int t = tid; t < 4 * N2; t += blockDim.x) sM[t] = M1[t];
    const T *cf = coef + e * kElasticCoef;
    T *X = Xs + g * N3;
    T *Yv = Xs + (3 + g) * N3;   // used only with two threads per column
    const bool col = lt < H * N2;
    const int h = lt / N2, c2 = lt - h * N2;   // half, column
    const int j = c2 / N1, i = c2 % N1, k0 = h * KH;
    const int64_t n = (int64_t)d.Lx * d.Ly * d.Lz;
    T y[KH];
#pragma unroll
    for (int k = 0; k < KH; ++k) y[k] = T(0);
    // Input component D: load it, then terms 0 and 1 of every group and term 2 of group D.
    // Barriers: after the load (xs ready), after each contraction pass (its slab ready), and
    // after the last pass of a term (the slabs free again); the last term of a component also
    // frees xs for the next load.  The loops stay rolled: one copy of the contractions, their
    // registers allocated once.
#pragma unroll 1
    for (int D = 0; D < 3; ++D) {
        for (int t = tid; t < N3; t += blockDim.x) {
            const int kk = t / N2, jj = (t / N1) % N1, ii = t % N1;
            const int K = P * ez + kk, J = P * ey + jj, I = P * ex + ii;
            xs[t] = is_free(d, K, J, I) ? x[D * n + free_index(d, K, J, I)] : T(0);
        }
        __syncthreads();
#pragma unroll 1
        for (int S = 0; S < 3; ++S) {
            // group g's term S on component D (g is uniform per wavefront)
            const bool active = col && has_term(g, D, S);
            const T *Mx = sM + term_mat(0, g, D, S) * N2, *My = sM + term_mat(1, g, D, S) * N2,
                    *Mz = sM + term_mat(2, g, D, S) * N2;
            const T w = g == D ? cf[3 * D + S] : (S == 0 ? mu : lam) * cf[9 + g + D - 1];   // s_xy, s_xz, s_yz at 9..11
            if constexpr (H == 2) {
                if (active) x_half<T, N1, KH>(Mx, xs, X, j, i, k0);
                __syncthreads();
                if (active) y_half<T, N1, KH>(My, X, Yv, j, i, k0);
                __syncthreads();
                if (active) z_half<T, N1, KH>(Mz, Yv, j, i, k0, w, y);
                __syncthreads();
            } else {
                if (active) x_pass<T, N1>(Mx, xs, X, j, i);
                __syncthreads();
                if (active) yz_pass<T, N1>(My, Mz, X, j, i, w, y);
                __syncthreads();
            }
        }
    }
    if (col) {
        const int64_t slot = (int64_t)d.nx * d.ny * d.nz * N3;
#pragma unroll
        for (int kk = 0; kk < KH; ++kk)
            if (k0 + kk < N1) E[g * slot + elem_index<N1>(d, ex, ey, ez, k0 + kk, j, i)] = y[kk];
    }
}

}  // namespace
}  // namespace dev

using namespace dev;

template <typename T>
void launch_op_elastic_box(const Dims &d, const T *M1, const T *coef, T mu, T lam, const T *x, T *E, const Exec &e) {
    const int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
#define CALL(P)                                                                                                   \
    hipLaunchKernelGGL((k_op_elastic_box<T, P>), dim3((unsigned)ncell), dim3(3 * el_group(P)), 0, e.s, e.gate, d, M1,  \
                       coef, mu, lam, x, E)
    VSR_P_SWITCH(d.p, CALL)
#undef CALL
}

template void launch_op_elastic_box<double>(const Dims &, const double *, const double *, double, double, const double *,
                                            double *, const Exec &);
template void launch_op_elastic_box<float>(const Dims &, const float *, const float *, float, float, const float *,
                                           float *, const Exec &);

}  // namespace vsr
