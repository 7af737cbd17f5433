// Primal linear elasticity operator on axis-aligned cells (Sec. 3.1), FP64.
//
// a(v, u) = int 2 mu eps(v) : eps(u) + lam div v div u.  On a box cell every block A_cd of
// the component blocks is a sum of Kronecker products of the 1-D reference matrices
// A (int phi_a' phi_b'), B (int phi_a phi_b) and C (int phi_a' phi_b, the test function
// differentiated), each taken with the q-point GLL rule of the scalar operator:
//   A_cc = sum_a k_ca (B x B x A placed with A on axis a),  k_ca = (mu + (mu + lam) [a = c]) |J| (2/h_a)^2
//   A_cd = mu s_cd (C^T on axis c, C on axis d, B on the third)
//        + lam s_cd (C on axis c, C^T on axis d, B on the third),      s_cd = |J| (2/h_c) (2/h_d)
// (from mu d_d v_c d_c u_d + lam d_c v_c d_d u_d).  One workgroup per cell, thread (j, i) one
// z-column; each of the 21 terms runs its x contraction through LDS and its y and z
// contractions in the thread's registers, accumulating the three output components there.  The cell's results go
// to three element vectors (one per component) for k_gather.
#include "device_common.h"

namespace vsr {
namespace dev {
namespace {

constexpr int MA = 0, MB = 1, MC = 2, MCT = 3;   // the 1-D matrices

// per-cell coefficients: k[c][a] at 3 c + a (9), then s_xy, s_xz, s_yz
constexpr int kElasticCoef = 12;

// The matrix on `axis` of the term of block (C, D) that puts mc on axis C and md on axis D
// (the mass matrix on the third axis).
constexpr int mat_on(int axis, int C, int D, int mc, int md) { return axis == C ? mc : (axis == D ? md : MB); }

// y[C] += w (Mz x My x Mx) xs for thread (j, i)'s z-column: the x contraction through LDS X
// (two barriers), y and z in registers.
template <int N1, int C, int MZ, int MY, int MX>
__device__ __forceinline__ void term(const double *sM, const double *xs, double *X, bool col, int j, int i, double w,
                                     double (&y)[3][N1]) {
    constexpr int N2 = N1 * N1;
    __syncthreads();   // X is free
    if (col) {
        const double *Mx = sM + MX * N2;
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            double s = 0;
#pragma unroll
            for (int ii = 0; ii < N1; ++ii) s += Mx[i * N1 + ii] * xs[(k * N1 + j) * N1 + ii];
            X[(k * N1 + j) * N1 + i] = s;
        }
    }
    __syncthreads();
    if (col) {
        const double *My = sM + MY * N2, *Mz = sM + MZ * N2;
        double Y[N1];
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            double s = 0;
#pragma unroll
            for (int jj = 0; jj < N1; ++jj) s += My[j * N1 + jj] * X[(k * N1 + jj) * N1 + i];
            Y[k] = s;
        }
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            double s = 0;
#pragma unroll
            for (int kk = 0; kk < N1; ++kk) s += Mz[k * N1 + kk] * Y[kk];
            y[C][k] += w * s;
        }
    }
}

// the two terms of block (C, D), C != D: mu (C^T on axis C, C on axis D), lam (C on axis C,
// C^T on axis D)
template <int N1, int C, int D>
__device__ __forceinline__ void coupling(const double *sM, const double *xs, double *X, bool col, int j, int i, double mu,
                                         double lam, double s, double (&y)[3][N1]) {
    term<N1, C, mat_on(2, C, D, MCT, MC), mat_on(1, C, D, MCT, MC), mat_on(0, C, D, MCT, MC)>(sM, xs, X, col, j, i, mu * s, y);
    term<N1, C, mat_on(2, C, D, MC, MCT), mat_on(1, C, D, MC, MCT), mat_on(0, C, D, MC, MCT)>(sM, xs, X, col, j, i, lam * s, y);
}

template <int P>
__global__ void __launch_bounds__((P + 1) * (P + 1) < 64 ? 64 : (P + 1) * (P + 1))
    k_op_elastic_box(const double *__restrict__ gate, Dims d, const double *__restrict__ M1, const double *__restrict__ coef,
                     double mu, double lam, const double *__restrict__ x, double *__restrict__ E) {
    if (gated(gate)) return;
    constexpr int N1 = P + 1, N2 = N1 * N1, N3 = N2 * N1;
    // A, B, C, C^T: [m][row = test][col = trial], in LDS while the cell blocks leave room
    constexpr bool MLDS = (4 * N2 + 2 * N3) * 8 <= 64 * 1024;
    __shared__ double sMl[MLDS ? 4 * N2 : 1];
    __shared__ double xs[N3];          // the input component's cell block [k][j][i]
    __shared__ double X[N3];           // after the x contraction
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    const int ex = (int)(e % d.nx), ey = (int)((e / d.nx) % d.ny), ez = (int)(e / ((int64_t)d.nx * d.ny));
    if constexpr (MLDS)
        for (int t = tid; t < 4 * N2; t += blockDim.x) sMl[t] = M1[t];
    const double *sM = MLDS ? (const double *)sMl : M1;
    const double *cf = coef + e * kElasticCoef;
    const bool col = tid < N2;
    const int j = tid / N1, i = tid % N1;
    const int64_t n = (int64_t)d.Lx * d.Ly * d.Lz;
    const double sxy = cf[9], sxz = cf[10], syz = cf[11];
    double y[3][N1];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < N1; ++k) y[c][k] = 0.0;
    auto load = [&](int dcomp) {
        __syncthreads();   // xs is free
        for (int t = tid; t < N3; t += blockDim.x) {
            const int kk = t / N2, jj = (t / N1) % N1, ii = t % N1;
            const int K = P * ez + kk, J = P * ey + jj, I = P * ex + ii;
            xs[t] = is_free(d, K, J, I) ? x[dcomp * n + free_index(d, K, J, I)] : 0.0;
        }
    };
    // input component 0: A_00 (stiffness on one axis, mass on the others), then A_10, A_20
    load(0);
    term<N1, 0, MB, MB, MA>(sM, xs, X, col, j, i, cf[0], y);
    term<N1, 0, MB, MA, MB>(sM, xs, X, col, j, i, cf[1], y);
    term<N1, 0, MA, MB, MB>(sM, xs, X, col, j, i, cf[2], y);
    coupling<N1, 1, 0>(sM, xs, X, col, j, i, mu, lam, sxy, y);
    coupling<N1, 2, 0>(sM, xs, X, col, j, i, mu, lam, sxz, y);
    load(1);
    term<N1, 1, MB, MB, MA>(sM, xs, X, col, j, i, cf[3], y);
    term<N1, 1, MB, MA, MB>(sM, xs, X, col, j, i, cf[4], y);
    term<N1, 1, MA, MB, MB>(sM, xs, X, col, j, i, cf[5], y);
    coupling<N1, 0, 1>(sM, xs, X, col, j, i, mu, lam, sxy, y);
    coupling<N1, 2, 1>(sM, xs, X, col, j, i, mu, lam, syz, y);
    load(2);
    term<N1, 2, MB, MB, MA>(sM, xs, X, col, j, i, cf[6], y);
    term<N1, 2, MB, MA, MB>(sM, xs, X, col, j, i, cf[7], y);
    term<N1, 2, MA, MB, MB>(sM, xs, X, col, j, i, cf[8], y);
    coupling<N1, 0, 2>(sM, xs, X, col, j, i, mu, lam, sxz, y);
    coupling<N1, 1, 2>(sM, xs, X, col, j, i, mu, lam, syz, y);
    if (col) {
        const int64_t slot = (int64_t)d.nx * d.ny * d.nz * N3;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < N1; ++k) E[c * slot + elem_index<N1>(d, ex, ey, ez, k, j, i)] = y[c][k];
    }
}

}  // namespace
}  // namespace dev

using namespace dev;

void launch_op_elastic_box(const Dims &d, const double *M1, const double *coef, double mu, double lam, const double *x,
                           double *E, const Exec &e) {
    const int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
#define CALL(P)                                                                                                   \
    hipLaunchKernelGGL((k_op_elastic_box<P>), dim3((unsigned)ncell), dim3((P + 1) * (P + 1) < 64 ? 64 : (P + 1) * (P + 1)), \
                       0, e.s, e.gate, d, M1, coef, mu, lam, x, E)
    VSR_P_SWITCH(d.p, CALL)
#undef CALL
}

}  // namespace vsr
