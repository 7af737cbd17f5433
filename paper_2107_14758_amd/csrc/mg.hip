// Geometric multigrid V(1,1) cycle for the p-coarse (Q1) problem (Sec. 2.8): damped
// point-Jacobi relaxation on every level, 27-point Galerkin stencils, trilinear index-space
// transfers between levels, dense inverse on the coarsest level.  gfx950, wave64.
//
// Levels too large for one workgroup take four launches each (pre-smoothing fused with the
// residual, restriction, prolongation-correction, post-smoothing), one thread per vertex with
// the stencil's 27 coefficients read coalesced ([s][vertex] storage).  All levels from the
// first one with at most kMGTailVertices vertices down to the coarsest run in a single
// workgroup of 1024 threads in one launch (barriers between the steps; the level vectors stay
// in L2), which at the 16^3 workloads is the whole cycle.
#include "device_common.h"

namespace vsr {

namespace {
using namespace dev;

constexpr int kMGTailThreads = 1024;
constexpr int kMGStepThreads = 256;

template <typename T>
struct MGLevelView {
    int ux, uy, uz;   // interior vertices per axis (cells - 1)
    int64_t nv;
    const T *st, *dinv;
    T *x, *b, *r, *t;
};

template <typename T>
__device__ __forceinline__ MGLevelView<T> view(const MGLevel<T> &L) {
    return MGLevelView<T>{L.cx - 1, L.cy - 1, L.cz - 1, (int64_t)(L.cx - 1) * (L.cy - 1) * (L.cz - 1),
                          L.st, L.dinv, L.x, L.b, L.r, L.t};
}

// sum_s st[s][i] v[j(s)] over the interior neighbours j(s) of vertex i = (X, Y, Z)
template <typename T, typename F>
__device__ __forceinline__ T stencil_apply(const MGLevelView<T> &L, int64_t i, int X, int Y, int Z, F v) {
    T acc = 0;
#pragma unroll
    for (int s = 0; s < 27; ++s) {
        const int jx = X + s % 3 - 1, jy = Y + (s / 3) % 3 - 1, jz = Z + s / 9 - 1;
        if (jx < 0 || jx >= L.ux || jy < 0 || jy >= L.uy || jz < 0 || jz >= L.uz) continue;
        acc += L.st[(int64_t)s * L.nv + i] * v(jx + (int64_t)L.ux * (jy + (int64_t)L.uy * jz));
    }
    return acc;
}

template <typename T>
__device__ __forceinline__ void coords(const MGLevelView<T> &L, int64_t i, int &X, int &Y, int &Z) {
    X = (int)(i % L.ux);
    Y = (int)((i / L.ux) % L.uy);
    Z = (int)(i / ((int64_t)L.ux * L.uy));
}

// x = w D^{-1} b (one Jacobi step from zero) and r = b - A x
template <typename T>
__device__ __forceinline__ void presmooth_residual(const MGLevelView<T> &L, T w, int64_t i) {
    int X, Y, Z;
    coords(L, i, X, Y, Z);
    L.x[i] = w * L.dinv[i] * L.b[i];
    const T Ax = stencil_apply(L, i, X, Y, Z, [&](int64_t j) { return w * L.dinv[j] * L.b[j]; });
    L.r[i] = L.b[i] - Ax;
}

// b_c[I] = (P^T r_f)[I]: the 27 fine vertices 2I + d (1-based) with weights 2^-(nonzero d)
template <typename T>
__device__ __forceinline__ void restrict_vertex(const MGLevelView<T> &F, const MGLevelView<T> &C, int64_t I) {
    int X, Y, Z;
    coords(C, I, X, Y, Z);
    T acc = 0;
#pragma unroll
    for (int s = 0; s < 27; ++s) {
        const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
        const T wgt = T((dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0));
        const int fx = 2 * X + 1 + dx, fy = 2 * Y + 1 + dy, fz = 2 * Z + 1 + dz;   // 0-based fine
        acc += wgt * F.r[fx + (int64_t)F.ux * (fy + (int64_t)F.uy * fz)];
    }
    C.b[I] = acc;
}

// 1D parents of fine interior vertex f (0-based): coarse 0-based indices and weights
__device__ __forceinline__ int parents(int f, int uc, int J[2], double w[2]) {
    const int fi = f + 1;   // 1-based
    int n = 0;
    if (fi % 2 == 0) {
        J[0] = fi / 2 - 1; w[0] = 1.0; n = 1;
    } else {
        const int a = (fi - 1) / 2, b = (fi + 1) / 2;   // 1-based coarse
        if (a >= 1 && a <= uc) { J[n] = a - 1; w[n] = 0.5; ++n; }
        if (b >= 1 && b <= uc) { J[n] = b - 1; w[n] = 0.5; ++n; }
    }
    return n;
}

// t_f = x_f + P x_c
template <typename T>
__device__ __forceinline__ void prolong_vertex(const MGLevelView<T> &F, const MGLevelView<T> &C, int64_t i) {
    int X, Y, Z;
    coords(F, i, X, Y, Z);
    int Jx[2], Jy[2], Jz[2];
    double wx[2], wy[2], wz[2];
    const int nx = parents(X, C.ux, Jx, wx), ny = parents(Y, C.uy, Jy, wy), nz = parents(Z, C.uz, Jz, wz);
    T acc = F.x[i];
    for (int c = 0; c < nz; ++c)
        for (int b = 0; b < ny; ++b)
            for (int a = 0; a < nx; ++a)
                acc += T(wx[a] * wy[b] * wz[c]) * C.x[Jx[a] + (int64_t)C.ux * (Jy[b] + (int64_t)C.uy * Jz[c])];
    F.t[i] = acc;
}

// x = t + w D^{-1} (b - A t)
template <typename T>
__device__ __forceinline__ void postsmooth(const MGLevelView<T> &L, T w, int64_t i) {
    int X, Y, Z;
    coords(L, i, X, Y, Z);
    const T At = stencil_apply(L, i, X, Y, Z, [&](int64_t j) { return L.t[j]; });
    L.x[i] = L.t[i] + w * L.dinv[i] * (L.b[i] - At);
}

enum { MG_PRE = 0, MG_RESTRICT = 1, MG_PROLONG = 2, MG_POST = 3 };

template <typename T, int STEP>
__global__ void __launch_bounds__(kMGStepThreads) k_mg_step(const double *__restrict__ gate, MGLevel<T> fine,
                                                            MGLevel<T> coarse, T w) {
    if (gated(gate)) return;
    const MGLevelView<T> F = view(fine), C = view(coarse);
    const int64_t n = STEP == MG_RESTRICT ? C.nv : F.nv;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (STEP == MG_PRE) presmooth_residual(F, w, i);
        else if (STEP == MG_RESTRICT) restrict_vertex(F, C, i);
        else if (STEP == MG_PROLONG) prolong_vertex(F, C, i);
        else postsmooth(F, w, i);
    }
}

// Levels l0 .. nlev-1 in one workgroup: down to the coarsest level, its solve with the dense
// inverse (at most kMGTailCoarsest unknowns: below the tail level's size / 8), and back up.
template <typename T>
__global__ void __launch_bounds__(kMGTailThreads) k_mg_tail(const double *__restrict__ gate, MGCycle<T> M, int l0) {
    if (gated(gate)) return;
    const int tid = threadIdx.x;
    const int last = M.nlev - 1;
    for (int l = l0; l < last; ++l) {
        const MGLevelView<T> F = view(M.L[l]), C = view(M.L[l + 1]);
        for (int64_t i = tid; i < F.nv; i += kMGTailThreads) presmooth_residual(F, M.omega, i);
        __syncthreads();
        for (int64_t i = tid; i < C.nv; i += kMGTailThreads) restrict_vertex(F, C, i);
        __syncthreads();
    }
    {   // coarsest: x = A^{-1} b with the symmetric dense inverse read column-wise (coalesced)
        const MGLevelView<T> C = view(M.L[last]);
        for (int64_t i = tid; i < C.nv; i += kMGTailThreads) {
            T acc[4] = {0, 0, 0, 0};
            for (int64_t j = 0; j < C.nv; ++j) acc[j & 3] += M.cinv[j * C.nv + i] * C.b[j];
            C.x[i] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        }
        __syncthreads();
    }
    for (int l = last - 1; l >= l0; --l) {
        const MGLevelView<T> F = view(M.L[l]), C = view(M.L[l + 1]);
        for (int64_t i = tid; i < F.nv; i += kMGTailThreads) prolong_vertex(F, C, i);
        __syncthreads();
        for (int64_t i = tid; i < F.nv; i += kMGTailThreads) postsmooth(F, M.omega, i);
        __syncthreads();
    }
}

template <typename T, int STEP>
void step(const MGCycle<T> &M, int l, const Exec &e) {
    const MGLevel<T> &F = M.L[l], &C = M.L[l + 1 < M.nlev ? l + 1 : l];
    const int64_t nf = (int64_t)(F.cx - 1) * (F.cy - 1) * (F.cz - 1), nc = (int64_t)(C.cx - 1) * (C.cy - 1) * (C.cz - 1);
    hipLaunchKernelGGL((k_mg_step<T, STEP>), dim3(grid_for(STEP == MG_RESTRICT ? nc : nf, kMGStepThreads)),
                       dim3(kMGStepThreads), 0, e.s, e.gate, F, C, M.omega);
}

}  // namespace

template <typename T>
void launch_mg_vcycle(const MGCycle<T> &M, const Exec &e) {
    if (M.nlev < 1 || M.nlev > kMGMaxLevels) throw Error(VSR_EINVAL, "multigrid level count out of range");
    const int last = M.nlev - 1;
    const int64_t ncoarse = (int64_t)(M.L[last].cx - 1) * (M.L[last].cy - 1) * (M.L[last].cz - 1);
    if (M.nlev == 1) {   // the direct solve
        launch_dense_gemv<T>((int)ncoarse, M.cinv, M.L[0].b, M.L[0].x, T(1), T(0), e);
        return;
    }
    int tail = last;
    for (int l = 0; l < last; ++l)
        if ((int64_t)(M.L[l].cx - 1) * (M.L[l].cy - 1) * (M.L[l].cz - 1) <= kMGTailVertices) {
            tail = l;
            break;
        }
    for (int l = 0; l < tail; ++l) {
        step<T, MG_PRE>(M, l, e);
        step<T, MG_RESTRICT>(M, l, e);
    }
    if (tail < last) {
        // the tail level has at most kMGTailVertices vertices and the coarsest fewer than an
        // eighth of them, so the coarsest solve fits the single workgroup too
        if (ncoarse > kMGTailCoarsest) throw Error(VSR_EINVAL, "coarsest multigrid level too large for the tail launch");
        hipLaunchKernelGGL((k_mg_tail<T>), dim3(1), dim3(kMGTailThreads), 0, e.s, e.gate, M, tail);
    } else {
        // only the coarsest level is small enough (or no level is): its solve spreads over the GPU
        launch_dense_gemv<T>((int)ncoarse, M.cinv, M.L[last].b, M.L[last].x, T(1), T(0), e);
    }
    for (int l = tail - 1; l >= 0; --l) {
        step<T, MG_PROLONG>(M, l, e);
        step<T, MG_POST>(M, l, e);
    }
}

template void launch_mg_vcycle<float>(const MGCycle<float> &, const Exec &);
template void launch_mg_vcycle<double>(const MGCycle<double> &, const Exec &);

}  // namespace vsr
