// Launch wrappers of the HIP kernels (gfx950).  All pointers are device pointers;
// every launch goes to `stream`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vsr {

struct Dims {
    int nx, ny, nz;       // cells per axis
    int p, q;
    int Lx, Ly, Lz;       // free lattice extents (p*n - 1)
};

// y += A x (y must be zeroed by the caller); Cartesian (separable) or general metric.
template <typename T>
void launch_op_kron(const Dims &d, const T *AB1d, const T *mu, const T *x, T *y, hipStream_t s);
template <typename T>
void launch_op_general(const Dims &d, const T *IDq, const T *Gw, const T *x, T *y, hipStream_t s);
// b += sum_K R_K^T (I x I x I)^T (wdet .* f)
void launch_load_vector(const Dims &d, const double *IDq, const double *wdet, const double *f, double *b,
                        hipStream_t s);

// One 1D lattice pass: out = alpha * (table along `axis`) in + beta * out.
template <typename Tin, typename Tout>
void launch_axis_pass(const int *rowptr, const int *col, const Tout *w, int axis, const int in_dims[3],
                      const int out_dims[3], const Tin *in, Tout *out, Tout alpha, Tout beta, hipStream_t s);

struct PatchArgs {
    int m, w;
    int n_leaf, n_sep, n_top, n_iface, top_pad, ntiles;
    int64_t off_invd, off_B1, off_B2, off_Lsep, off_P, off_Ltop, stride;
};

template <typename T>
void launch_patch_interior(const Dims &d, const PatchArgs &a, int npatch, const int *verts, const T *factor,
                           const T *mu, const T *lam, const T *afc, const T *rF, T *U, hipStream_t s);
template <typename T>
void launch_patch_boundary(const Dims &d, int npatch, const int *desc, const int64_t *off, const T *factor,
                           const T *mu, const T *lam, const T *afc, const T *rF, T *U, hipStream_t s);
template <typename T>
void launch_patch_assemble(const Dims &d, int interior_only, const T *U, T *zF, hipStream_t s);

// y = alpha * A x + beta * y for a dense row-major n x n matrix.
template <typename T>
void launch_dense_gemv(int n, const T *A, const T *x, T *y, T alpha, T beta, hipStream_t s);

// ---- vector kernels (double unless noted)
template <typename Tin, typename Tout>
void launch_cast(int64_t n, const Tin *x, Tout *y, hipStream_t s);
template <typename T>
void launch_fill(int64_t n, T *x, T v, hipStream_t s);
// partial sums of x.y into partials[nblocks]; returns nblocks used
int launch_dot_partial(int64_t n, const double *x, const double *y, double *partials, hipStream_t s);
// scal[slot] = sum(partials); mode: 0 plain, 1 alpha = scal[RZ]/sum, 2 beta = sum/scal[RZ] and RZ = sum
void launch_finalize(int nb, const double *partials, double *scal, int mode, hipStream_t s);
// x += alpha p ; r -= alpha q ; partial r.r
int launch_pcg_xr(int64_t n, double *x, double *r, const double *p, const double *q, const double *scal,
                  double *partials, hipStream_t s);
// p = z + beta p
void launch_pcg_p(int64_t n, double *p, const double *z, const double *scal, hipStream_t s);
// out(T) = r(double) - Az(T) ; out may alias Az
template <typename T>
void launch_residual(int64_t n, const double *r, const T *Az, T *out, hipStream_t s);
// y(double) = a * x(T) + b * y
template <typename T>
void launch_axpby_to_double(int64_t n, double a, const T *x, double b, double *y, hipStream_t s);

enum { SC_PQ = 0, SC_RZ = 1, SC_RR = 2, SC_ALPHA = 3, SC_BETA = 4, SC_RZNEW = 5, SC_TMP = 6, SC_N = 8 };

}  // namespace vsr
