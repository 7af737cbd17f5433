// Launch wrappers of the HIP kernels (gfx950).  All pointers are device pointers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vsr {

struct Dims {
    int nx, ny, nz;       // cells per axis
    int p, q;
    int Lx, Ly, Lz;       // free lattice extents (p*n - 1)
};

// Launch shapes chosen per (degree, precision) by the autotuner; none changes the
// arithmetic of any output value.
struct Tuning {
    int op_cpw64 = 1;       // cells per workgroup of the Cartesian operator kernel, FP64
    int op_cpw32 = 1;       // same, FP32 (both 1, 2 or 4; above 1 only for p <= 7)
    int axis_block = 256;   // threads per block of the 1D lattice passes (64..1024)
    int patch_unroll = 8;   // column loads in flight per thread in the patch panels (4, 8, 16)
    int opg_split64 = 0;    // workgroups per cell of the general operator, FP64 (1, 2; 0: by size)
    int opg_split32 = 0;    // same, FP32
    int axis_tiled = 0;     // lattice passes with whole lines staged in LDS (1) or streamed (0)
    int patch_threads = 256;   // threads per patch workgroup (256 or 512: more panel loads in flight)
};

// Where a launch goes: its stream, an optional gate (a device flag; when it is nonzero
// at kernel start every workgroup returns at once) and the launch shapes.
struct Exec {
    hipStream_t s = nullptr;
    const double *gate = nullptr;
    Tuning t{};
};

// y += A x (y must be zeroed by the caller); Cartesian (separable) or general metric.
template <typename T>
void launch_op_kron(const Dims &d, const T *AB1d, const T *mu, const T *x, T *y, const Exec &e);
template <typename T>
void launch_op_general(const Dims &d, const T *IDq, const T *Gw, const T *x, T *y, const Exec &e);
// b += sum_K R_K^T (I x I x I)^T (wdet .* f)
void launch_load_vector(const Dims &d, const double *IDq, const double *wdet, const double *f, double *b,
                        const Exec &e);

// One 1D lattice pass: out = alpha * (banded 1D matrix along `axis`) in + beta * out; output o
// reads in[start[o] + j], j < bw, along the axis with weight w[o * bw + j].
template <typename Tin, typename Tout>
void launch_axis_pass(const int *start, int bw, const Tout *w, int axis, const int in_dims[3],
                      const int out_dims[3], const Tin *in, Tout *out, Tout alpha, Tout beta, const Exec &e);

struct PatchArgs {
    int m, w;
    int n_leaf, n_sep, n_top, n_iface, top_pad, ntiles;
    int64_t off_invd, off_B1, off_B2, off_Lsep, off_P, off_Ltop, stride;
};

// All patches in one launch (interior first, then boundary).
template <typename T>
void launch_patch_all(const Dims &d, const PatchArgs &a, int n_int, const int *verts, const int *fidx, const T *fint, int n_bnd,
                      const int *desc, const int64_t *off, const T *fbnd, const T *mu, const T *lam, const T *afc,
                      const T *rF, T *U, const Exec &e);
template <typename T>
void launch_patch_assemble(const Dims &d, int interior_only, const T *U, T *zF, const Exec &e);

// y = alpha * A x + beta * y for a dense row-major n x n matrix.
template <typename T>
void launch_dense_gemv(int n, const T *A, const T *x, T *y, T alpha, T beta, const Exec &e);

// ---- vector kernels (double unless noted)
template <typename Tin, typename Tout>
void launch_cast(int64_t n, const Tin *x, Tout *y, const Exec &e);
template <typename T>
void launch_fill(int64_t n, T *x, T v, const Exec &e);
// x.y reduced into scal (partials: 1024 doubles of scratch; two launches, the second adds the
// partials in a fixed order).  mode: 0 plain (TMP), 1 p.q -> alpha = RZ / p.q,
// 2 r.z -> beta = r.z / RZ and RZ = r.z, 3 RZ = r.z, 4 RR = r.r, 5 RR = r.r after an x update
// with the stopping test of a device-driven PCG (see SC_DONE).  mirror (may be NULL): host-
// visible copy of DONE written with it.
void launch_dot(int64_t n, const double *x, const double *y, double *partials, double *scal, int mode, double *mirror,
                const Exec &e);
// Start of a device-driven PCG after RR = b.b: BB = RR, IT = 0, stopping data, DONE when b = 0
// or b is not finite (mirrored).  Not gated.
void launch_pcg_start(double *scal, double rtol, int max_iterations, double *mirror, const Exec &e);
// x += alpha p ; r -= alpha q ; q = 0 ; r.r reduced into scal by mode (4 or 5)
void launch_pcg_xr(int64_t n, double *x, double *r, const double *p, double *q, double *scal, double *partials, int mode,
                   double *mirror, const Exec &e);
// p = z + beta p
void launch_pcg_p(int64_t n, double *p, const double *z, const double *scal, const Exec &e);
// out(T) = r(double) - Az(T), then Az = 0 ; out must not alias Az
template <typename T>
void launch_residual(int64_t n, const double *r, T *Az, T *out, const Exec &e);
// y(double) = a * x(T) + b * y
template <typename T>
void launch_axpby_to_double(int64_t n, double a, const T *x, double b, double *y, const Exec &e);
// Device scalars of one PCG.  A device-driven PCG (batched solves) keeps its stopping state
// here: DONE is nonzero once the member stops; STATUS 1 converged, 2 non-finite residual,
// 3 iteration cap; IT counts x updates.
enum {
    SC_PQ = 0, SC_RZ = 1, SC_RR = 2, SC_ALPHA = 3, SC_BETA = 4, SC_RZNEW = 5, SC_TMP = 6,
    SC_DONE = 8, SC_BB = 9, SC_RTOL2 = 10, SC_IT = 11, SC_MAXIT = 12, SC_STATUS = 13,
    SC_N = 16
};

}  // namespace vsr
