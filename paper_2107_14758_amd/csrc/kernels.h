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
    int op_cpw32 = 4;       // same, FP32 (both 1, 2 or 4; above 1 only for p <= 7)
    int patch_unroll = 4;   // column loads in flight per thread in the patch panels (4, 8, 16)
    int opg_split64 = 0;    // workgroups per cell of the general operator, FP64 (1, 2; 0: by size)
    int opg_split32 = 0;    // same, FP32
    int patch_threads = 256;   // threads per patch workgroup (256, 512, or 1024 with unroll 4 or 8)
};

// Where a launch goes: its stream, an optional gate (a device flag; when it is nonzero
// at kernel start every workgroup returns at once) and the launch shapes.
struct Exec {
    hipStream_t s = nullptr;
    const double *gate = nullptr;
    Tuning t{};
};

// Cell-local operator y_K = A^K x_K into the element vector E ((p+1)^3 values per cell, in
// rows of x across cells: local node (k, j, i) of cell (ex, ey, ez) at
// (((ez ny + ey)(p+1) + k)(p+1) + j) nx (p+1) + ex (p+1) + i).  Cartesian (separable) cells:
// one slot.  General metric: `slots` partial slots (the return value), slot s at
// s ncell (p+1)^3.  launch_gather turns E into the lattice vector.
template <typename T>
void launch_op_kron(const Dims &d, const T *AB1d, const T *mu, const T *x, T *E, const Exec &e);
// General (trilinear) cells: IDq = [Iq (q x (p+1)), Dq (q x (p+1)), GLL points x_q (q), weights
// w_q (q)]; geo: kGeoStride values per cell, the halved edge differences of its corners
// X[c][b][a] (x fastest): 0.5 (X[c][b][1] - X[c][b][0]) at 3 (2c + b), 0.5 (X[c][1][a] -
// X[c][0][a]) at 12 + 3 (2c + a), 0.5 (X[1][b][a] - X[0][b][a]) at 24 + 3 (2b + a), then kappa
// at 36 (make_cell_geometry).
constexpr int kGeoStride = 40;
// Returns the number of element-vector slots written (workgroups per cell).  In FP64 from
// degree kOpgMfmaMinP on, the x and y contractions run on the matrix cores (op_mfma.hip):
// 8^3 cells at p = 15 take 0.15 instead of 0.39 ms; below it the padding of q to 32 costs
// more than the matrix cores gain, and in FP32 they gain nothing measurable.
constexpr int kOpgMfmaMinP = 13;
template <typename T>
int launch_op_general(const Dims &d, const T *IDq, const T *geo, const T *x, T *E, const Exec &e);
template <typename T>
int launch_op_general_mfma(const Dims &d, int split, const T *IDq, const T *geo, const T *x, T *E, const Exec &e);
// Cartesian operator followed by a restriction of the cell results (Sec. 2.4, 2.5): kind 1
// stores (That^T x3) (A^K x_K) per cell in the element-vector layout (launch_gather_sub then
// assembles FDM covectors), kind 2 stores the 8 Q1 corner values (N^T x3) (A^K x_K) per cell
// at E[8 cell + corner] (launch_coarse_gather assembles them).  Entries at Dirichlet nodes are
// dropped first.  AB1d = [A, B, That (node x function), Nh (2 x (p+1): the linear hats at the
// GLL nodes)], each row-major.
template <typename T>
void launch_op_kron_restrict(const Dims &d, int kind, const T *AB1d, const T *mu, const T *x, T *E, const Exec &e);
// out = rT - (the single-slot element vector E summed per free node), all in T.
template <typename T>
void launch_gather_sub(const Dims &d, const T *E, const T *rT, T *out, const Exec &e);
// c3 = c0 - (the per-cell corner values e8 summed over the 8 cells around each interior vertex).
template <typename T>
void launch_coarse_gather(const Dims &d, const T *c0, const T *e8, T *c3, const Exec &e);
// out = sum over the cells and slots that share each free node of E (r == nullptr), or
// out = r - that sum (in T).  Deterministic: a fixed summation order, no atomics.  With
// dotv, also the partial sums of dotv . out, one per workgroup (gather_blocks of them), into
// partials for launch_finalize.
template <typename T>
void launch_gather(const Dims &d, int slots, const T *E, const double *r, T *out, const Exec &e,
                   const double *dotv = nullptr, double *partials = nullptr);
// ncomp independent gathers in one launch: out + c n = the sum of the single-slot element
// vector E + c ncell (p+1)^3 per free node (with r: r + c n minus that sum), for c < ncomp
// (n = free nodes).
template <typename T>
void launch_gather_components(const Dims &d, int ncomp, const T *E, T *out, const Exec &e, const double *r = nullptr);
int64_t gather_blocks(const Dims &d);
// Adds nb partial sums in a fixed order and applies them to scal by mode (see launch_dot).
void launch_finalize(int nb, const double *partials, double *scal, int mode, double *mirror, const Exec &e);
// Cell blocks E_K = (I x I x I)^T (wdet .* f) of the load vector, in the element-vector
// layout (one slot); launch_gather with slots = 1 turns them into b = sum_K R_K^T E_K.
void launch_load_vector(const Dims &d, const double *IDq, const double *wdet, const double *f, double *E,
                        const Exec &e);

// Lattice transfers, each in one launch (M x M x M with a cell-blocked 1D map M):
// FDM restriction r~ = T^T r and prolongation z = T z~ on the free fine lattice (Sec. 2.4);
// Q1 restriction P^T (fine -> interior coarse vertices) and prolongation P (Sec. 2.5).
// kind is one of XFER_* (vsr_internal.h) and M its OA x K block matrix (transfer_block);
// out = alpha * (map) in + beta * out.  With out64 non-null every output is also stored
// there widened to FP64; with partials non-null too, each workgroup leaves its sum of
// dotv . out64 over the outputs it owns in partials[block] (transfer_blocks of them, zeros
// from workgroups that own none) for launch_finalize.
// box_mode (XFER_FDM_PROLONG up to degree kFusedScatterMaxP): 1 = in holds the patch solves'
// star boxes ((2p-1)^3 per mesh vertex) and the prolongation reads their assembled sum (the
// scatter-add of Sec. 2.5) instead of a lattice vector; 2 = the same with only the interior
// vertices' stars; 0 = a lattice vector.  ncomp > 1: that many independent inputs (lattice
// vectors, or with box_mode the star boxes of that many patch-solve launches) and outputs one
// after another in `in`, `out` and out64 (no dotv or partials), one launch.
template <typename Tin, typename T>
void launch_transfer(int kind, int p, const int ncell[3], const int in_dims[3], const int out_dims[3], const T *M,
                     const Tin *in, T *out, T alpha, T beta, const Exec &e, double *out64 = nullptr,
                     const double *dotv = nullptr, double *partials = nullptr, int box_mode = 0, int ncomp = 1);
// Workgroups of one launch_transfer of this kind.
int transfer_blocks(int kind, int p, const int ncell[3]);

struct PatchArgs {
    int m, w;
    int n_leaf, n_sep, n_top, n_iface, top_pad, ntiles;
    int64_t off_invd, off_B1, off_B2, off_Lsep, off_Sy, off_Ltop, stride;
    int det;   // 1: every panel sum taken by one thread in a fixed order (no LDS atomics)
};

// All patches in one launch (interior first, then boundary).  U receives the patch
// solutions (patch_solution_entries values): up to degree kFusedScatterMaxP one (2p-1)^3
// box per mesh vertex, read by the fused prolongation; above it 8 lattice vectors of n free
// nodes each, one per vertex-parity class (vx mod 2) + 2 (vy mod 2) + 4 (vz mod 2), read by
// launch_patch_assemble.  Either way, entries no star writes must hold zero (the caller
// zeroes U once; the kernel writes its stars' entries only).
// Independent problems of one structure (the same mesh, degree and patch layout) in one launch:
// problem c's arrays start c strides after the first's (elements of T).
struct CompStrides {
    int64_t fint = 0, fbnd = 0, mu = 0, rF = 0, U = 0;
};
// ncomp > 1: that many such problems, blockIdx.y selecting one.
template <typename T>
void launch_patch_all(const Dims &d, const PatchArgs &a, int n_int, const int *verts, const int *fidx, const T *fint, int n_bnd,
                      const int *desc, const int64_t *off, const T *fbnd, const T *mu, const T *lam, const T *afc,
                      const T *rF, T *U, const Exec &e, int ncomp = 1, CompStrides cs = CompStrides{});

// Additive Schwarz sum z_F = sum_j Rbar_j^T u_j (Sec. 2.5) into a lattice vector (degrees above
// kFusedScatterMaxP; up to it the prolongation reads the star boxes itself).
// ncomp > 1: that many (U, zF) pairs one after another, one launch.
template <typename T>
void launch_patch_assemble(const Dims &d, const T *U, T *zF, const Exec &e, int ncomp = 1);
// Primal linear elasticity on axis-aligned cells (Sec. 3.1), FP64 or FP32: the three components'
// cell results of y = A x into E (three element vectors of ncell (p+1)^3, one per output
// component; launch_gather_components sums them).  M1: the 1-D matrices A, B, C, C^T ((p+1)^2 each,
// row = test index; C[a][b] = int phi_a' phi_b); coef: 12 per cell (k[c][a] at 3c + a, then
// s_xy, s_xz, s_yz); x: 3 n values, component after component.
template <typename T>
void launch_op_elastic_box(const Dims &d, const T *M1, const T *coef, T mu, T lam, const T *x, T *E, const Exec &e);

constexpr int kFusedScatterMaxP = 7;
// Length of U for launch_patch_all.
inline int64_t patch_solution_entries(const Dims &d) {
    const int64_t w = 2 * d.p - 1;
    return d.p <= kFusedScatterMaxP ? (int64_t)(d.nx + 1) * (d.ny + 1) * (d.nz + 1) * w * w * w
                                    : 8 * (int64_t)d.Lx * d.Ly * d.Lz;
}

// y = alpha * A x + beta * y for a dense row-major n x n matrix.
template <typename T>
void launch_dense_gemv(int n, const T *A, const T *x, T *y, T alpha, T beta, const Exec &e);

// Geometric multigrid for the p-coarse (Q1) problem (Sec. 2.8).  Level l has cx x cy x cz
// cells and (cx-1)(cy-1)(cz-1) interior vertices (x fastest); st: its 27-point stencil stored
// [s][vertex], s = (dz+1) 9 + (dy+1) 3 + (dx+1); dinv: inverse diagonal; x, b, r, t: work
// vectors (solution, right-hand side, residual, corrected iterate).  Level l+1 halves every
// axis; transfers are trilinear in index space.  cinv: dense inverse of the last level.
constexpr int kMGMaxLevels = 12;
constexpr int64_t kMGTailVertices = 1024;   // levels this small run in one single-workgroup launch
constexpr int64_t kMGTailCoarsest = 128;    // coarsest solved inside that launch up to this size
template <typename T>
struct MGLevel {
    int cx = 0, cy = 0, cz = 0;
    const T *st = nullptr, *dinv = nullptr;
    T *x = nullptr, *b = nullptr, *r = nullptr, *t = nullptr;
};
template <typename T>
struct MGCycle {
    int nlev = 0;
    T omega = T(2) / T(3);   // damped point-Jacobi weight
    const T *cinv = nullptr;
    MGLevel<T> L[kMGMaxLevels];
};
// One V(1,1) cycle from zero: L[0].x = B L[0].b (one Jacobi step before and after the coarse
// correction on every level, the coarsest solved with cinv).  nlev = 1 is the direct solve.
template <typename T>
void launch_mg_vcycle(const MGCycle<T> &M, const Exec &e);

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
// Start of a device-driven PCG after RR = b.b: BB = RR, IT = 0, stopping data (stagnation
// test over `window` iterations for a drop of r.r below factor^2 of its reference; window 0:
// none), DONE when b = 0 or b is not finite (mirrored).  Not gated.
void launch_pcg_start(double *scal, double rtol, int max_iterations, int window, double factor, double *mirror,
                      const Exec &e);
// x += alpha p ; r -= alpha q ; r.r reduced into scal by mode (4 or 5)
void launch_pcg_xr(int64_t n, double *x, double *r, const double *p, const double *q, double *scal, double *partials, int mode,
                   double *mirror, const Exec &e);
// p = z + beta p
void launch_pcg_p(int64_t n, double *p, const double *z, const double *scal, const Exec &e);
// y(double) = a * x(T) + b * y; with dotv, also the partial sums of dotv . y (one per
// workgroup; the return value is their count) into partials for launch_finalize
template <typename T>
int launch_axpby_to_double(int64_t n, double a, const T *x, double b, double *y, const Exec &e,
                           const double *dotv = nullptr, double *partials = nullptr);
// Device scalars of one PCG.  A device-driven PCG (batched solves) keeps its stopping state
// here: DONE is nonzero once the member stops; STATUS 1 converged, 2 non-finite residual,
// 3 iteration cap, 4 stagnated (r.r has not fallen below SFAC2 times its reference value
// REF for WIN consecutive iterations; REF is b.b at the start and each r.r that did fall
// below it; SINCE counts the iterations since; WIN 0: no test); IT counts x updates.
// Behind the SC_N scalars lie HCAP pairs
// (alpha_j, beta_j) of the current (P)CG run: an initial r.z (mode 3) empties the record,
// every step length (mode 1) appends alpha_j and counts it in NA, every direction update
// (mode 2) stores beta_{NA-1}; steps past HCAP are not recorded.  They are the
// coefficients of the run's Lanczos tridiagonal (condition estimate of P^{-1} A).
enum {
    SC_PQ = 0, SC_RZ = 1, SC_RR = 2, SC_ALPHA = 3, SC_BETA = 4, SC_RZNEW = 5, SC_TMP = 6,
    SC_NA = 7, SC_DONE = 8, SC_BB = 9, SC_RTOL2 = 10, SC_IT = 11, SC_MAXIT = 12, SC_STATUS = 13,
    SC_HCAP = 14, SC_REF = 15, SC_SINCE = 16, SC_WIN = 17, SC_SFAC2 = 18, SC_N = 24
};

}  // namespace vsr
