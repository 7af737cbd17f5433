// C ABI (include/vsr.h): problem setup, operator/relaxation applies, PCG driver.
//
// Method references: Brubeck & Farrell, "A scalable and robust vertex-star
// relaxation for high-order FEM", Sec. 2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "kernels.h"
#include "vsr_internal.h"

using namespace vsr;

namespace vsr {
thread_local std::string g_last_error_text;
}
namespace {

template <typename F>
vsr_status guarded(F &&f) {
    try {
        f();
        return VSR_OK;
    } catch (const Error &e) {
        vsr::g_last_error_text = e.what();
        return e.status;
    } catch (const std::bad_alloc &) {
        vsr::g_last_error_text = "host allocation failed";
        return VSR_ENOMEM;
    } catch (const std::exception &e) {
        vsr::g_last_error_text = e.what();
        return VSR_EINVAL;
    }
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct vsr_problem {
    Dims d{};
    int64_t n = 0, ncell = 0;
    vsr_options opt{};
    hipStream_t stream = nullptr;
    bool fp32 = false, cartesian = false;
    OneD od;
    std::vector<void *> allocs;

    // operator data (FP64 and FP32 copies)
    double *AB64 = nullptr, *IDq64 = nullptr, *mu64 = nullptr, *geo64 = nullptr, *wdet = nullptr;
    float *AB32 = nullptr, *IDq32 = nullptr, *mu32 = nullptr, *geo32 = nullptr;
    // relaxation data in the cycle precision
    void *mu_sur = nullptr, *lam = nullptr, *afc = nullptr, *fint = nullptr, *fbnd = nullptr;
    int64_t mu_len = 0, fint_len = 0, fbnd_len = 0;   // elements of mu_sur, fint, fbnd
    int n_int = 0, n_bnd = 0;
    int *verts = nullptr, *bdesc = nullptr, *fidx = nullptr;   // fidx: factor of each interior star
    int64_t *boff = nullptr;
    PatchArgs pa{};
    int64_t factor_entries = 0;       // structurally nonzero entries over all patches
    double bytes_patch_launch = 0;    // algorithmic bytes of one patch-solve launch (all stars)
    double *xm64[4] = {};             // cell blocks of T^T, T, P^T, P (transfer_block)
    float *xm32[4] = {};
    int cdim[3] = {0, 0, 0};
    int nc = 0;
    void *A0inv = nullptr;
    int coarse_gmg = 0;               // 1: the coarse problem is solved by a multigrid V-cycle
    MGCycle<float> mg32{};
    MGCycle<double> mg64{};
    // work buffers (cycle precision unless noted)
    void *rF = nullptr, *zF = nullptr, *U = nullptr;   // zF: assembled patch solutions (p > 7)
    void *c3 = nullptr, *c4 = nullptr;    // coarse right-hand side and solution
    void *z1 = nullptr, *res = nullptr;   // cycle iterate and cycle residual
    void *rF0 = nullptr, *c0 = nullptr, *e8 = nullptr;   // T^T r, P^T r and per-cell Q1 corner values
                                                        // of the Cartesian V-cycle
    double *E64 = nullptr;                // element vectors of the operator (2 slots per cell)
    void *E32 = nullptr;
    double *vp = nullptr, *vq = nullptr, *vr = nullptr, *vz = nullptr, *vt = nullptr;
    double *scal = nullptr, *partials = nullptr, *host_scal = nullptr;
    double omega = 1.0, lmin = 0.0, lmax = 0.0;
    double setup_seconds = 0.0;
    // launch context: an optional gate (set while a batched solve drives this problem)
    // and the launch shapes chosen by the autotuner
    const double *gate = nullptr;
    double *mirror = nullptr;         // host-visible copy of the stop flag (batched solves)
    Tuning tune{};
    uint64_t tune_version = 0;        // bumped by every vsr_set_tuning
    double *vx = nullptr;             // solution of a batched solve
    vsr_batch *self = nullptr;        // batch of this problem alone (graph-replayed single solves)
    // host copies of the setup inputs, for the FP64 setup a stagnated FP32 solve continues on
    int in_nx = 0, in_ny = 0, in_nz = 0;
    std::vector<double> in_vertices, in_kappa, in_mu;
    vsr_problem *twin = nullptr;      // that FP64 setup (made at the first stagnation)
    double *ve = nullptr;             // its correction e
    Exec ex() const { return Exec{stream, gate, tune}; }
    // profiling of the interior patch-solve launches
    bool profiling = false;
    bool capturing = false;           // launches are being recorded into a graph
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;   // reusable pool
    size_t events_used = 0;

    ~vsr_problem() {
        for (auto &e : events) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        if (host_scal) (void)hipHostFree(host_scal);
        for (void *p : allocs) (void)hipFree(p);
    }

    template <typename T>
    T *dalloc(size_t count) {
        void *p = nullptr;
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (hipMalloc(&p, bytes) != hipSuccess) throw Error(VSR_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        allocs.push_back(p);
        return static_cast<T *>(p);
    }
    template <typename T>
    T *upload(const std::vector<T> &v) {
        T *p = dalloc<T>(v.size());
        if (!v.empty()) VSR_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return p;
    }
    template <typename T>
    T *upload_as(const std::vector<double> &v) {
        std::vector<T> c(v.begin(), v.end());
        return upload(c);
    }
    // Move `bytes` of device data from *slot to dst (device memory the caller owns) and free
    // the old allocation: *slot then points at dst.
    void move_to(void **slot, void *dst, size_t bytes) {
        VSR_HIP(hipMemcpy(dst, *slot, bytes, hipMemcpyDeviceToDevice));
        auto it = std::find(allocs.begin(), allocs.end(), *slot);
        if (it != allocs.end()) {
            (void)hipFree(*it);
            allocs.erase(it);
        }
        *slot = dst;
    }
};

namespace {

// Dense coarse inverse up to this many Q1 unknowns (21^3 cells) under coarse_solver = 0.
constexpr int kAutoDenseCoarse = 8000;

// Device copy of a multigrid hierarchy in the cycle precision T.  Level 0's right-hand side and
// solution are the coarse-space vectors c3 and c4 of the Q1 transfers.
template <typename T>
void build_mg(vsr_problem *P, const MGHierarchyHost &H, MGCycle<T> &M) {
    M = MGCycle<T>{};
    M.nlev = (int)H.levels.size();
    M.cinv = (const T *)P->A0inv;
    for (int l = 0; l < M.nlev; ++l) {
        const MGLevelHost &h = H.levels[l];
        MGLevel<T> &L = M.L[l];
        L.cx = h.cx; L.cy = h.cy; L.cz = h.cz;
        const int64_t nv = (int64_t)(h.cx - 1) * (h.cy - 1) * (h.cz - 1);
        std::vector<double> dinv(nv);
        for (int64_t i = 0; i < nv; ++i) {
            const double dg = h.st[(size_t)13 * nv + i];
            if (!(dg > 0)) throw Error(VSR_ENOTSPD, "non-positive diagonal in a multigrid level");
            dinv[i] = 1.0 / dg;
        }
        L.st = P->upload_as<T>(h.st);
        L.dinv = P->upload_as<T>(dinv);
        L.r = P->dalloc<T>(nv);
        L.t = P->dalloc<T>(nv);
        if (l == 0) {
            L.b = (T *)P->c3;
            L.x = (T *)P->c4;
        } else {
            L.b = P->dalloc<T>(nv);
            L.x = P->dalloc<T>(nv);
        }
    }
}

// The cell-local operator into the element vector of precision T; returns its slots per cell.
template <typename T>
int op_cells(vsr_problem *P, const T *x, T *E) {
    if constexpr (std::is_same<T, double>::value) {
        if (P->cartesian) {
            launch_op_kron<double>(P->d, P->AB64, P->mu64, x, E, P->ex());
            return 1;
        }
        return launch_op_general<double>(P->d, P->IDq64, P->geo64, x, E, P->ex());
    } else {
        if (P->cartesian) {
            launch_op_kron<float>(P->d, P->AB32, P->mu32, x, E, P->ex());
            return 1;
        }
        return launch_op_general<float>(P->d, P->IDq32, P->geo32, x, E, P->ex());
    }
}

template <typename T>
T *elem(vsr_problem *P) {
    if constexpr (std::is_same<T, double>::value) return P->E64;
    else return (T *)P->E32;
}

// y = A x
template <typename T>
void op_apply(vsr_problem *P, const T *x, T *y) {
    const int slots = op_cells<T>(P, x, elem<T>(P));
    launch_gather<T>(P->d, slots, elem<T>(P), nullptr, y, P->ex());
    VSR_HIP(hipGetLastError());
}

// out = r - A x (out in T)
template <typename T>
void op_residual(vsr_problem *P, const double *r, const T *x, T *out) {
    const int slots = op_cells<T>(P, x, elem<T>(P));
    launch_gather<T>(P->d, slots, elem<T>(P), r, out, P->ex());
    VSR_HIP(hipGetLastError());
}

template <typename T>
const T *xm(const vsr_problem *P, int kind) {
    if constexpr (std::is_same<T, double>::value) return P->xm64[kind];
    else return P->xm32[kind];
}

// out = alpha * S in + beta * out,  S = T (sum_j Rbar_j^T A_j^{-1} Rbar_j) T^T  (Sec. 2.4-2.6);
// out64, dotv and partials as for launch_transfer (the prolongation writes out)
// rF_given (may be NULL): T^T of the input, already formed (in is then not read).
template <typename T, typename Tin>
void relax_apply(vsr_problem *P, const Tin *in, T *out, T alpha, T beta, double *out64 = nullptr,
                 const double *dotv = nullptr, double *partials = nullptr, const T *rF_given = nullptr) {
    const int L[3] = {P->d.Lx, P->d.Ly, P->d.Lz}, NC[3] = {P->d.nx, P->d.ny, P->d.nz};
    const T *rF = rF_given ? rF_given : (const T *)P->rF;
    T *U = (T *)P->U;
    if (!rF_given)
        launch_transfer<Tin, T>(XFER_FDM_RESTRICT, P->d.p, NC, L, L, xm<T>(P, XFER_FDM_RESTRICT), in, (T *)P->rF, T(1),
                                T(0), P->ex());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool prof = P->profiling && !P->capturing;
    if (prof) {
        if (P->events_used == P->events.size()) {
            VSR_HIP(hipEventCreate(&e0));
            VSR_HIP(hipEventCreate(&e1));
            P->events.push_back({e0, e1});
        }
        e0 = P->events[P->events_used].first;
        e1 = P->events[P->events_used].second;
        VSR_HIP(hipEventRecord(e0, P->stream));
    }
    launch_patch_all<T>(P->d, P->pa, P->n_int, P->verts, P->fidx, (const T *)P->fint, P->n_bnd, P->bdesc, P->boff,
                        (const T *)P->fbnd, (const T *)P->mu_sur, (const T *)P->lam, (const T *)P->afc, rF, U, P->ex());
    if (prof) {
        VSR_HIP(hipEventRecord(e1, P->stream));
        ++P->events_used;
    }
    if (P->d.p <= kFusedScatterMaxP) {
        // scatter-add of the star boxes fused into the prolongation's window loads (measured
        // faster up to degree 7; above it the windows' scattered box loads cost more than a
        // separate assembly pass)
        launch_transfer<T, T>(XFER_FDM_PROLONG, P->d.p, NC, L, L, xm<T>(P, XFER_FDM_PROLONG), U, out, alpha, beta,
                              P->ex(), out64, dotv, partials, P->opt.interior_patches_only ? 2 : 1);
    } else {
        T *zF = (T *)P->zF;
        launch_patch_assemble<T>(P->d, U, zF, P->ex());
        launch_transfer<T, T>(XFER_FDM_PROLONG, P->d.p, NC, L, L, xm<T>(P, XFER_FDM_PROLONG), zF, out, alpha, beta,
                              P->ex(), out64, dotv, partials);
    }
    VSR_HIP(hipGetLastError());
}

template <typename T>
const T *ab(const vsr_problem *P) {
    if constexpr (std::is_same<T, double>::value) return P->AB64;
    else return P->AB32;
}
template <typename T>
const T *mu_of(const vsr_problem *P) {
    if constexpr (std::is_same<T, double>::value) return P->mu64;
    else return P->mu32;
}

// c4 = A0^{-1} c3: dense inverse or multigrid V-cycle
template <typename T>
void coarse_solve(vsr_problem *P) {
    if (P->coarse_gmg) {
        if constexpr (std::is_same<T, double>::value) launch_mg_vcycle<double>(P->mg64, P->ex());
        else launch_mg_vcycle<float>(P->mg32, P->ex());
    } else {
        launch_dense_gemv<T>(P->nc, (const T *)P->A0inv, (const T *)P->c3, (T *)P->c4, T(1), T(0), P->ex());
    }
}

// out = alpha * P A0^{-1} P^T in + beta * out  (Sec. 2.5)
template <typename T, typename Tin>
void coarse_apply(vsr_problem *P, const Tin *in, T *out, T alpha, T beta) {
    if (P->nc == 0) {
        if (beta == T(0)) launch_fill<T>(P->n, out, T(0), P->ex());
        return;
    }
    const int L[3] = {P->d.Lx, P->d.Ly, P->d.Lz}, NC[3] = {P->d.nx, P->d.ny, P->d.nz};
    const int *c = P->cdim;
    T *c3 = (T *)P->c3, *c4 = (T *)P->c4;
    launch_transfer<Tin, T>(XFER_COARSE_RESTRICT, P->d.p, NC, L, c, xm<T>(P, XFER_COARSE_RESTRICT), in, c3, T(1), T(0),
                            P->ex());
    coarse_solve<T>(P);
    launch_transfer<T, T>(XFER_COARSE_PROLONG, P->d.p, NC, c, L, xm<T>(P, XFER_COARSE_PROLONG), c4, out, alpha, beta,
                          P->ex());
    VSR_HIP(hipGetLastError());
}

// z = M r in the cycle precision T; mode 0: preconditioner, 1: relaxation, 2: coarse.
// dot_mode >= 0: r.z is reduced into the PCG scalars by that mode (see launch_dot) in the
// same pass that writes z.
template <typename T>
void precondition(vsr_problem *P, const double *r, double *z, int mode, int dot_mode) {
    T *z1 = (T *)P->z1;
    const T w = (T)P->omega;
    if (mode == 1) {
        relax_apply<T, double>(P, r, z1, T(1), T(0));
    } else if (mode == 2) {
        coarse_apply<T, double>(P, r, z1, T(1), T(0));
    } else if (P->opt.cycle == 1) {
        relax_apply<T, double>(P, r, z1, T(1), T(0));
        coarse_apply<T, double>(P, r, z1, T(1), T(1));
    } else if (P->cartesian) {
        // hybrid V(1,1) on separable cells, with the two cycle residuals only ever restricted:
        // T^T (r - A z2) = T^T r - sum_K R_K^T That^T A^K z2_K and P^T (r - A z1) likewise, the
        // restrictions applied per cell by the operator kernel (Sec. 2.4, 2.5)
        const int L[3] = {P->d.Lx, P->d.Ly, P->d.Lz}, NC[3] = {P->d.nx, P->d.ny, P->d.nz};
        T *rF0 = (T *)P->rF0, *rF = (T *)P->rF, *c0 = (T *)P->c0, *c3 = (T *)P->c3, *c4 = (T *)P->c4, *e8 = (T *)P->e8;
        const T *AB = ab<T>(P), *mu = mu_of<T>(P);
        launch_transfer<double, T>(XFER_FDM_RESTRICT, P->d.p, NC, L, L, xm<T>(P, XFER_FDM_RESTRICT), r, rF0, T(1), T(0),
                                   P->ex());
        launch_transfer<double, T>(XFER_COARSE_RESTRICT, P->d.p, NC, L, P->cdim, xm<T>(P, XFER_COARSE_RESTRICT), r, c0,
                                   T(1), T(0), P->ex());
        relax_apply<T, T>(P, nullptr, z1, w, T(0), nullptr, nullptr, nullptr, rF0);   // z1 = w S r
        if (P->nc > 0) {
            launch_op_kron_restrict<T>(P->d, 2, AB, mu, z1, e8, P->ex());  // c3 = P^T (r - A z1)
            launch_coarse_gather<T>(P->d, c0, e8, c3, P->ex());
            coarse_solve<T>(P);                                             // c4 = A0^{-1} c3
            launch_transfer<T, T>(XFER_COARSE_PROLONG, P->d.p, NC, P->cdim, L, xm<T>(P, XFER_COARSE_PROLONG), c4, z1,
                                  T(1), T(1), P->ex());                     // z2 = z1 + P c4
        }
        launch_op_kron_restrict<T>(P->d, 1, AB, mu, z1, elem<T>(P), P->ex());   // rF = T^T (r - A z2)
        launch_gather_sub<T>(P->d, elem<T>(P), rF0, rF, P->ex());
        const bool dot = dot_mode >= 0;
        relax_apply<T, T>(P, nullptr, z1, w, T(1), z, dot ? r : nullptr, dot ? P->partials : nullptr, rF);
        if (dot)
            launch_finalize(transfer_blocks(XFER_FDM_PROLONG, P->d.p, NC), P->partials, P->scal, dot_mode, P->mirror,
                            P->ex());
        VSR_HIP(hipGetLastError());
        return;
    } else {
        // hybrid V(1,1): z1 = w S r; z2 = z1 + C (r - A z1); z = z2 + w S (r - A z2)
        T *res = (T *)P->res;
        relax_apply<T, double>(P, r, z1, w, T(0));
        op_residual<T>(P, r, z1, res);
        coarse_apply<T, T>(P, res, z1, T(1), T(1));
        op_residual<T>(P, r, z1, res);
        // the last prolongation also writes z in FP64 and, when asked, the partials of r.z
        const bool dot = dot_mode >= 0;
        relax_apply<T, T>(P, res, z1, w, T(1), z, dot ? r : nullptr, dot ? P->partials : nullptr);
        if (dot) {
            const int NC[3] = {P->d.nx, P->d.ny, P->d.nz};
            launch_finalize(transfer_blocks(XFER_FDM_PROLONG, P->d.p, NC), P->partials, P->scal, dot_mode, P->mirror,
                            P->ex());
        }
        VSR_HIP(hipGetLastError());
        return;
    }
    if (dot_mode >= 0) {
        const int nb = launch_axpby_to_double<T>(P->n, 1.0, z1, 0.0, z, P->ex(), r, P->partials);
        launch_finalize(nb, P->partials, P->scal, dot_mode, P->mirror, P->ex());
    } else {
        launch_axpby_to_double<T>(P->n, 1.0, z1, 0.0, z, P->ex());
    }
    VSR_HIP(hipGetLastError());
}

void precond(vsr_problem *P, const double *r, double *z, int mode, int dot_mode = -1) {
    if (P->fp32) precondition<float>(P, r, z, mode, dot_mode);
    else precondition<double>(P, r, z, mode, dot_mode);
}

double read_scalar(vsr_problem *P, int slot) {
    VSR_HIP(hipMemcpyAsync(P->host_scal, P->scal + slot, sizeof(double), hipMemcpyDeviceToHost, P->stream));
    VSR_HIP(hipStreamSynchronize(P->stream));
    return *P->host_scal;
}

void dot_into(vsr_problem *P, const double *x, const double *y, int mode) {
    launch_dot(P->n, x, y, P->partials, P->scal, mode, P->mirror, P->ex());
}

double dot(vsr_problem *P, const double *x, const double *y) {
    dot_into(P, x, y, 0);
    return read_scalar(P, SC_TMP);
}

// ---- PCG (Hestenes-Stiefel) in pieces shared by the host-driven and the batched solves.
// x = 0, r = b, RR = b.b
void pcg_init(vsr_problem *P, const double *b, double *x) {
    launch_fill<double>(P->n, x, 0.0, P->ex());
    launch_cast<double, double>(P->n, b, P->vr, P->ex());
    dot_into(P, b, b, 4);
}

// z = M r, RZ = r.z, p = z
void pcg_first_direction(vsr_problem *P) {
    precond(P, P->vr, P->vz, 0, 3);
    launch_cast<double, double>(P->n, P->vz, P->vp, P->ex());
}

// q = A p, alpha = RZ / p.q, x += alpha p, r -= alpha q, RR = r.r; rr_mode 4 leaves the
// stopping test to the host, 5 counts the update and takes the test on the device
void pcg_update(vsr_problem *P, double *x, int rr_mode) {
    const int slots = op_cells<double>(P, P->vp, P->E64);
    launch_gather<double>(P->d, slots, P->E64, nullptr, P->vq, P->ex(), P->vp, P->partials);
    launch_finalize((int)gather_blocks(P->d), P->partials, P->scal, 1, P->mirror, P->ex());
    launch_pcg_xr(P->n, x, P->vr, P->vp, P->vq, P->scal, P->partials, rr_mode, P->mirror, P->ex());
}

// z = M r, beta = r.z / RZ, RZ = r.z, p = z + beta p
void pcg_direction(vsr_problem *P) {
    precond(P, P->vr, P->vz, 0, 2);
    launch_pcg_p(P->n, P->vp, P->vz, P->scal, P->ex());
}

// ||b - A x||_2 in FP64 (ungated)
double true_residual(vsr_problem *P, const double *b, const double *x) {
    op_residual<double>(P, b, x, P->vt);
    return std::sqrt(std::max(0.0, dot(P, P->vt, P->vt)));
}

// Extreme eigenvalues of the Lanczos tridiagonal of k CG steps: step lengths alpha_0..k-1,
// direction updates beta_0..k-2 (CG-Lanczos relation; Saad, Iterative Methods for Sparse
// Linear Systems, Sec. 6.7.3).
void lanczos_extremes(const std::vector<double> &alphas, const std::vector<double> &betas, double &lo, double &hi) {
    const int k = (int)alphas.size();
    std::vector<double> dg(k), of(std::max(k - 1, 0));
    for (int j = 0; j < k; ++j) {
        dg[j] = 1.0 / alphas[j] + (j ? betas[j - 1] / alphas[j - 1] : 0.0);
        if (j + 1 < k) of[j] = std::sqrt(betas[j]) / alphas[j];
    }
    tridiag_extremes(dg, of, lo, hi);
}

// Condition estimate of the last PCG run from the (alpha, beta) record behind the device
// scalars (see SC_NA); na is the record's length read with the scalars.
void ritz_of_run(vsr_problem *P, int na, vsr_solve_info &info) {
    info.ritz_min = info.ritz_max = info.kappa_estimate = 0.0;
    if (na < 1) return;
    std::vector<double> h(2 * (size_t)na);
    VSR_HIP(hipMemcpy(h.data(), P->scal + SC_N, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<double> alphas(na), betas(na - 1);
    for (int j = 0; j < na; ++j) alphas[j] = h[2 * j];
    for (int j = 0; j + 1 < na; ++j) betas[j] = h[2 * j + 1];
    for (double a : alphas)
        if (!(a > 0) || !std::isfinite(a)) return;   // breakdown: no estimate
    lanczos_extremes(alphas, betas, info.ritz_min, info.ritz_max);
    if (info.ritz_min > 0) info.kappa_estimate = info.ritz_max / info.ritz_min;
}

// splitmix64 (Steele, Lea & Flood 2014): output i of the stream seeded with `seed`
uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// CG-Lanczos on S A (Sec. 2.5): extreme Ritz values of the Lanczos tridiagonal assembled
// from k steps of CG preconditioned by the patch relaxation.
void estimate_damping(vsr_problem *P) {
    int steps = P->opt.lanczos_steps > 0 ? P->opt.lanczos_steps : 20;
    std::vector<double> h(P->n);
    for (int64_t i = 0; i < P->n; ++i) h[i] = (double)(splitmix64_at(P->opt.seed, (uint64_t)i) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    VSR_HIP(hipMemcpy(P->vr, h.data(), P->n * sizeof(double), hipMemcpyHostToDevice));
    launch_fill<double>(P->n, P->vt, 0.0, P->ex());
    precond(P, P->vr, P->vz, 1);
    dot_into(P, P->vr, P->vz, 3);
    double rz0 = read_scalar(P, SC_RZ);
    launch_cast<double, double>(P->n, P->vz, P->vp, P->ex());
    std::vector<double> alphas, betas;
    for (int j = 0; j < steps; ++j) {
        op_apply<double>(P, P->vp, P->vq);
        dot_into(P, P->vp, P->vq, 1);
        launch_pcg_xr(P->n, P->vt, P->vr, P->vp, P->vq, P->scal, P->partials, 4, nullptr, P->ex());
        double alpha = read_scalar(P, SC_ALPHA);
        precond(P, P->vr, P->vz, 1);
        dot_into(P, P->vr, P->vz, 2);
        double beta = read_scalar(P, SC_BETA);
        double rz = read_scalar(P, SC_RZNEW);
        alphas.push_back(alpha);
        betas.push_back(beta);
        if (!(alpha > 0) || !std::isfinite(alpha)) throw Error(VSR_ENOCONV, "Lanczos breakdown");
        if (rz <= 1e-28 * rz0) break;
        launch_pcg_p(P->n, P->vp, P->vz, P->scal, P->ex());
    }
    lanczos_extremes(alphas, betas, P->lmin, P->lmax);
    const double a = 0.25;
    P->omega = 2.0 / ((1 + a) * P->lmax + (1 - a) * P->lmin);
}

// ---- autotuner: launch shapes per (GPU architecture, p, cycle precision, operator kind).
std::mutex g_tune_mutex;
std::map<std::string, Tuning> g_tune_cache;

std::string tune_key(vsr_problem *P) {
    int dev = 0;
    VSR_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    VSR_HIP(hipGetDeviceProperties(&prop, dev));
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    std::ostringstream k;
    k << arch << " p=" << P->d.p << " prec=" << (P->fp32 ? "f32" : "f64") << " op=" << (P->cartesian ? "kron" : "general");
    return k.str();
}

bool tune_from_file(const char *path, const std::string &key, Tuning &t) {
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {   // the last entry for a key wins
        if (line.compare(0, key.size(), key) != 0 || line.size() <= key.size() || line[key.size()] != ' ') continue;
        Tuning c;
        if (std::sscanf(line.c_str() + key.size(),
                        " cpw64=%d cpw32=%d patch_unroll=%d split64=%d split32=%d patch_threads=%d",
                        &c.op_cpw64, &c.op_cpw32, &c.patch_unroll, &c.opg_split64, &c.opg_split32,
                        &c.patch_threads) == 6) {
            t = c;
            found = true;
        }
    }
    return found;
}

// Mean time of `reps` back-to-back runs of fn on the problem's stream, after one warm-up run.
template <typename F>
double time_ms(vsr_problem *P, F &&fn, int reps = 5) {
    hipEvent_t a, b;
    VSR_HIP(hipEventCreate(&a));
    VSR_HIP(hipEventCreate(&b));
    fn();
    VSR_HIP(hipEventRecord(a, P->stream));
    for (int r = 0; r < reps; ++r) fn();
    VSR_HIP(hipEventRecord(b, P->stream));
    VSR_HIP(hipEventSynchronize(b));
    float ms = 0;
    VSR_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

// Coordinate search over each shape with the others fixed; every candidate produces the
// same values, so only time decides.
void autotune(vsr_problem *P) {
    const std::string key = tune_key(P);
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            P->tune = it->second;
            return;
        }
    }
    Tuning t;
    if (tune_from_file(P->opt.tune_cache, key, t)) {
        P->tune = t;
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        g_tune_cache[key] = t;
        return;
    }
    P->tune = Tuning{};
    launch_fill<double>(P->n, P->vp, 1.0, P->ex());
    auto pick = [&](int &field, std::initializer_list<int> cands, auto &&fn) {
        double best = 1e300;
        int arg = field;
        for (int c : cands) {
            field = c;
            double ms = time_ms(P, fn);
            if (ms < best) { best = ms; arg = c; }
        }
        field = arg;
    };
    const bool small = (P->d.p + 1) * (P->d.p + 1) <= 64;
    if (P->cartesian && small) {
        pick(P->tune.op_cpw64, {1, 2, 4}, [&] { op_apply<double>(P, P->vp, P->vq); });
        if (P->fp32) {
            launch_cast<double, float>(P->n, P->vp, (float *)P->z1, P->ex());
            pick(P->tune.op_cpw32, {1, 2, 4}, [&] { op_apply<float>(P, (const float *)P->z1, (float *)P->res); });
        }
    }
    if (!P->cartesian) {
        pick(P->tune.opg_split64, {1, 2}, [&] { op_apply<double>(P, P->vp, P->vq); });
        if (P->fp32) {
            launch_cast<double, float>(P->n, P->vp, (float *)P->z1, P->ex());
            pick(P->tune.opg_split32, {1, 2}, [&] { op_apply<float>(P, (const float *)P->z1, (float *)P->res); });
        }
    }
    // patch solves: loads in flight per thread jointly with the workgroup size
    auto pick_patch = [&](auto &&fn) {
        double best = 1e300;
        Tuning keep = P->tune;
        for (int nth : {256, 512, 1024})
            for (int u : {4, 8, 16}) {
                if (nth == 1024 && u == 16) continue;   // 128 VGPRs at 1024 threads
                P->tune.patch_threads = nth;
                P->tune.patch_unroll = u;
                double ms = time_ms(P, fn);
                if (ms < best) {
                    best = ms;
                    keep = P->tune;
                }
            }
        P->tune = keep;
    };
    auto patch = [&](auto zero) {
        using T = decltype(zero);
        launch_patch_all<T>(P->d, P->pa, P->n_int, P->verts, P->fidx, (const T *)P->fint, P->n_bnd, P->bdesc, P->boff,
                            (const T *)P->fbnd, (const T *)P->mu_sur, (const T *)P->lam, (const T *)P->afc,
                            (const T *)P->rF, (T *)P->U, P->ex());
    };
    if (P->fp32) {
        launch_fill<float>(P->n, (float *)P->rF, 1.f, P->ex());
        if (P->n_int + P->n_bnd > 0) pick_patch([&] { patch(0.f); });
    } else {
        launch_fill<double>(P->n, (double *)P->rF, 1.0, P->ex());
        if (P->n_int + P->n_bnd > 0) pick_patch([&] { patch(0.0); });
    }
    // nodes that no star of a parity class covers must read as zero in the assembly
    if (P->fp32) launch_fill<float>(patch_solution_entries(P->d), (float *)P->U, 0.f, P->ex());
    else launch_fill<double>(patch_solution_entries(P->d), (double *)P->U, 0.0, P->ex());
    VSR_HIP(hipStreamSynchronize(P->stream));
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    g_tune_cache[key] = P->tune;
    if (P->opt.tune_cache) {
        std::ofstream f(P->opt.tune_cache, std::ios::app);
        f << key << " cpw64=" << P->tune.op_cpw64 << " cpw32=" << P->tune.op_cpw32
          << " patch_unroll=" << P->tune.patch_unroll << " split64=" << P->tune.opg_split64
          << " split32=" << P->tune.opg_split32 << " patch_threads=" << P->tune.patch_threads << "\n";
    }
}

template <typename T>
void upload_patch_data(vsr_problem *P, const PatchSet &S, const std::vector<double> &mu_sur) {
    P->mu_sur = P->upload_as<T>(mu_sur);
    P->lam = P->upload_as<T>(P->od.lam);
    int p = P->d.p, m = p - 1;
    std::vector<double> afc(2 * m);
    for (int t = 1; t <= m; ++t) {
        afc[t - 1] = P->od.Af[(size_t)t * (p + 1) + p];
        afc[m + t - 1] = P->od.Af[(size_t)t * (p + 1) + 0];
    }
    P->afc = P->upload_as<T>(afc);
    P->fint = P->upload_as<T>(S.interior_factor);
    P->fbnd = P->upload_as<T>(S.boundary_factor);
    P->mu_len = (int64_t)mu_sur.size();
    P->fint_len = (int64_t)S.interior_factor.size();
    P->fbnd_len = (int64_t)S.boundary_factor.size();
}

}  // namespace

// Batched solves: members, the streams they are spread over and the recorded iteration.
struct vsr_batch {
    std::vector<vsr_problem *> members;
    std::vector<int> stream_of;            // member -> index into streams
    std::vector<hipStream_t> streams;
    hipStream_t origin = nullptr;          // fork/join point and graph launch stream
    std::vector<hipEvent_t> events;        // [0] fork, [1 + j] join of stream j
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double *host_done = nullptr;           // pinned and mapped: each member's stop flag, written by its kernels
    double *dev_done = nullptr;            // the same memory as the device sees it
    hipEvent_t poll[2] = {nullptr, nullptr};
    bool eager = false;
    bool owns_members = true;
    std::vector<uint64_t> recorded_tune;   // each member's tune_version when the graph was recorded

    ~vsr_batch();
    void solve(const double *const *b_dev, double *const *x_dev, double rtol, vsr_solve_info *infos);

    // Run fn(member) for every member on its stream, forked from and joined back to origin.
    template <typename F>
    void for_members(F &&fn) {
        VSR_HIP(hipEventRecord(events[0], origin));
        for (hipStream_t st : streams) VSR_HIP(hipStreamWaitEvent(st, events[0], 0));
        for (size_t i = 0; i < members.size(); ++i) {
            vsr_problem *P = members[i];
            hipStream_t keep = P->stream;
            P->stream = streams[stream_of[i]];
            try {
                fn(P);
            } catch (...) {
                P->stream = keep;
                P->gate = nullptr;
                P->mirror = nullptr;
                throw;
            }
            P->stream = keep;
        }
        for (size_t j = 0; j < streams.size(); ++j) {
            VSR_HIP(hipEventRecord(events[1 + j], streams[j]));
            VSR_HIP(hipStreamWaitEvent(origin, events[1 + j], 0));
        }
    }

    // One lockstep PCG iteration of every member, each gated by its own stop flag (mirrored to
    // host memory as it changes).
    void iteration() {
        int i = 0;
        for_members([&](vsr_problem *P) {
            P->gate = P->scal + SC_DONE;
            P->mirror = dev_done + i++;
            pcg_update(P, P->vx, 5);
            pcg_direction(P);
            P->gate = nullptr;
            P->mirror = nullptr;
        });
    }
    bool all_done() const {
        const volatile double *f = host_done;
        for (size_t i = 0; i < members.size(); ++i)
            if (f[i] == 0.0) return false;
        return true;
    }
};

namespace {

void destroy_problem(vsr_problem *P) {
    if (!P) return;
    destroy_problem(P->twin);
    delete P->self;
    delete P;
}

// Streams, events, graph state and device scalars of a batch over `members`.
vsr_batch *make_batch(int count, vsr_problem *const *members, int nstreams, bool eager, bool owns) {
    auto B = std::make_unique<vsr_batch>();
    B->owns_members = false;   // until everything below has succeeded
    const int ns = std::max(1, std::min(nstreams, count));
    B->streams.resize(ns, nullptr);
    for (auto &st : B->streams) VSR_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    VSR_HIP(hipStreamCreateWithFlags(&B->origin, hipStreamNonBlocking));
    B->events.resize(1 + ns, nullptr);
    for (auto &e : B->events) VSR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto &e : B->poll) VSR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // largest member first onto the least loaded stream
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return members[a]->n > members[b]->n; });
    std::vector<double> load(ns, 0.0);
    B->stream_of.assign(count, 0);
    for (int i : order) {
        int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        B->stream_of[i] = j;
        load[j] += (double)members[i]->n;
    }
    VSR_HIP(hipHostMalloc((void **)&B->host_done, sizeof(double) * count, hipHostMallocMapped | hipHostMallocCoherent));
    VSR_HIP(hipHostGetDevicePointer((void **)&B->dev_done, B->host_done, 0));
    for (int i = 0; i < count; ++i) B->host_done[i] = 1.0;
    B->eager = eager;
    B->members.assign(members, members + count);
    B->owns_members = owns;
    return B.release();
}

}  // namespace

vsr_batch::~vsr_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (hipEvent_t e : poll)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t st : streams) (void)hipStreamDestroy(st);
    if (origin) (void)hipStreamDestroy(origin);
    if (host_done) (void)hipHostFree(host_done);
    if (owns_members)
        for (vsr_problem *m : members) destroy_problem(m);
}

// Stagnation test window of a device-driven PCG on P (FP32 relaxation only; 0: no test).
int stagnation_window(const vsr_problem *P) {
    if (!P->fp32 || P->opt.stagnation_window < 0) return 0;
    return P->opt.stagnation_window > 0 ? P->opt.stagnation_window : 10;
}

// The FP64-relaxation setup of an FP32 problem, from the inputs kept at its setup.
vsr_problem *make_fp64_twin(vsr_problem *P) {
    if (P->in_vertices.empty()) throw Error(VSR_EINVAL, "no setup inputs kept for a stagnation restart");
    vsr_mesh m{P->in_nx, P->in_ny, P->in_nz, P->in_vertices.data()};
    vsr_coefficients c{P->in_kappa.empty() ? nullptr : P->in_kappa.data(),
                       P->in_mu.empty() ? nullptr : P->in_mu.data()};
    vsr_options o = P->opt;
    o.relax_fp32 = 0;
    vsr_problem *Q = nullptr;
    if (vsr_setup(&m, P->d.p, &c, &o, &Q) != VSR_OK)
        throw Error(VSR_ENOMEM, std::string("FP64 setup for the stagnation restart failed: ") + g_last_error_text);
    try {
        Q->ve = Q->dalloc<double>(Q->n);
        Q->self = make_batch(1, &Q, 1, Q->opt.batch_eager != 0, false);
    } catch (...) {
        destroy_problem(Q);
        throw;
    }
    return Q;
}

struct Continued {
    int iterations = 0;
    bool converged = false;
    double rel_residual = 0;   // recursive residual of the continuation over ||b||_2
};

// A stagnated FP32-relaxation solve continued from its x with the FP64 relaxation: PCG on
// A e = r, r = b - A x, to the tolerance rtol ||b||_2 / ||r||_2, then x += e.
Continued continue_fp64(vsr_problem *P, const double *b, double *x, double rtol, double bb) {
    if (!P->twin) P->twin = make_fp64_twin(P);
    vsr_problem *Q = P->twin;
    op_residual<double>(P, b, x, P->vt);
    const double rn = std::sqrt(std::max(0.0, dot(P, P->vt, P->vt)));   // synchronizes P's stream
    const double bn = std::sqrt(bb);
    Continued c;
    c.rel_residual = rn / bn;
    if (rn <= rtol * bn) {
        c.converged = true;
        return c;
    }
    const double *bv[1] = {P->vt};
    double *xv[1] = {Q->ve};
    vsr_solve_info qi{};
    try {
        Q->self->solve(bv, xv, rtol * bn / rn, &qi);
    } catch (const Error &e) {
        if (e.status != VSR_ENOCONV) throw;
    }
    launch_axpby_to_double<double>(P->n, 1.0, Q->ve, 1.0, x, P->ex());
    c.iterations = qi.iterations;
    c.converged = qi.converged != 0;
    c.rel_residual = qi.rel_residual * rn / bn;
    return c;
}

// Lockstep PCG of every member (see vsr_pcg_solve_batch).  The graph of one iteration is
// recorded at the first solve and replayed; the active count is polled one replay behind,
// so the GPU always has the next iteration queued (a replay after the last member stops
// runs gated, doing nothing).
void vsr_batch::solve(const double *const *b_dev, double *const *x_dev, double rtol, vsr_solve_info *infos) {
    const int count = (int)members.size();
    for (vsr_problem *P : members) VSR_HIP(hipStreamSynchronize(P->stream));
    double t0 = now_s();
    int maxit = 0;
    for (vsr_problem *P : members) maxit = std::max(maxit, P->opt.max_iterations > 0 ? P->opt.max_iterations : 1000);
    {
        int i = 0;
        for_members([&](vsr_problem *P) {
            pcg_init(P, b_dev[i], P->vx);
            launch_pcg_start(P->scal, rtol, P->opt.max_iterations > 0 ? P->opt.max_iterations : 1000,
                             stagnation_window(P), P->opt.stagnation_factor > 0 ? P->opt.stagnation_factor : 1.0,
                             dev_done + i, P->ex());
            P->gate = P->scal + SC_DONE;
            pcg_first_direction(P);
            P->gate = nullptr;
            ++i;
        });
    }
    if (exec) {   // a member retuned since the recording: the graph holds its old launch shapes
        bool stale = recorded_tune.size() != members.size();
        for (size_t k = 0; k < members.size() && !stale; ++k) stale = recorded_tune[k] != members[k]->tune_version;
        if (stale) {
            VSR_HIP(hipGraphExecDestroy(exec));
            VSR_HIP(hipGraphDestroy(graph));
            exec = nullptr;
            graph = nullptr;
        }
    }
    if (!eager && !exec) {
        recorded_tune.clear();
        for (vsr_problem *P : members) recorded_tune.push_back(P->tune_version);
        for (vsr_problem *P : members) P->capturing = true;
        VSR_HIP(hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal));
        try {
            iteration();
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(origin, &g);
            if (g) (void)hipGraphDestroy(g);
            for (vsr_problem *P : members) P->capturing = false;
            throw;
        }
        VSR_HIP(hipStreamEndCapture(origin, &graph));
        for (vsr_problem *P : members) P->capturing = false;
        VSR_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    int replays = 0;
    for (;;) {
        if (eager) iteration();
        else VSR_HIP(hipGraphLaunch(exec, origin));
        VSR_HIP(hipEventRecord(poll[replays & 1], origin));
        ++replays;
        if (replays >= 2) {   // wait for the replay before the one just queued, then read the flags
            VSR_HIP(hipEventSynchronize(poll[(replays - 2) & 1]));
            if (all_done()) break;
        }
        if (replays > maxit + 1) break;
    }
    VSR_HIP(hipStreamSynchronize(origin));
    double t1 = now_s();
    bool all = true, bad_rhs = false;
    std::string failed;
    for (int i = 0; i < count; ++i) {
        vsr_problem *P = members[i];
        launch_cast<double, double>(P->n, P->vx, x_dev[i], P->ex());
        VSR_HIP(hipMemcpyAsync(P->host_scal, P->scal, sizeof(double) * SC_N, hipMemcpyDeviceToHost, P->stream));
        VSR_HIP(hipStreamSynchronize(P->stream));
        const double it = P->host_scal[SC_IT];
        double status = P->host_scal[SC_STATUS];
        const double bb = P->host_scal[SC_BB], rr = P->host_scal[SC_RR];
        const int na = it > 0 ? (int)P->host_scal[SC_NA] : 0;
        vsr_solve_info loc{};
        loc.iterations = (int32_t)it;
        loc.rel_residual = bb > 0 ? std::sqrt(rr / bb) : 0.0;
        loc.solve_seconds = t1 - t0;
        if (status == 4.0) {   // stagnated: continue on the FP64 relaxation
            const double tc = now_s();
            Continued c = continue_fp64(P, b_dev[i], x_dev[i], rtol, bb);
            loc.iterations += c.iterations;
            loc.fp64_iterations = c.iterations;
            loc.rel_residual = c.rel_residual;
            loc.solve_seconds += now_s() - tc;
            status = c.converged ? 1.0 : 3.0;
        }
        const double tr = true_residual(P, b_dev[i], x_dev[i]);
        loc.converged = status == 1.0 ? 1 : 0;
        loc.true_rel_residual = bb > 0 ? tr / std::sqrt(bb) : 0.0;
        loc.omega = P->omega;
        loc.lambda_min = P->lmin;
        loc.lambda_max = P->lmax;
        loc.setup_seconds = P->setup_seconds;
        ritz_of_run(P, na, loc);
        if (infos) infos[i] = loc;
        if (status == 2.0 && bb - bb != 0.0) bad_rhs = true;
        if (status != 1.0) {
            all = false;
            failed += (failed.empty() ? "" : ", ") + std::to_string(i);
        }
    }
    if (bad_rhs) throw Error(VSR_EINVAL, "non-finite right-hand side");
    if (!all) {
        if (count == 1) throw Error(VSR_ENOCONV, "PCG did not converge in " + std::to_string(infos ? infos[0].iterations :
                                                   (int)members[0]->host_scal[SC_IT]) + " iterations");
        throw Error(VSR_ENOCONV, "batched PCG: members not converged: " + failed);
    }
}

// ---- primal linear elasticity with the SDC relaxation (Sec. 3.1) ----------------------------
// The SDC preconditioner is block-Jacobi over the displacement components; on box cells each
// diagonal block A_jj is the scalar separable operator with per-axis coefficients
// (mu + (mu + lam) [a = j]) times the Poisson scalings, so component j's relaxation is the
// scalar vertex-star FDM relaxation of a scalar problem set up with those scalings.
struct vsr_elasticity {
    vsr_problem *comp[3] = {nullptr, nullptr, nullptr};   // per component: its SDC relaxation
    Dims d{};
    int64_t n = 0;       // free nodes per component (the vector has 3 n entries)
    int64_t ncell = 0;
    int nc = 0;          // interior vertices per component (coarse space)
    double mu = 0, lam = 0;
    double omega = 1, lmin = 0, lmax = 0, setup_seconds = 0;
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr;                  // joins the solve's own stream to the caller's and back
    hipEvent_t it_ev[2] = {nullptr, nullptr};   // end of the last two iterations
    hipStream_t origin = nullptr;               // the solve's own stream (graph capture needs one)
    hipGraph_t graph = nullptr;                 // one PCG iteration, recorded for the output vector graph_x
    hipGraphExec_t exec = nullptr;
    const double *graph_x = nullptr;
    const double *gate = nullptr;               // during a solve: the stop flag every launch checks
    double *host_done = nullptr, *dev_done = nullptr;   // mapped host copy of the stop flag
    std::vector<void *> allocs;
    double *M1 = nullptr, *coef = nullptr, *E = nullptr, *A0inv = nullptr;
    double *vr = nullptr, *vz = nullptr, *vp = nullptr, *vq = nullptr, *vt = nullptr;
    // the V-cycle in its precision (FP32 with relax_fp32, else FP64): 1-D matrices, cell
    // coefficients and coarse inverse in that precision (FP32 copies; the FP64 ones otherwise),
    // the cycle's iterate z1 and residual t (3 n each), the coarse vectors (3 nc each)
    bool fp32 = false;
    CompStrides cs{};   // the components' patch arrays lie one after another (see the setup)
    float *M1f = nullptr, *coeff = nullptr, *A0f = nullptr;
    void *cz = nullptr, *ct = nullptr, *cc0 = nullptr, *cc1 = nullptr;
    Exec ex() const { return Exec{stream, gate, Tuning{}}; }
    template <typename T>
    T *dalloc(size_t count) {
        void *p = nullptr;
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (hipMalloc(&p, bytes) != hipSuccess) throw Error(VSR_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        allocs.push_back(p);
        return static_cast<T *>(p);
    }
    ~vsr_elasticity() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (origin) (void)hipStreamSynchronize(origin);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (vsr_problem *c : comp) destroy_problem(c);
        for (void *p : allocs) (void)hipFree(p);
        if (origin) (void)hipStreamDestroy(origin);
        if (host_done) (void)hipHostFree(host_done);
        for (hipEvent_t e : it_ev)
            if (e) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
    }
};

namespace {

// y = A x for the 3-component vector (x, y: 3 n, component after component), FP64
void el_op(vsr_elasticity *L, const double *x, double *y) {
    launch_op_elastic_box<double>(L->d, L->M1, L->coef, L->mu, L->lam, x, L->E, L->ex());
    launch_gather_components<double>(L->d, 3, L->E, y, L->ex());
}

double el_dot(vsr_elasticity *L, const double *x, const double *y) {
    vsr_problem *P = L->comp[0];
    launch_dot(3 * L->n, x, y, P->partials, P->scal, 0, nullptr, L->ex());
    return read_scalar(P, SC_TMP);
}

template <typename T> const T *el_m1(const vsr_elasticity *L);
template <> const double *el_m1<double>(const vsr_elasticity *L) { return L->M1; }
template <> const float *el_m1<float>(const vsr_elasticity *L) { return L->M1f; }
template <typename T> const T *el_coef(const vsr_elasticity *L);
template <> const double *el_coef<double>(const vsr_elasticity *L) { return L->coef; }
template <> const float *el_coef<float>(const vsr_elasticity *L) { return L->coeff; }
template <typename T> const T *el_a0(const vsr_elasticity *L);
template <> const double *el_a0<double>(const vsr_elasticity *L) { return L->A0inv; }
template <> const float *el_a0<float>(const vsr_elasticity *L) { return L->A0f; }

// t = r - A z in the cycle's precision T (r in FP64); the element vector E holds T values here
template <typename T>
void el_residual(vsr_elasticity *L, const double *r, const T *z, T *t) {
    T *E = (T *)L->E;
    launch_op_elastic_box<T>(L->d, el_m1<T>(L), el_coef<T>(L), (T)L->mu, (T)L->lam, z, E, L->ex());
    launch_gather_components<T>(L->d, 3, E, t, L->ex(), r);
}

// out_c = alpha S_c in_c + beta out_c for the three components (with out64: also written in
// FP64): component c's scalar FDM vertex-star relaxation in its working precision T.  The
// components' patch data lie one after another, so each phase (the FDM restriction, the patch
// solves, the scatter-add and prolongation) is one launch over all three.
template <typename T, typename Tin>
void el_relax(vsr_elasticity *L, const Tin *in, T *out, T alpha, T beta, double *out64) {
    vsr_problem *P = L->comp[0];
    const int Ld[3] = {P->d.Lx, P->d.Ly, P->d.Lz}, NC[3] = {P->d.nx, P->d.ny, P->d.nz};
    const Exec e{L->stream, L->gate, P->tune};
    launch_transfer<Tin, T>(XFER_FDM_RESTRICT, P->d.p, NC, Ld, Ld, xm<T>(P, XFER_FDM_RESTRICT), in, (T *)P->rF, T(1),
                            T(0), e, nullptr, nullptr, nullptr, 0, 3);
    launch_patch_all<T>(P->d, P->pa, P->n_int, P->verts, P->fidx, (const T *)P->fint, P->n_bnd, P->bdesc, P->boff,
                        (const T *)P->fbnd, (const T *)P->mu_sur, (const T *)P->lam, (const T *)P->afc, (const T *)P->rF,
                        (T *)P->U, e, 3, L->cs);
    if (P->d.p <= kFusedScatterMaxP) {
        launch_transfer<T, T>(XFER_FDM_PROLONG, P->d.p, NC, Ld, Ld, xm<T>(P, XFER_FDM_PROLONG), (const T *)P->U, out, alpha,
                              beta, e, out64, nullptr, nullptr, P->opt.interior_patches_only ? 2 : 1, 3);
    } else {
        launch_patch_assemble<T>(P->d, (const T *)P->U, (T *)P->zF, e, 3);
        launch_transfer<T, T>(XFER_FDM_PROLONG, P->d.p, NC, Ld, Ld, xm<T>(P, XFER_FDM_PROLONG), (const T *)P->zF, out, alpha,
                              beta, e, out64, nullptr, nullptr, 0, 3);
    }
    VSR_HIP(hipGetLastError());
}

// out = alpha P A0^{-1} P^T in + beta out with Q1 in every component (with out64: also in
// FP64); the three restrictions and the three prolongations are one launch each
template <typename T, typename Tin>
void el_coarse(vsr_elasticity *L, const Tin *in, T *out, T alpha, T beta, double *out64) {
    if (L->nc == 0) {
        if (beta == T(0)) launch_fill<T>(3 * L->n, out, T(0), L->ex());
        if (out64) launch_axpby_to_double<T>(3 * L->n, 1.0, out, 0.0, out64, L->ex());
        return;
    }
    vsr_problem *P = L->comp[0];
    const int Ld[3] = {L->d.Lx, L->d.Ly, L->d.Lz}, NC[3] = {L->d.nx, L->d.ny, L->d.nz};
    T *c0 = (T *)L->cc0, *c1 = (T *)L->cc1;
    launch_transfer<Tin, T>(XFER_COARSE_RESTRICT, L->d.p, NC, Ld, P->cdim, xm<T>(P, XFER_COARSE_RESTRICT), in, c0, T(1),
                            T(0), L->ex(), nullptr, nullptr, nullptr, 0, 3);
    launch_dense_gemv<T>(3 * L->nc, el_a0<T>(L), c0, c1, T(1), T(0), L->ex());
    launch_transfer<T, T>(XFER_COARSE_PROLONG, L->d.p, NC, P->cdim, Ld, xm<T>(P, XFER_COARSE_PROLONG), c1, out, alpha,
                          beta, L->ex(), out64, nullptr, nullptr, 0, 3);
}

// z = M r in the cycle's precision T.  mode 0: the hybrid V(1,1) z1 = w S r,
// z2 = z1 + C (r - A z1), z = z2 + w S (r - A z2); mode 1: S r; mode 2: C r.
template <typename T>
void el_precond_t(vsr_elasticity *L, const double *r, double *z, int mode) {
    T *z1 = (T *)L->cz, *t = (T *)L->ct;
    const T w = (T)L->omega;
    if (mode == 1) return el_relax<T, double>(L, r, z1, T(1), T(0), z);
    if (mode == 2) return el_coarse<T, double>(L, r, z1, T(1), T(0), z);
    el_relax<T, double>(L, r, z1, w, T(0), nullptr);        // z1 = w S r
    el_residual<T>(L, r, z1, t);                            // t = r - A z1
    el_coarse<T, T>(L, t, z1, T(1), T(1), nullptr);         // z2 = z1 + C t
    el_residual<T>(L, r, z1, t);                            // t = r - A z2
    el_relax<T, T>(L, t, z1, w, T(1), z);                   // z = z2 + w S t
}

void el_precond(vsr_elasticity *L, const double *r, double *z, int mode) {
    if (L->fp32) el_precond_t<float>(L, r, z, mode);
    else el_precond_t<double>(L, r, z, mode);
}

// CG-Lanczos on S A from the splitmix64 start vector (the scalar estimate's recipe, 3 n entries)
void el_damping(vsr_elasticity *L, int steps, uint64_t seed) {
    const int64_t N = 3 * L->n;
    std::vector<double> h(N);
    for (int64_t i = 0; i < N; ++i) h[i] = (double)(splitmix64_at(seed, (uint64_t)i) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    VSR_HIP(hipMemcpy(L->vr, h.data(), N * sizeof(double), hipMemcpyHostToDevice));
    el_precond(L, L->vr, L->vz, 1);
    double rz = el_dot(L, L->vr, L->vz);
    const double rz0 = rz;
    launch_axpby_to_double<double>(N, 1.0, L->vz, 0.0, L->vp, L->ex());
    std::vector<double> alphas, betas;
    for (int j = 0; j < steps; ++j) {
        el_op(L, L->vp, L->vq);
        const double alpha = rz / el_dot(L, L->vp, L->vq);
        if (!(alpha > 0) || !std::isfinite(alpha)) throw Error(VSR_ENOCONV, "Lanczos breakdown");
        launch_axpby_to_double<double>(N, -alpha, L->vq, 1.0, L->vr, L->ex());
        el_precond(L, L->vr, L->vz, 1);
        const double rzn = el_dot(L, L->vr, L->vz);
        alphas.push_back(alpha);
        betas.push_back(rzn / rz);
        if (rzn <= 1e-28 * rz0) break;
        launch_axpby_to_double<double>(N, 1.0, L->vz, betas.back(), L->vp, L->ex());
        rz = rzn;
    }
    lanczos_extremes(alphas, betas, L->lmin, L->lmax);
    L->omega = 2.0 / ((1 + 0.25) * L->lmax + (1 - 0.25) * L->lmin);
}

}  // namespace

extern "C" {

void vsr_default_options(vsr_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->lanczos_steps = 20;
    opt->max_iterations = 1000;
}

vsr_status vsr_setup(const vsr_mesh *mesh, int32_t p, const vsr_coefficients *coef, const vsr_options *opt,
                     vsr_problem **out) {
    return guarded([&] {
        if (!mesh || !out || !mesh->vertices) throw Error(VSR_EINVAL, "NULL argument");
        *out = nullptr;
        if (p < 2 || p > 15) throw Error(VSR_EINVAL, "p must be in [2, 15]");
        if (mesh->nx < 2 || mesh->ny < 2 || mesh->nz < 2) throw Error(VSR_EINVAL, "every mesh axis needs at least 2 cells");
        double t0 = now_s();
        auto P = std::make_unique<vsr_problem>();
        if (opt) P->opt = *opt;
        else vsr_default_options(&P->opt);
        int qdef = (3 * (p + 1) + 1) / 2;
        if (P->opt.quad_points != 0 && P->opt.quad_points != qdef)
            throw Error(VSR_EINVAL, "quad_points must be 0 or ceil(3(p+1)/2)");
        if (P->opt.cycle != 0 && P->opt.cycle != 1) throw Error(VSR_EINVAL, "cycle must be 0 or 1");
        P->stream = (hipStream_t)P->opt.stream;
        P->fp32 = P->opt.relax_fp32 != 0;
        int nx = mesh->nx, ny = mesh->ny, nz = mesh->nz;
        P->d = Dims{nx, ny, nz, p, qdef, p * nx - 1, p * ny - 1, p * nz - 1};
        P->n = (int64_t)P->d.Lx * P->d.Ly * P->d.Lz;
        P->ncell = (int64_t)nx * ny * nz;
        int64_t nv = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
        for (int64_t i = 0; i < 3 * nv; ++i)
            if (!std::isfinite(mesh->vertices[i])) throw Error(VSR_EINVAL, "non-finite vertex coordinate");
        const double *kappa = coef ? coef->kappa : nullptr;
        const double *muo = coef ? coef->mu_override : nullptr;
        if (kappa)
            for (int64_t e = 0; e < P->ncell; ++e)
                if (!std::isfinite(kappa[e])) throw Error(VSR_EINVAL, "non-finite kappa");
        if (muo)
            for (int64_t e = 0; e < 3 * P->ncell; ++e)
                if (!std::isfinite(muo[e])) throw Error(VSR_EINVAL, "non-finite mu_override");
        if (!(P->opt.stagnation_factor >= 0 && P->opt.stagnation_factor <= 1))
            throw Error(VSR_EINVAL, "stagnation_factor must be in [0, 1]");
        if (P->fp32 && P->opt.stagnation_window >= 0) {
            P->in_nx = nx;
            P->in_ny = ny;
            P->in_nz = nz;
            P->in_vertices.assign(mesh->vertices, mesh->vertices + 3 * nv);
            if (kappa) P->in_kappa.assign(kappa, kappa + P->ncell);
            if (muo) P->in_mu.assign(muo, muo + 3 * P->ncell);
        }
        // 1D data and geometry
        P->od = make_1d(p, qdef);
        Geometry g = make_geometry(nx, ny, nz, mesh->vertices, kappa, P->od, false);
        P->cartesian = g.cartesian;
        if (kappa)
            for (int64_t e = 0; e < P->ncell; ++e)
                if (!(kappa[e] > 0)) throw Error(VSR_ENOTSPD, "kappa must be positive");
        int n1 = p + 1;
        // [A, B, That, linear hats at the GLL nodes] for the Cartesian operator and its restrictions
        std::vector<double> ab(3 * n1 * n1 + 2 * n1), idq(2 * (size_t)qdef * n1 + 2 * (size_t)qdef);
        std::copy(P->od.A.begin(), P->od.A.end(), ab.begin());
        std::copy(P->od.B.begin(), P->od.B.end(), ab.begin() + n1 * n1);
        std::copy(P->od.T.begin(), P->od.T.end(), ab.begin() + 2 * n1 * n1);
        for (int k = 0; k < n1; ++k) {
            ab[3 * n1 * n1 + k] = 0.5 * (1.0 - P->od.xi[k]);
            ab[3 * n1 * n1 + n1 + k] = 0.5 * (1.0 + P->od.xi[k]);
        }
        std::copy(P->od.Iq.begin(), P->od.Iq.end(), idq.begin());
        std::copy(P->od.Dq.begin(), P->od.Dq.end(), idq.begin() + (size_t)qdef * n1);
        std::copy(P->od.xq.begin(), P->od.xq.end(), idq.begin() + 2 * (size_t)qdef * n1);
        std::copy(P->od.wq.begin(), P->od.wq.end(), idq.begin() + 2 * (size_t)qdef * n1 + qdef);
        P->AB64 = P->upload(ab);
        P->AB32 = P->upload_as<float>(ab);
        P->IDq64 = P->upload(idq);
        P->IDq32 = P->upload_as<float>(idq);
        P->mu64 = P->upload(g.mu);
        P->mu32 = P->upload_as<float>(g.mu);
        P->wdet = P->upload(g.wdet);
        if (!g.cartesian) {
            // the operator evaluates the metric from these per-cell corner data (the host's
            // metric stays on the host for the coarse matrices)
            const std::vector<double> cg = make_cell_geometry(nx, ny, nz, mesh->vertices, kappa);
            P->geo64 = P->upload(cg);
            if (P->fp32) P->geo32 = P->upload_as<float>(cg);
        }
        // patches (separable surrogate, Sec. 2.7)
        std::vector<double> mu_sur = muo ? std::vector<double>(muo, muo + 3 * P->ncell) : g.mu;
        for (double v : mu_sur)
            if (!(v > 0)) throw Error(VSR_ENOTSPD, "surrogate scalings must be positive");
        PatchSet S = make_patches(nx, ny, nz, P->od, mu_sur.data(), P->opt.interior_patches_only != 0,
                                  P->opt.share_factors != 0);
        P->n_int = (int)(S.interior_vertices.size() / 3);
        P->n_bnd = (int)S.boundary_off.size();
        P->verts = P->upload(S.interior_vertices);
        P->fidx = P->upload(S.interior_factor_of);
        P->bdesc = P->upload(S.boundary_desc);
        P->boff = P->upload(S.boundary_off);
        const InteriorLayout &L = S.L;
        PatchArgs &a = P->pa;
        a.m = L.m; a.w = L.w; a.n_leaf = L.n_leaf; a.n_sep = L.n_sep; a.n_top = L.n_top; a.n_iface = L.n_iface;
        a.top_pad = L.top_pad; a.ntiles = L.ntiles;
        a.off_invd = L.off_invd; a.off_B1 = L.off_B1; a.off_B2 = L.off_B2; a.off_Lsep = L.off_Lsep; a.off_Sy = L.off_Sy;
        a.off_Ltop = L.off_Ltop; a.stride = L.stride;
        a.det = P->opt.deterministic != 0;
        int m = L.m, w = L.w;
        // stored entries of one interior factor: leaves, B1 and B2, level-1 slice inverses, the
        // y-diagonal top x separator block, the top plane's inverse Schur complement
        const int64_t top_entries = (int64_t)L.n_top * (L.n_top + 1) / 2;
        int64_t per_patch = (int64_t)L.n_leaf + 2LL * 4 * m * m * w + 2LL * m * w * (w + 1) / 2 +
                            2LL * m * w * w + top_entries;
        int64_t bnd_nnz = 0, bnd_box = 0;
        for (int i = 0; i < P->n_bnd; ++i) {
            int ns = S.boundary_desc[8 * i + 7], nsl = S.boundary_desc[8 * i + 6];
            bnd_nnz += (int64_t)nsl * ns * (ns + 1) / 2;
            int64_t box = 1;   // the part of the star's box inside existing cells
            for (int a = 0; a < 3; ++a) box *= S.boundary_desc[8 * i + 3 + a] == AX_FULL ? w : m;
            bnd_box += box;
        }
        P->factor_entries = per_patch * S.n_interior_factors + S.boundary_entries;   // stored entries
        (void)bnd_nnz;
        size_t esz = P->fp32 ? sizeof(float) : sizeof(double);
        // one launch solves every patch: factors read twice (forward, backward) except the top
        // plane's inverse (read once), box in and out
        P->bytes_patch_launch =
            (double)esz * ((double)P->n_int * (2.0 * (double)(per_patch - top_entries) + (double)top_entries +
                                               2.0 * (double)w * w * w) +
                           2.0 * (double)bnd_nnz + 2.0 * (double)bnd_box);
        if (P->fp32) upload_patch_data<float>(P.get(), S, mu_sur);
        else upload_patch_data<double>(P.get(), S, mu_sur);
        // lattice transfers: the cell blocks of T^T, T, P^T, P
        const int nc3[3] = {nx, ny, nz};
        for (int ax = 0; ax < 3; ++ax) P->cdim[ax] = nc3[ax] - 1;
        for (int k = 0; k < 4; ++k) {
            const std::vector<double> M = transfer_block(k, P->od);
            P->xm64[k] = P->upload(M);
            P->xm32[k] = P->upload_as<float>(M);
        }
        // coarse space: dense inverse of the Q1 matrix, or its multigrid hierarchy (Sec. 2.8)
        P->nc = P->cdim[0] * P->cdim[1] * P->cdim[2];
        if (P->opt.coarse_solver < 0 || P->opt.coarse_solver > 2)
            throw Error(VSR_EINVAL, "coarse_solver must be 0 (automatic), 1 (dense) or 2 (multigrid)");
        P->coarse_gmg = P->opt.coarse_solver == 2 || (P->opt.coarse_solver == 0 && P->nc > kAutoDenseCoarse);
        MGHierarchyHost H;
        if (P->coarse_gmg) {
            H = make_mg_hierarchy(nx, ny, nz, P->od, g);
            if ((int)H.levels.size() > kMGMaxLevels) throw Error(VSR_EINVAL, "too many multigrid levels");
            P->A0inv = P->fp32 ? (void *)P->upload_as<float>(H.coarsest_inverse) : (void *)P->upload(H.coarsest_inverse);
        } else {
            std::vector<double> A0inv = make_coarse_inverse(nx, ny, nz, P->od, g);
            P->A0inv = P->fp32 ? (void *)P->upload_as<float>(A0inv) : (void *)P->upload(A0inv);
        }
        // work buffers
        size_t es = esz;
        auto alloc_t = [&](int64_t cnt) -> void * {
            return P->fp32 ? (void *)P->dalloc<float>(cnt) : (void *)P->dalloc<double>(cnt);
        };
        (void)es;
        P->rF = alloc_t(P->n);
        if (p > kFusedScatterMaxP) P->zF = alloc_t(P->n);
        P->U = alloc_t(patch_solution_entries(P->d));   // the star boxes (see launch_patch_all)
        P->z1 = alloc_t(P->n);
        P->res = alloc_t(P->n);
        {
            const int64_t eb = (int64_t)P->ncell * (p + 1) * (p + 1) * (p + 1) * 2;   // up to 2 slots per cell
            P->E64 = P->dalloc<double>(eb);
            if (P->fp32) P->E32 = P->dalloc<float>(eb);
        }
        P->c3 = alloc_t(P->nc);
        P->c4 = alloc_t(P->nc);
        if (P->cartesian) {
            P->rF0 = alloc_t(P->n);
            P->c0 = alloc_t(P->nc);
            P->e8 = alloc_t(P->ncell * 8);
        }
        if (P->coarse_gmg) {
            if (P->fp32) build_mg<float>(P.get(), H, P->mg32);
            else build_mg<double>(P.get(), H, P->mg64);
        }
        P->vp = P->dalloc<double>(P->n);
        P->vq = P->dalloc<double>(P->n);
        P->vr = P->dalloc<double>(P->n);
        P->vz = P->dalloc<double>(P->n);
        P->vt = P->dalloc<double>(P->n);
        {   // scalars and the (alpha, beta) record of one PCG run (max_iterations pairs)
            const int hcap = P->opt.max_iterations > 0 ? P->opt.max_iterations : 1000;
            std::vector<double> s0(SC_N + 2 * (size_t)hcap, 0.0);
            s0[SC_HCAP] = (double)hcap;
            P->scal = P->upload(s0);
        }
        // partial sums: dot passes (at most 8192 workgroups) and the lattice-line gathers
        const int NCp[3] = {P->d.nx, P->d.ny, P->d.nz};
        P->partials = P->dalloc<double>(std::max<int64_t>(
            std::max<int64_t>(8192, gather_blocks(P->d)), transfer_blocks(XFER_FDM_PROLONG, P->d.p, NCp)));
        VSR_HIP(hipHostMalloc((void **)&P->host_scal, sizeof(double) * SC_N, hipHostMallocDefault));
        if (P->fp32) launch_fill<float>(patch_solution_entries(P->d), (float *)P->U, 0.f, P->ex());
        else launch_fill<double>(patch_solution_entries(P->d), (double *)P->U, 0.0, P->ex());
        P->vx = P->dalloc<double>(P->n);
        if (P->opt.autotune) autotune(P.get());
        // damping (Sec. 2.5)
        if (P->opt.omega > 0) {
            P->omega = P->opt.omega;
        } else {
            estimate_damping(P.get());
        }
        VSR_HIP(hipStreamSynchronize(P->stream));
        P->setup_seconds = now_s() - t0;
        *out = P.release();
    });
}

int64_t vsr_num_dofs(const vsr_problem *prob) { return prob ? prob->n : -1; }

vsr_status vsr_load_vector(vsr_problem *P, const double *f, double *b) {
    return guarded([&] {
        if (!P || !f || !b) throw Error(VSR_EINVAL, "NULL argument");
        launch_load_vector(P->d, P->IDq64, P->wdet, f, P->E64, P->ex());
        launch_gather<double>(P->d, 1, P->E64, nullptr, b, P->ex());
        VSR_HIP(hipGetLastError());
    });
}

vsr_status vsr_apply_operator(vsr_problem *P, const double *x, double *y) {
    return guarded([&] {
        if (!P || !x || !y) throw Error(VSR_EINVAL, "NULL argument");
        op_apply<double>(P, x, y);
    });
}

vsr_status vsr_apply_operator_noalloc(vsr_problem *P, const double *x, double *y) {
    return guarded([&] {
        if (!P || !x || !y) throw Error(VSR_EINVAL, "NULL argument");
        // the element vector (up to 2 slots per cell) goes to the static workspace
        const int64_t n1 = P->d.p + 1;
        double *E = static_cast<double *>(static_workspace((size_t)P->ncell * n1 * n1 * n1 * 2 * sizeof(double)));
        const int slots = op_cells<double>(P, x, E);
        launch_gather<double>(P->d, slots, E, nullptr, y, P->ex());
        VSR_HIP(hipGetLastError());
    });
}

vsr_status vsr_apply_relaxation(vsr_problem *P, const double *r, double *z, int32_t mode) {
    return guarded([&] {
        if (!P || !r || !z) throw Error(VSR_EINVAL, "NULL argument");
        if (mode < 0 || mode > 2) throw Error(VSR_EINVAL, "mode must be 0, 1 or 2");
        precond(P, r, z, mode);
    });
}

vsr_status vsr_pcg_solve(vsr_problem *P, const double *b, double *x, double rtol, vsr_solve_info *info) {
    vsr_solve_info loc{};
    vsr_status st = guarded([&] {
        if (!P || !b || !x) throw Error(VSR_EINVAL, "NULL argument");
        if (!(rtol > 0)) throw Error(VSR_EINVAL, "rtol must be positive");
        if (!P->profiling) {
            // device-driven: the gated iteration replayed from a graph, the stop polled one
            // iteration behind (no host round trip between iterations)
            if (!P->self) P->self = make_batch(1, &P, 1, P->opt.batch_eager != 0, false);
            const double *bv[1] = {b};
            double *xv[1] = {x};
            P->self->solve(bv, xv, rtol, &loc);
            return;
        }
        // host-driven (profiling: every recorded patch launch belongs to a real iteration)
        double t0 = now_s();
        int maxit = P->opt.max_iterations > 0 ? P->opt.max_iterations : 1000;
        pcg_init(P, b, x);
        double bb = read_scalar(P, SC_RR);
        if (!std::isfinite(bb)) throw Error(VSR_EINVAL, "non-finite right-hand side");
        double rr = bb;
        int it = 0;
        bool conv = bb == 0.0;
        if (!conv) {
            pcg_first_direction(P);
            while (it < maxit) {
                pcg_update(P, x, 4);
                ++it;
                rr = read_scalar(P, SC_RR);
                if (!std::isfinite(rr)) break;
                // ||r||_2 <= rtol ||b||_2, tested on squares as the batched solve does on the device
                if (rr <= rtol * rtol * bb) {
                    conv = true;
                    break;
                }
                pcg_direction(P);
            }
        }
        VSR_HIP(hipStreamSynchronize(P->stream));
        double t1 = now_s();
        ritz_of_run(P, it > 0 ? (int)read_scalar(P, SC_NA) : 0, loc);
        double tr = true_residual(P, b, x);
        double bn = std::sqrt(bb);
        loc.iterations = it;
        loc.converged = conv ? 1 : 0;
        loc.rel_residual = bn > 0 ? std::sqrt(rr) / bn : 0.0;
        loc.true_rel_residual = bn > 0 ? tr / bn : 0.0;
        loc.omega = P->omega;
        loc.lambda_min = P->lmin;
        loc.lambda_max = P->lmax;
        loc.setup_seconds = P->setup_seconds;
        loc.solve_seconds = t1 - t0;
        if (!conv) throw Error(VSR_ENOCONV, "PCG did not converge in " + std::to_string(it) + " iterations");
    });
    if (info && P) *info = loc;
    return st;
}

vsr_status vsr_get_damping(const vsr_problem *P, double *omega, double *lmin, double *lmax) {
    return guarded([&] {
        if (!P) throw Error(VSR_EINVAL, "NULL argument");
        if (omega) *omega = P->omega;
        if (lmin) *lmin = P->lmin;
        if (lmax) *lmax = P->lmax;
    });
}

vsr_status vsr_set_profiling(vsr_problem *P, int32_t enable) {
    return guarded([&] {
        if (!P) throw Error(VSR_EINVAL, "NULL argument");
        P->profiling = enable != 0;
    });
}

vsr_status vsr_kernel_stats(vsr_problem *P, int64_t *launches, double *total_ms, double *bytes_per_launch) {
    return guarded([&] {
        if (!P) throw Error(VSR_EINVAL, "NULL argument");
        VSR_HIP(hipStreamSynchronize(P->stream));
        double tot = 0;
        for (size_t i = 0; i < P->events_used; ++i) {
            float ms = 0;
            VSR_HIP(hipEventElapsedTime(&ms, P->events[i].first, P->events[i].second));
            tot += ms;
        }
        if (launches) *launches = (int64_t)P->events_used;
        if (total_ms) *total_ms = tot;
        if (bytes_per_launch) *bytes_per_launch = P->bytes_patch_launch;
        P->events_used = 0;
    });
}

vsr_status vsr_factor_info(const vsr_problem *P, int64_t *num_patches, int64_t *factor_entries) {
    return guarded([&] {
        if (!P) throw Error(VSR_EINVAL, "NULL argument");
        if (num_patches) *num_patches = (int64_t)P->n_int + P->n_bnd;
        if (factor_entries) *factor_entries = P->factor_entries;
    });
}

void vsr_destroy(vsr_problem *P) { destroy_problem(P); }

vsr_status vsr_get_tuning(const vsr_problem *P, int32_t shapes[6]) {
    return guarded([&] {
        if (!P || !shapes) throw Error(VSR_EINVAL, "NULL argument");
        shapes[0] = P->tune.op_cpw64;
        shapes[1] = P->tune.op_cpw32;
        shapes[2] = P->tune.patch_unroll;
        shapes[3] = P->tune.opg_split64;
        shapes[4] = P->tune.opg_split32;
        shapes[5] = P->tune.patch_threads;
    });
}

vsr_status vsr_set_tuning(vsr_problem *P, const int32_t shapes[6]) {
    return guarded([&] {
        if (!P || !shapes) throw Error(VSR_EINVAL, "NULL argument");
        auto cpw_ok = [](int c) { return c == 1 || c == 2 || c == 4; };
        if (!cpw_ok(shapes[0]) || !cpw_ok(shapes[1])) throw Error(VSR_EINVAL, "operator cells per workgroup must be 1, 2 or 4");
        if (shapes[2] != 4 && shapes[2] != 8 && shapes[2] != 16) throw Error(VSR_EINVAL, "unroll must be 4, 8 or 16");
        for (int i = 3; i < 5; ++i)
            if (shapes[i] < 0 || shapes[i] > 2) throw Error(VSR_EINVAL, "workgroups per cell must be 0, 1 or 2");
        if (shapes[5] != 256 && shapes[5] != 512 && shapes[5] != 1024)
            throw Error(VSR_EINVAL, "patch threads must be 256, 512 or 1024");
        if (shapes[5] == 1024 && shapes[2] == 16) throw Error(VSR_EINVAL, "1024 patch threads take an unroll of 4 or 8");
        VSR_HIP(hipStreamSynchronize(P->stream));
        Tuning t;
        t.op_cpw64 = shapes[0];
        t.op_cpw32 = shapes[1];
        t.patch_unroll = shapes[2];
        t.opg_split64 = shapes[3];
        t.opg_split32 = shapes[4];
        t.patch_threads = shapes[5];
        P->tune = t;
        ++P->tune_version;   // recorded iterations (its own, a batch's) are re-recorded at their next solve
        delete P->self;
        P->self = nullptr;
    });
}

vsr_status vsr_batch_create(int32_t count, vsr_problem *const *members, const vsr_options *opt, vsr_batch **out) {
    return guarded([&] {
        if (!out) throw Error(VSR_EINVAL, "NULL argument");
        *out = nullptr;
        if (count < 1 || !members) throw Error(VSR_EINVAL, "a batch needs count >= 1 members");
        for (int32_t i = 0; i < count; ++i) {
            if (!members[i]) throw Error(VSR_EINVAL, "NULL member " + std::to_string(i));
            for (int32_t j = 0; j < i; ++j)
                if (members[j] == members[i]) throw Error(VSR_EINVAL, "member " + std::to_string(i) + " repeated");
        }
        vsr_options o;
        if (opt) o = *opt;
        else vsr_default_options(&o);
        if (o.batch_streams < 0 || o.batch_streams > 16) throw Error(VSR_EINVAL, "batch_streams must be in [0, 16]");
        *out = make_batch(count, members, o.batch_streams > 0 ? o.batch_streams : 4, o.batch_eager != 0, true);
    });
}

vsr_status vsr_setup_batch(int32_t count, const vsr_mesh *meshes, const int32_t *p, const vsr_coefficients *coefs,
                           const vsr_options *opt, vsr_batch **out) {
    std::vector<vsr_problem *> made;
    vsr_status st = guarded([&] {
        if (!out) throw Error(VSR_EINVAL, "NULL argument");
        *out = nullptr;
        if (count < 1 || !meshes || !p) throw Error(VSR_EINVAL, "a batch needs count >= 1, meshes and degrees");
        for (int32_t i = 0; i < count; ++i) {
            vsr_problem *P = nullptr;
            vsr_status s1 = vsr_setup(&meshes[i], p[i], coefs ? &coefs[i] : nullptr, opt, &P);
            if (s1 != VSR_OK) throw Error(s1, "member " + std::to_string(i) + ": " + vsr::g_last_error_text);
            made.push_back(P);
        }
        vsr_status s2 = vsr_batch_create(count, made.data(), opt, out);
        if (s2 != VSR_OK) throw Error(s2, vsr::g_last_error_text);
        made.clear();
    });
    for (vsr_problem *P : made) delete P;
    return st;
}

int32_t vsr_batch_size(const vsr_batch *B) { return B ? (int32_t)B->members.size() : -1; }

vsr_problem *vsr_batch_member(vsr_batch *B, int32_t i) {
    if (!B || i < 0 || i >= (int32_t)B->members.size()) return nullptr;
    return B->members[i];
}

vsr_status vsr_pcg_solve_batch(vsr_batch *B, const double *const *b_dev, double *const *x_dev, double rtol,
                               vsr_solve_info *infos) {
    return guarded([&] {
        if (!B || !b_dev || !x_dev) throw Error(VSR_EINVAL, "NULL argument");
        if (!(rtol > 0)) throw Error(VSR_EINVAL, "rtol must be positive");
        for (size_t i = 0; i < B->members.size(); ++i)
            if (!b_dev[i] || !x_dev[i]) throw Error(VSR_EINVAL, "NULL vector of member " + std::to_string(i));
        B->solve(b_dev, x_dev, rtol, infos);
    });
}

void vsr_destroy_batch(vsr_batch *B) { delete B; }

vsr_status vsr_elasticity_setup(const vsr_mesh *mesh, int32_t p, double mu, double lambda, const vsr_options *opt,
                                vsr_elasticity **out) {
    return guarded([&] {
        if (!mesh || !out || !mesh->vertices) throw Error(VSR_EINVAL, "NULL argument");
        *out = nullptr;
        if (!(mu > 0) || !(lambda >= 0) || !std::isfinite(mu) || !std::isfinite(lambda))
            throw Error(VSR_EINVAL, "need mu > 0 and lambda >= 0");
        if (p < 2 || p > 15) throw Error(VSR_EINVAL, "p must be in [2, 15]");
        const int nx = mesh->nx, ny = mesh->ny, nz = mesh->nz;
        if (nx < 2 || ny < 2 || nz < 2) throw Error(VSR_EINVAL, "every mesh axis needs at least 2 cells");
        const double t0 = now_s();
        // axis-aligned boxes: vertex (k, j, i) = (X[i], Y[j], Z[k])
        const double *V = mesh->vertices;
        auto vert = [&](int k, int j, int i, int a) { return V[3 * (((int64_t)k * (ny + 1) + j) * (nx + 1) + i) + a]; };
        std::vector<double> X(nx + 1), Y(ny + 1), Z(nz + 1);
        for (int i = 0; i <= nx; ++i) X[i] = vert(0, 0, i, 0);
        for (int j = 0; j <= ny; ++j) Y[j] = vert(0, j, 0, 1);
        for (int k = 0; k <= nz; ++k) Z[k] = vert(k, 0, 0, 2);
        double scale = 0;
        for (double v : X) scale = std::max(scale, std::fabs(v));
        for (double v : Y) scale = std::max(scale, std::fabs(v));
        for (double v : Z) scale = std::max(scale, std::fabs(v));
        const double tol = 1e-12 * std::max(scale, 1e-300);
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i <= nx; ++i)
                    if (!(std::fabs(vert(k, j, i, 0) - X[i]) <= tol && std::fabs(vert(k, j, i, 1) - Y[j]) <= tol &&
                          std::fabs(vert(k, j, i, 2) - Z[k]) <= tol))
                        throw Error(VSR_EINVAL, "elasticity needs a mesh of axis-aligned boxes (a tensor grid)");
        for (int i = 0; i < nx; ++i) if (!(X[i + 1] > X[i])) throw Error(VSR_EMESH, "cell with non-positive length");
        for (int j = 0; j < ny; ++j) if (!(Y[j + 1] > Y[j])) throw Error(VSR_EMESH, "cell with non-positive length");
        for (int k = 0; k < nz; ++k) if (!(Z[k + 1] > Z[k])) throw Error(VSR_EMESH, "cell with non-positive length");
        auto L = std::make_unique<vsr_elasticity>();
        vsr_options o;
        if (opt) o = *opt;
        else vsr_default_options(&o);
        L->mu = mu;
        L->lam = lambda;
        L->stream = (hipStream_t)o.stream;
        VSR_HIP(hipEventCreateWithFlags(&L->fork, hipEventDisableTiming));
        for (hipEvent_t &e : L->it_ev) VSR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        VSR_HIP(hipStreamCreateWithFlags(&L->origin, hipStreamNonBlocking));
        VSR_HIP(hipHostMalloc((void **)&L->host_done, sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
        VSR_HIP(hipHostGetDevicePointer((void **)&L->dev_done, L->host_done, 0));
        *L->host_done = 0.0;
        const int64_t ncell = (int64_t)nx * ny * nz;
        // SDC scalings of each component (exact on boxes): (mu + (mu + lam) [a = j]) |J| (2 / h_a)^2
        std::vector<double> coef((size_t)ncell * 12);
        std::vector<std::vector<double>> mus(3, std::vector<double>((size_t)ncell * 3));
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const int64_t e = ((int64_t)k * ny + j) * nx + i;
                    const double h[3] = {X[i + 1] - X[i], Y[j + 1] - Y[j], Z[k + 1] - Z[k]};
                    const double vol = h[0] * h[1] * h[2] / 8.0;
                    for (int c = 0; c < 3; ++c)
                        for (int a = 0; a < 3; ++a) {
                            const double kk = (mu + (a == c ? mu + lambda : 0.0)) * vol * (2 / h[a]) * (2 / h[a]);
                            coef[e * 12 + 3 * c + a] = kk;
                            mus[c][e * 3 + a] = kk;
                        }
                    coef[e * 12 + 9] = vol * (2 / h[0]) * (2 / h[1]);
                    coef[e * 12 + 10] = vol * (2 / h[0]) * (2 / h[2]);
                    coef[e * 12 + 11] = vol * (2 / h[1]) * (2 / h[2]);
                }
        // the component problems: their patches and FDM transfers give the SDC relaxation (no
        // damping estimate of their own; the multigrid coarse setup is the cheap one they skip using)
        vsr_options oc = o;
        oc.omega = 1.0;
        oc.coarse_solver = 2;
        oc.autotune = 0;
        for (int c = 0; c < 3; ++c) {
            vsr_coefficients cf{nullptr, mus[c].data()};
            vsr_status st = vsr_setup(mesh, p, &cf, &oc, &L->comp[c]);
            if (st != VSR_OK) throw Error(st, g_last_error_text);
        }
        vsr_problem *P0 = L->comp[0];
        L->d = P0->d;
        L->n = P0->n;
        L->ncell = ncell;
        // the three components' patch arrays (factors, scalings, FDM residuals, star boxes,
        // assembled solutions) moved next to each other, so that each phase of the SDC
        // relaxation runs as one launch over all three
        {
            const size_t tb = P0->fp32 ? sizeof(float) : sizeof(double);
            const int64_t ulen = patch_solution_entries(P0->d);
            for (int c = 1; c < 3; ++c)
                if (L->comp[c]->fint_len != P0->fint_len || L->comp[c]->fbnd_len != P0->fbnd_len ||
                    L->comp[c]->mu_len != P0->mu_len || L->comp[c]->fp32 != P0->fp32)
                    throw Error(VSR_EINVAL, "elasticity components differ in structure");
            auto merge = [&](void *vsr_problem::*member, int64_t len) {
                char *base = L->dalloc<char>(3 * (size_t)len * tb);
                for (int c = 0; c < 3; ++c) L->comp[c]->move_to(&(L->comp[c]->*member), base + c * (size_t)len * tb, len * tb);
            };
            merge(&vsr_problem::fint, P0->fint_len);
            merge(&vsr_problem::fbnd, P0->fbnd_len);
            merge(&vsr_problem::mu_sur, P0->mu_len);
            merge(&vsr_problem::rF, P0->n);
            merge(&vsr_problem::U, ulen);
            if (P0->zF) merge(&vsr_problem::zF, P0->n);
            L->cs = CompStrides{P0->fint_len, P0->fbnd_len, P0->mu_len, P0->n, ulen};
        }
        const int n1 = p + 1;
        // 1-D matrices A, B, C (C[a][b] = sum_q w_q l_a'(x_q) l_b(x_q)) and C^T
        const OneD &od = P0->od;
        std::vector<double> M1(4 * (size_t)n1 * n1, 0.0);
        for (int a = 0; a < n1; ++a)
            for (int b = 0; b < n1; ++b) {
                M1[a * n1 + b] = od.A[a * n1 + b];
                M1[n1 * n1 + a * n1 + b] = od.B[a * n1 + b];
                double cab = 0;
                for (int q = 0; q < od.q; ++q) cab += od.wq[q] * od.Dq[q * n1 + a] * od.Iq[q * n1 + b];
                M1[2 * n1 * n1 + a * n1 + b] = cab;
                M1[3 * n1 * n1 + b * n1 + a] = cab;
            }
        L->M1 = L->dalloc<double>(M1.size());
        VSR_HIP(hipMemcpy(L->M1, M1.data(), M1.size() * sizeof(double), hipMemcpyHostToDevice));
        L->coef = L->dalloc<double>(coef.size());
        VSR_HIP(hipMemcpy(L->coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice));
        L->E = L->dalloc<double>(3 * (size_t)ncell * n1 * n1 * n1);
        const int64_t N = 3 * L->n;
        L->vr = L->dalloc<double>(N);
        L->vz = L->dalloc<double>(N);
        L->vp = L->dalloc<double>(N);
        L->vq = L->dalloc<double>(N);
        L->vt = L->dalloc<double>(N);
        // the V-cycle's precision follows the component relaxations'
        L->fp32 = o.relax_fp32 != 0;
        const size_t tsz = L->fp32 ? sizeof(float) : sizeof(double);
        auto upload_f = [&](const std::vector<double> &v) {
            std::vector<float> f(v.begin(), v.end());
            float *d = L->dalloc<float>(f.size());
            VSR_HIP(hipMemcpy(d, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
            return d;
        };
        if (L->fp32) {
            L->M1f = upload_f(M1);
            L->coeff = upload_f(coef);
        }
        L->cz = L->dalloc<char>(N * tsz);
        L->ct = L->dalloc<char>(N * tsz);
        // vector Q1 coarse space, exact solve
        L->nc = (nx - 1) * (ny - 1) * (nz - 1);
        if (L->nc > 0) {
            if (3LL * L->nc > 12000) throw Error(VSR_EINVAL, "elasticity coarse space limited to 12,000 unknowns");
            std::vector<double> A0 = elasticity_q1_matrix(X, Y, Z, od, mu, lambda);
            std::vector<double> A0i = spd_inverse(3 * L->nc, A0);
            L->A0inv = L->dalloc<double>(A0i.size());
            VSR_HIP(hipMemcpy(L->A0inv, A0i.data(), A0i.size() * sizeof(double), hipMemcpyHostToDevice));
            if (L->fp32) L->A0f = upload_f(A0i);
            L->cc0 = L->dalloc<char>(3 * L->nc * tsz);
            L->cc1 = L->dalloc<char>(3 * L->nc * tsz);
        }
        if (o.omega > 0) L->omega = o.omega;
        else el_damping(L.get(), o.lanczos_steps > 0 ? o.lanczos_steps : 20, o.seed);
        VSR_HIP(hipStreamSynchronize(L->stream));
        L->setup_seconds = now_s() - t0;
        *out = L.release();
    });
}

int64_t vsr_elasticity_num_dofs(const vsr_elasticity *L) { return L ? 3 * L->n : -1; }

vsr_status vsr_elasticity_load_vector(vsr_elasticity *L, const double *f, double *b) {
    return guarded([&] {
        if (!L || !f || !b) throw Error(VSR_EINVAL, "NULL argument");
        const int q = L->comp[0]->d.q;
        const int64_t per = L->ncell * (int64_t)q * q * q;
        for (int c = 0; c < 3; ++c) {
            vsr_status st = vsr_load_vector(L->comp[c], f + c * per, b + c * L->n);
            if (st != VSR_OK) throw Error(st, g_last_error_text);
        }
    });
}

vsr_status vsr_elasticity_apply_operator(vsr_elasticity *L, const double *x, double *y) {
    return guarded([&] {
        if (!L || !x || !y) throw Error(VSR_EINVAL, "NULL argument");
        el_op(L, x, y);
        VSR_HIP(hipGetLastError());
    });
}

vsr_status vsr_elasticity_apply_relaxation(vsr_elasticity *L, const double *r, double *z, int32_t mode) {
    return guarded([&] {
        if (!L || !r || !z) throw Error(VSR_EINVAL, "NULL argument");
        if (mode < 0 || mode > 2) throw Error(VSR_EINVAL, "mode must be 0, 1 or 2");
        el_precond(L, r, z, mode);
        VSR_HIP(hipGetLastError());
    });
}

vsr_status vsr_elasticity_damping(const vsr_elasticity *L, double *omega, double *lmin, double *lmax) {
    return guarded([&] {
        if (!L) throw Error(VSR_EINVAL, "NULL argument");
        if (omega) *omega = L->omega;
        if (lmin) *lmin = L->lmin;
        if (lmax) *lmax = L->lmax;
    });
}

vsr_status vsr_elasticity_pcg_solve(vsr_elasticity *L, const double *b, double *x, double rtol, vsr_solve_info *info) {
    vsr_solve_info loc{};
    vsr_status st = guarded([&] {
        if (!L || !b || !x) throw Error(VSR_EINVAL, "NULL argument");
        if (!(rtol > 0)) throw Error(VSR_EINVAL, "rtol must be positive");
        const int64_t N = 3 * L->n;
        vsr_problem *P = L->comp[0];   // its scalars and partials serve the 3n-vector PCG
        const int maxit = P->opt.max_iterations > 0 ? P->opt.max_iterations : 1000;
        VSR_HIP(hipStreamSynchronize(L->stream));
        const double t0 = now_s();
        // device-driven: step lengths, directions and the stopping test stay on the device;
        // every launch after the start checks the stop flag, and the host polls its mapped
        // copy one iteration behind, so the GPU never waits for the host between iterations
        L->gate = nullptr;
        *L->host_done = 0.0;
        launch_fill<double>(N, x, 0.0, L->ex());
        launch_axpby_to_double<double>(N, 1.0, b, 0.0, L->vr, L->ex());
        launch_dot(N, b, b, P->partials, P->scal, 4, nullptr, L->ex());                  // RR = b.b
        launch_pcg_start(P->scal, rtol, maxit, 0, 0.0, L->dev_done, L->ex());
        L->gate = P->scal + SC_DONE;
        const hipStream_t user = L->stream;
        auto iteration = [&] {
            el_op(L, L->vp, L->vq);
            launch_dot(N, L->vp, L->vq, P->partials, P->scal, 1, nullptr, L->ex());       // alpha = RZ / p.q
            launch_pcg_xr(N, x, L->vr, L->vp, L->vq, P->scal, P->partials, 5, L->dev_done, L->ex());
            el_precond(L, L->vr, L->vz, 0);
            launch_dot(N, L->vr, L->vz, P->partials, P->scal, 2, nullptr, L->ex());       // beta, RZ
            launch_pcg_p(N, L->vp, L->vz, P->scal, L->ex());
        };
        try {
            el_precond(L, L->vr, L->vz, 0);
            launch_dot(N, L->vr, L->vz, P->partials, P->scal, 3, nullptr, L->ex());    // RZ = r.z
            launch_axpby_to_double<double>(N, 1.0, L->vz, 0.0, L->vp, L->ex());
            // the iterations run on the library's own stream, forked from the caller's, as
            // replays of one recorded iteration; the recording holds x's address and is made
            // again for another x
            VSR_HIP(hipEventRecord(L->fork, user));
            VSR_HIP(hipStreamWaitEvent(L->origin, L->fork, 0));
            L->stream = L->origin;
            if (!L->exec || L->graph_x != x) {
                if (L->exec) VSR_HIP(hipGraphExecDestroy(L->exec));
                if (L->graph) VSR_HIP(hipGraphDestroy(L->graph));
                L->exec = nullptr;
                L->graph = nullptr;
                L->graph_x = nullptr;
                VSR_HIP(hipStreamBeginCapture(L->origin, hipStreamCaptureModeThreadLocal));
                try {
                    iteration();
                } catch (...) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(L->origin, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                VSR_HIP(hipStreamEndCapture(L->origin, &L->graph));
                VSR_HIP(hipGraphInstantiate(&L->exec, L->graph, nullptr, nullptr, 0));
                L->graph_x = x;
            }
            // the device stops by itself (DONE) at convergence or at max_iterations; the host
            // stops queueing once the replay before the last one queued shows DONE
            for (int enq = 1; enq <= maxit + 1; ++enq) {
                VSR_HIP(hipGraphLaunch(L->exec, L->origin));
                VSR_HIP(hipEventRecord(L->it_ev[enq & 1], L->origin));
                if (enq >= 2) {
                    VSR_HIP(hipEventSynchronize(L->it_ev[(enq - 1) & 1]));
                    if (*(volatile double *)L->host_done != 0.0) break;
                }
            }
        } catch (...) {
            L->stream = user;
            L->gate = nullptr;
            throw;
        }
        VSR_HIP(hipEventRecord(L->fork, L->origin));
        VSR_HIP(hipStreamWaitEvent(user, L->fork, 0));
        L->stream = user;
        L->gate = nullptr;
        VSR_HIP(hipStreamSynchronize(L->stream));
        const double t1 = now_s();
        VSR_HIP(hipMemcpy(P->host_scal, P->scal, SC_N * sizeof(double), hipMemcpyDeviceToHost));
        const double bb = P->host_scal[SC_BB], rr = P->host_scal[SC_RR], status = P->host_scal[SC_STATUS];
        const int it = (int)P->host_scal[SC_IT], na = (int)P->host_scal[SC_NA];
        if (!std::isfinite(bb)) throw Error(VSR_EINVAL, "non-finite right-hand side");
        const bool conv = status == 1.0;
        el_op(L, x, L->vt);
        launch_axpby_to_double<double>(N, 1.0, b, -1.0, L->vt, L->ex());
        const double tr = std::sqrt(std::max(0.0, el_dot(L, L->vt, L->vt)));
        const double bn = std::sqrt(bb);
        loc.iterations = it;
        loc.converged = conv ? 1 : 0;
        loc.rel_residual = bn > 0 ? std::sqrt(rr) / bn : 0.0;
        loc.true_rel_residual = bn > 0 ? tr / bn : 0.0;
        loc.omega = L->omega;
        loc.lambda_min = L->lmin;
        loc.lambda_max = L->lmax;
        loc.setup_seconds = L->setup_seconds;
        loc.solve_seconds = t1 - t0;
        ritz_of_run(P, it > 0 ? na : 0, loc);
        if (!conv) throw Error(VSR_ENOCONV, "PCG did not converge in " + std::to_string(it) + " iterations");
    });
    if (info && L) *info = loc;
    return st;
}

void vsr_elasticity_destroy(vsr_elasticity *L) { delete L; }

const char *vsr_last_error(void) { return vsr::g_last_error_text.c_str(); }

}  // extern "C"
