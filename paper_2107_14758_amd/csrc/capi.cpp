// C ABI (include/vsr.h): problem setup, operator/relaxation applies, PCG driver.
//
// Method references: Brubeck & Farrell, "A scalable and robust vertex-star
// relaxation for high-order FEM", Sec. 2.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
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

struct Table {
    int *rowptr = nullptr, *col = nullptr;
    double *w64 = nullptr;
    float *w32 = nullptr;
    int n_out = 0, n_in = 0;
};

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
    double *AB64 = nullptr, *IDq64 = nullptr, *mu64 = nullptr, *Gw64 = nullptr, *wdet = nullptr;
    float *AB32 = nullptr, *IDq32 = nullptr, *mu32 = nullptr, *Gw32 = nullptr;
    // relaxation data in the cycle precision
    void *mu_sur = nullptr, *lam = nullptr, *afc = nullptr, *fint = nullptr, *fbnd = nullptr;
    int n_int = 0, n_bnd = 0;
    int *verts = nullptr, *bdesc = nullptr;
    int64_t *boff = nullptr;
    PatchArgs pa{};
    int64_t factor_entries = 0;       // structurally nonzero entries over all patches
    double bytes_patch_launch = 0;    // algorithmic bytes of one interior patch-solve launch
    Table tab[4][3];                  // [TT, T, PT, P][axis]
    int cdim[3] = {0, 0, 0};
    int nc = 0;
    void *A0inv = nullptr;
    // work buffers (cycle precision unless noted)
    void *t1 = nullptr, *t2 = nullptr, *rF = nullptr, *zF = nullptr, *U = nullptr;
    void *c1 = nullptr, *c2 = nullptr, *c3 = nullptr, *c4 = nullptr;
    void *z1 = nullptr, *az = nullptr;
    double *vp = nullptr, *vq = nullptr, *vr = nullptr, *vz = nullptr, *vt = nullptr;
    double *scal = nullptr, *partials = nullptr, *host_scal = nullptr;
    double omega = 1.0, lmin = 0.0, lmax = 0.0;
    double setup_seconds = 0.0;
    // profiling of the interior patch-solve launches
    bool profiling = false;
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
};

namespace {

template <typename T>
void op_apply(vsr_problem *P, const T *x, T *y) {
    launch_fill<T>(P->n, y, T(0), P->stream);
    if constexpr (std::is_same<T, double>::value) {
        if (P->cartesian) launch_op_kron<double>(P->d, P->AB64, P->mu64, x, y, P->stream);
        else launch_op_general<double>(P->d, P->IDq64, P->Gw64, x, y, P->stream);
    } else {
        if (P->cartesian) launch_op_kron<float>(P->d, P->AB32, P->mu32, x, y, P->stream);
        else launch_op_general<float>(P->d, P->IDq32, P->Gw32, x, y, P->stream);
    }
    VSR_HIP(hipGetLastError());
}

template <typename T>
const T *wt(const Table &t) {
    if constexpr (std::is_same<T, double>::value) return t.w64;
    else return t.w32;
}

// out = alpha * S in + beta * out,  S = T (sum_j Rbar_j^T A_j^{-1} Rbar_j) T^T  (Sec. 2.4-2.6)
template <typename T, typename Tin>
void relax_apply(vsr_problem *P, const Tin *in, T *out, T alpha, T beta) {
    const int L[3] = {P->d.Lx, P->d.Ly, P->d.Lz};
    T *t1 = (T *)P->t1, *t2 = (T *)P->t2, *rF = (T *)P->rF, *zF = (T *)P->zF, *U = (T *)P->U;
    const Table *TT = P->tab[0], *Tp = P->tab[1];
    launch_axis_pass<Tin, T>(TT[0].rowptr, TT[0].col, wt<T>(TT[0]), 0, L, L, in, t1, T(1), T(0), P->stream);
    launch_axis_pass<T, T>(TT[1].rowptr, TT[1].col, wt<T>(TT[1]), 1, L, L, t1, t2, T(1), T(0), P->stream);
    launch_axis_pass<T, T>(TT[2].rowptr, TT[2].col, wt<T>(TT[2]), 2, L, L, t2, rF, T(1), T(0), P->stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (P->profiling) {
        if (P->events_used == P->events.size()) {
            VSR_HIP(hipEventCreate(&e0));
            VSR_HIP(hipEventCreate(&e1));
            P->events.push_back({e0, e1});
        }
        e0 = P->events[P->events_used].first;
        e1 = P->events[P->events_used].second;
        VSR_HIP(hipEventRecord(e0, P->stream));
    }
    launch_patch_interior<T>(P->d, P->pa, P->n_int, P->verts, (const T *)P->fint, (const T *)P->mu_sur, (const T *)P->lam,
                             (const T *)P->afc, rF, U, P->stream);
    if (P->profiling) {
        VSR_HIP(hipEventRecord(e1, P->stream));
        ++P->events_used;
    }
    launch_patch_boundary<T>(P->d, P->n_bnd, P->bdesc, P->boff, (const T *)P->fbnd, (const T *)P->mu_sur, (const T *)P->lam,
                             (const T *)P->afc, rF, U, P->stream);
    launch_patch_assemble<T>(P->d, P->opt.interior_patches_only, U, zF, P->stream);
    launch_axis_pass<T, T>(Tp[0].rowptr, Tp[0].col, wt<T>(Tp[0]), 0, L, L, zF, t1, T(1), T(0), P->stream);
    launch_axis_pass<T, T>(Tp[1].rowptr, Tp[1].col, wt<T>(Tp[1]), 1, L, L, t1, t2, T(1), T(0), P->stream);
    launch_axis_pass<T, T>(Tp[2].rowptr, Tp[2].col, wt<T>(Tp[2]), 2, L, L, t2, out, alpha, beta, P->stream);
    VSR_HIP(hipGetLastError());
}

// out = alpha * P A0^{-1} P^T in + beta * out  (Sec. 2.5)
template <typename T, typename Tin>
void coarse_apply(vsr_problem *P, const Tin *in, T *out, T alpha, T beta) {
    if (P->nc == 0) {
        if (beta == T(0)) launch_fill<T>(P->n, out, T(0), P->stream);
        return;
    }
    const int L[3] = {P->d.Lx, P->d.Ly, P->d.Lz};
    const int *c = P->cdim;
    const int d1[3] = {c[0], L[1], L[2]}, d2[3] = {c[0], c[1], L[2]}, d3[3] = {c[0], c[1], c[2]};
    T *c1 = (T *)P->c1, *c2 = (T *)P->c2, *c3 = (T *)P->c3, *c4 = (T *)P->c4;
    const Table *R = P->tab[2], *Pr = P->tab[3];
    launch_axis_pass<Tin, T>(R[0].rowptr, R[0].col, wt<T>(R[0]), 0, L, d1, in, c1, T(1), T(0), P->stream);
    launch_axis_pass<T, T>(R[1].rowptr, R[1].col, wt<T>(R[1]), 1, d1, d2, c1, c2, T(1), T(0), P->stream);
    launch_axis_pass<T, T>(R[2].rowptr, R[2].col, wt<T>(R[2]), 2, d2, d3, c2, c3, T(1), T(0), P->stream);
    launch_dense_gemv<T>(P->nc, (const T *)P->A0inv, c3, c4, T(1), T(0), P->stream);
    launch_axis_pass<T, T>(Pr[2].rowptr, Pr[2].col, wt<T>(Pr[2]), 2, d3, d2, c4, c2, T(1), T(0), P->stream);
    launch_axis_pass<T, T>(Pr[1].rowptr, Pr[1].col, wt<T>(Pr[1]), 1, d2, d1, c2, c1, T(1), T(0), P->stream);
    launch_axis_pass<T, T>(Pr[0].rowptr, Pr[0].col, wt<T>(Pr[0]), 0, d1, L, c1, out, alpha, beta, P->stream);
    VSR_HIP(hipGetLastError());
}

// z = M r in the cycle precision T; mode 0: preconditioner, 1: relaxation, 2: coarse.
template <typename T>
void precondition(vsr_problem *P, const double *r, double *z, int mode) {
    T *z1 = (T *)P->z1, *az = (T *)P->az;
    const T w = (T)P->omega;
    if (mode == 1) {
        relax_apply<T, double>(P, r, z1, T(1), T(0));
    } else if (mode == 2) {
        coarse_apply<T, double>(P, r, z1, T(1), T(0));
    } else if (P->opt.cycle == 1) {
        relax_apply<T, double>(P, r, z1, T(1), T(0));
        coarse_apply<T, double>(P, r, z1, T(1), T(1));
    } else {
        // hybrid V(1,1): z1 = w S r; z2 = z1 + C (r - A z1); z = z2 + w S (r - A z2)
        relax_apply<T, double>(P, r, z1, w, T(0));
        op_apply<T>(P, z1, az);
        launch_residual<T>(P->n, r, az, az, P->stream);
        coarse_apply<T, T>(P, az, z1, T(1), T(1));
        op_apply<T>(P, z1, az);
        launch_residual<T>(P->n, r, az, az, P->stream);
        relax_apply<T, T>(P, az, z1, w, T(1));
    }
    launch_axpby_to_double<T>(P->n, 1.0, z1, 0.0, z, P->stream);
    VSR_HIP(hipGetLastError());
}

void precond(vsr_problem *P, const double *r, double *z, int mode) {
    if (P->fp32) precondition<float>(P, r, z, mode);
    else precondition<double>(P, r, z, mode);
}

double read_scalar(vsr_problem *P, int slot) {
    VSR_HIP(hipMemcpyAsync(P->host_scal, P->scal + slot, sizeof(double), hipMemcpyDeviceToHost, P->stream));
    VSR_HIP(hipStreamSynchronize(P->stream));
    return *P->host_scal;
}

double dot(vsr_problem *P, const double *x, const double *y) {
    int nb = launch_dot_partial(P->n, x, y, P->partials, P->stream);
    launch_finalize(nb, P->partials, P->scal, 0, P->stream);
    return read_scalar(P, SC_TMP);
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
    launch_fill<double>(P->n, P->vt, 0.0, P->stream);
    precond(P, P->vr, P->vz, 1);
    int nb = launch_dot_partial(P->n, P->vr, P->vz, P->partials, P->stream);
    launch_finalize(nb, P->partials, P->scal, 3, P->stream);
    double rz0 = read_scalar(P, SC_RZ);
    launch_cast<double, double>(P->n, P->vz, P->vp, P->stream);
    std::vector<double> alphas, betas;
    for (int j = 0; j < steps; ++j) {
        op_apply<double>(P, P->vp, P->vq);
        nb = launch_dot_partial(P->n, P->vp, P->vq, P->partials, P->stream);
        launch_finalize(nb, P->partials, P->scal, 1, P->stream);
        nb = launch_pcg_xr(P->n, P->vt, P->vr, P->vp, P->vq, P->scal, P->partials, P->stream);
        double alpha = read_scalar(P, SC_ALPHA);
        precond(P, P->vr, P->vz, 1);
        nb = launch_dot_partial(P->n, P->vr, P->vz, P->partials, P->stream);
        launch_finalize(nb, P->partials, P->scal, 2, P->stream);
        double beta = read_scalar(P, SC_BETA);
        double rz = read_scalar(P, SC_RZNEW);
        alphas.push_back(alpha);
        betas.push_back(beta);
        if (!(alpha > 0) || !std::isfinite(alpha)) throw Error(VSR_ENOCONV, "Lanczos breakdown");
        if (rz <= 1e-28 * rz0) break;
        launch_pcg_p(P->n, P->vp, P->vz, P->scal, P->stream);
    }
    int k = (int)alphas.size();
    std::vector<double> dg(k), of(std::max(k - 1, 0));
    for (int j = 0; j < k; ++j) {
        dg[j] = 1.0 / alphas[j] + (j ? betas[j - 1] / alphas[j - 1] : 0.0);
        if (j + 1 < k) of[j] = std::sqrt(betas[j]) / alphas[j];
    }
    tridiag_extremes(dg, of, P->lmin, P->lmax);
    const double a = 0.25;
    P->omega = 2.0 / ((1 + a) * P->lmax + (1 - a) * P->lmin);
}

Table make_table(vsr_problem *P, const AxisTable &t) {
    Table r;
    r.n_out = t.n_out;
    r.n_in = t.n_in;
    r.rowptr = P->upload(t.rowptr);
    r.col = P->upload(t.col);
    r.w64 = P->upload(t.w);
    r.w32 = P->upload_as<float>(t.w);
    return r;
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
        // 1D data and geometry
        P->od = make_1d(p, qdef);
        Geometry g = make_geometry(nx, ny, nz, mesh->vertices, kappa, P->od, false);
        P->cartesian = g.cartesian;
        if (kappa)
            for (int64_t e = 0; e < P->ncell; ++e)
                if (!(kappa[e] > 0)) throw Error(VSR_ENOTSPD, "kappa must be positive");
        int n1 = p + 1;
        std::vector<double> ab(2 * n1 * n1), idq(2 * (size_t)qdef * n1);
        std::copy(P->od.A.begin(), P->od.A.end(), ab.begin());
        std::copy(P->od.B.begin(), P->od.B.end(), ab.begin() + n1 * n1);
        std::copy(P->od.Iq.begin(), P->od.Iq.end(), idq.begin());
        std::copy(P->od.Dq.begin(), P->od.Dq.end(), idq.begin() + (size_t)qdef * n1);
        P->AB64 = P->upload(ab);
        P->AB32 = P->upload_as<float>(ab);
        P->IDq64 = P->upload(idq);
        P->IDq32 = P->upload_as<float>(idq);
        P->mu64 = P->upload(g.mu);
        P->mu32 = P->upload_as<float>(g.mu);
        P->wdet = P->upload(g.wdet);
        if (!g.cartesian) {
            P->Gw64 = P->upload(g.Gw);
            if (P->fp32) P->Gw32 = P->upload_as<float>(g.Gw);
        }
        // patches (separable surrogate, Sec. 2.7)
        std::vector<double> mu_sur = muo ? std::vector<double>(muo, muo + 3 * P->ncell) : g.mu;
        for (double v : mu_sur)
            if (!(v > 0)) throw Error(VSR_ENOTSPD, "surrogate scalings must be positive");
        PatchSet S = make_patches(nx, ny, nz, P->od, mu_sur.data(), P->opt.interior_patches_only != 0);
        P->n_int = (int)(S.interior_vertices.size() / 3);
        P->n_bnd = (int)S.boundary_off.size();
        P->verts = P->upload(S.interior_vertices);
        P->bdesc = P->upload(S.boundary_desc);
        P->boff = P->upload(S.boundary_off);
        const InteriorLayout &L = S.L;
        PatchArgs &a = P->pa;
        a.m = L.m; a.w = L.w; a.n_leaf = L.n_leaf; a.n_sep = L.n_sep; a.n_top = L.n_top; a.n_iface = L.n_iface;
        a.top_pad = L.top_pad; a.ntiles = L.ntiles;
        a.off_invd = L.off_invd; a.off_B1 = L.off_B1; a.off_B2 = L.off_B2; a.off_Lsep = L.off_Lsep; a.off_P = L.off_P;
        a.off_Ltop = L.off_Ltop; a.stride = L.stride;
        int m = L.m, w = L.w;
        int64_t per_patch = (int64_t)L.n_leaf + 2LL * 4 * m * m * w + 2LL * m * w * (w + 1) / 2 +
                            2LL * m * w * L.n_top + (int64_t)L.n_top * (L.n_top + 1) / 2;
        int64_t bnd_nnz = 0;
        for (int i = 0; i < P->n_bnd; ++i) {
            int ns = S.boundary_desc[8 * i + 7], nsl = S.boundary_desc[8 * i + 6];
            bnd_nnz += (int64_t)nsl * ns * (ns + 1) / 2;
        }
        P->factor_entries = per_patch * P->n_int + bnd_nnz;
        size_t esz = P->fp32 ? sizeof(float) : sizeof(double);
        P->bytes_patch_launch = (double)esz * (double)P->n_int * (2.0 * per_patch + 2.0 * (double)w * w * w);
        if (P->fp32) upload_patch_data<float>(P.get(), S, mu_sur);
        else upload_patch_data<double>(P.get(), S, mu_sur);
        // transfer tables
        int nc3[3] = {nx, ny, nz};
        for (int ax = 0; ax < 3; ++ax) {
            P->tab[0][ax] = make_table(P.get(), table_fdm_restrict(nc3[ax], P->od));
            P->tab[1][ax] = make_table(P.get(), table_fdm_prolong(nc3[ax], P->od));
            P->tab[2][ax] = make_table(P.get(), table_coarse_restrict(nc3[ax], P->od));
            P->tab[3][ax] = make_table(P.get(), table_coarse_prolong(nc3[ax], P->od));
            P->cdim[ax] = nc3[ax] - 1;
        }
        // coarse space
        std::vector<double> A0inv = make_coarse_inverse(nx, ny, nz, P->od, g);
        P->nc = P->cdim[0] * P->cdim[1] * P->cdim[2];
        P->A0inv = P->fp32 ? (void *)P->upload_as<float>(A0inv) : (void *)P->upload(A0inv);
        // work buffers
        size_t es = esz;
        int64_t w3 = (int64_t)w * w * w;
        auto alloc_t = [&](int64_t cnt) -> void * {
            return P->fp32 ? (void *)P->dalloc<float>(cnt) : (void *)P->dalloc<double>(cnt);
        };
        (void)es;
        P->t1 = alloc_t(P->n);
        P->t2 = alloc_t(P->n);
        P->rF = alloc_t(P->n);
        P->zF = alloc_t(P->n);
        P->U = alloc_t(nv * w3);
        P->z1 = alloc_t(P->n);
        P->az = alloc_t(P->n);
        P->c1 = alloc_t((int64_t)P->cdim[0] * P->d.Ly * P->d.Lz);
        P->c2 = alloc_t((int64_t)P->cdim[0] * P->cdim[1] * P->d.Lz);
        P->c3 = alloc_t(P->nc);
        P->c4 = alloc_t(P->nc);
        P->vp = P->dalloc<double>(P->n);
        P->vq = P->dalloc<double>(P->n);
        P->vr = P->dalloc<double>(P->n);
        P->vz = P->dalloc<double>(P->n);
        P->vt = P->dalloc<double>(P->n);
        P->scal = P->dalloc<double>(SC_N);
        P->partials = P->dalloc<double>(1024);
        VSR_HIP(hipHostMalloc((void **)&P->host_scal, sizeof(double) * SC_N, hipHostMallocDefault));
        if (P->fp32) launch_fill<float>(nv * w3, (float *)P->U, 0.f, P->stream);
        else launch_fill<double>(nv * w3, (double *)P->U, 0.0, P->stream);
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
        launch_fill<double>(P->n, b, 0.0, P->stream);
        launch_load_vector(P->d, P->IDq64, P->wdet, f, b, P->stream);
        VSR_HIP(hipGetLastError());
    });
}

vsr_status vsr_apply_operator(vsr_problem *P, const double *x, double *y) {
    return guarded([&] {
        if (!P || !x || !y) throw Error(VSR_EINVAL, "NULL argument");
        op_apply<double>(P, x, y);
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
        double t0 = now_s();
        int maxit = P->opt.max_iterations > 0 ? P->opt.max_iterations : 1000;
        int64_t n = P->n;
        hipStream_t s = P->stream;
        launch_fill<double>(n, x, 0.0, s);
        launch_cast<double, double>(n, b, P->vr, s);
        int nb = launch_dot_partial(n, b, b, P->partials, s);
        launch_finalize(nb, P->partials, P->scal, 4, s);
        double bb = read_scalar(P, SC_RR);
        if (!std::isfinite(bb)) throw Error(VSR_EINVAL, "non-finite right-hand side");
        double bn = std::sqrt(bb), rn = bn;
        int it = 0;
        bool conv = bn == 0.0;
        if (!conv) {
            precond(P, P->vr, P->vz, 0);
            nb = launch_dot_partial(n, P->vr, P->vz, P->partials, s);
            launch_finalize(nb, P->partials, P->scal, 3, s);
            launch_cast<double, double>(n, P->vz, P->vp, s);
            while (it < maxit) {
                op_apply<double>(P, P->vp, P->vq);
                nb = launch_dot_partial(n, P->vp, P->vq, P->partials, s);
                launch_finalize(nb, P->partials, P->scal, 1, s);
                nb = launch_pcg_xr(n, x, P->vr, P->vp, P->vq, P->scal, P->partials, s);
                launch_finalize(nb, P->partials, P->scal, 4, s);
                ++it;
                double rr = read_scalar(P, SC_RR);
                rn = std::sqrt(rr);
                if (!std::isfinite(rn)) break;
                if (rn <= rtol * bn) {
                    conv = true;
                    break;
                }
                precond(P, P->vr, P->vz, 0);
                nb = launch_dot_partial(n, P->vr, P->vz, P->partials, s);
                launch_finalize(nb, P->partials, P->scal, 2, s);
                launch_pcg_p(n, P->vp, P->vz, P->scal, s);
            }
        }
        VSR_HIP(hipStreamSynchronize(s));
        double t1 = now_s();
        // true residual in FP64
        op_apply<double>(P, x, P->vq);
        launch_residual<double>(n, b, P->vq, P->vt, s);
        double tr = std::sqrt(std::max(0.0, dot(P, P->vt, P->vt)));
        loc.iterations = it;
        loc.converged = conv ? 1 : 0;
        loc.rel_residual = bn > 0 ? rn / bn : 0.0;
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

void vsr_destroy(vsr_problem *P) { delete P; }

const char *vsr_last_error(void) { return vsr::g_last_error_text.c_str(); }

}  // extern "C"
