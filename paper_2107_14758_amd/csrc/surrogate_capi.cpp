// C ABI of the learned separable surrogate (include/vsr.h): features, Theorem-1 ratios,
// minimax labels, and the MLP's inference, gradient and Adam training on the GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "surrogate.h"
#include "vsr_internal.h"

using namespace vsr;

namespace vsr {
extern thread_local std::string g_last_error_text;
}

namespace {

template <typename F>
vsr_status run(F &&f) {
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

// Device buffer released at scope exit.
template <typename T>
struct DBuf {
    T *p = nullptr;
    explicit DBuf(size_t n) {
        if (hipMalloc((void **)&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
            throw Error(VSR_ENOMEM, "device allocation failed");
    }
    ~DBuf() {
        if (p) (void)hipFree(p);
    }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
};

template <typename T>
void h2d(T *d, const T *h, size_t n) {
    VSR_HIP(hipMemcpy(d, h, n * sizeof(T), hipMemcpyHostToDevice));
}
template <typename T>
void d2h(T *h, const T *d, size_t n) {
    VSR_HIP(hipMemcpy(h, d, n * sizeof(T), hipMemcpyDeviceToHost));
}

void check_cells(int64_t ncell, const double *corners) {
    if (ncell < 0 || (ncell > 0 && !corners)) throw Error(VSR_EINVAL, "bad cell arguments");
    if (ncell > (int64_t)1 << 30) throw Error(VSR_EINVAL, "too many cells");
    for (int64_t i = 0; i < 24 * ncell; ++i)
        if (!std::isfinite(corners[i])) throw Error(VSR_EINVAL, "non-finite corner coordinate");
}

// features + mu_avg (kappa = 1) for host cells; optional outputs
void features_and_mu(int64_t ncell, const double *corners, const double *kappa, int p, float *feat_dev,
                     std::vector<double> &mu_avg) {
    int q = (3 * (p + 1) + 1) / 2;
    OneD od = make_1d(p, q);
    DBuf<double> dc(24 * ncell), dk(ncell), dxq(q), dwq(q), dmu(3 * ncell);
    DBuf<float> dfeat(feat_dev ? 1 : 74 * ncell);
    h2d(dc.p, corners, 24 * ncell);
    if (kappa) h2d(dk.p, kappa, ncell);
    h2d(dxq.p, od.xq.data(), q);
    h2d(dwq.p, od.wq.data(), q);
    launch_features((int)ncell, dc.p, kappa ? dk.p : nullptr, q, dxq.p, dwq.p, feat_dev ? feat_dev : dfeat.p, dmu.p, nullptr);
    VSR_HIP(hipGetLastError());
    mu_avg.resize(3 * ncell);
    d2h(mu_avg.data(), dmu.p, 3 * ncell);
}

}  // namespace

extern "C" {

int32_t vsr_mlp_num_params(void) { return mlp_num_params(); }

vsr_status vsr_surrogate_features(int64_t ncell, const double *corners, const double *kappa, int32_t p, float *features_dev,
                                  double *mu_avg) {
    return run([&] {
        check_cells(ncell, corners);
        if (p < 2 || p > 15) throw Error(VSR_EINVAL, "p must be in [2, 15]");
        if (ncell == 0) return;
        std::vector<double> mu;
        features_and_mu(ncell, corners, kappa, p, features_dev, mu);
        if (mu_avg) std::memcpy(mu_avg, mu.data(), mu.size() * sizeof(double));
    });
}

vsr_status vsr_surrogate_ratio(int64_t ncell, const double *corners, const double *mu, double *ratio) {
    return run([&] {
        check_cells(ncell, corners);
        if (!mu || !ratio) throw Error(VSR_EINVAL, "NULL argument");
        if (ncell == 0) return;
        for (int64_t i = 0; i < 3 * ncell; ++i)
            if (!(mu[i] > 0)) throw Error(VSR_EINVAL, "scalings must be positive");
        DBuf<double> dc(24 * ncell), dm(3 * ncell), dr(ncell);
        h2d(dc.p, corners, 24 * ncell);
        h2d(dm.p, mu, 3 * ncell);
        launch_ratio((int)ncell, dc.p, dm.p, dr.p, nullptr);
        VSR_HIP(hipGetLastError());
        d2h(ratio, dr.p, ncell);
    });
}

vsr_status vsr_surrogate_labels(int64_t ncell, const double *corners, int32_t p, double *delta, double *ratio) {
    return run([&] {
        check_cells(ncell, corners);
        if (!delta) throw Error(VSR_EINVAL, "NULL argument");
        if (p < 2 || p > 15) throw Error(VSR_EINVAL, "p must be in [2, 15]");
        if (ncell == 0) return;
        std::vector<double> mu;
        features_and_mu(ncell, corners, nullptr, p, nullptr, mu);
        DBuf<double> dc(24 * ncell), dm(3 * ncell), dd(3 * ncell), dr(ncell);
        h2d(dc.p, corners, 24 * ncell);
        h2d(dm.p, mu.data(), 3 * ncell);
        launch_labels((int)ncell, dc.p, dm.p, dd.p, dr.p, nullptr);
        VSR_HIP(hipGetLastError());
        d2h(delta, dd.p, 3 * ncell);
        if (ratio) d2h(ratio, dr.p, ncell);
    });
}

vsr_status vsr_mlp_forward(const float *params, int32_t bf16, const float *X, int64_t n, float *Y) {
    return run([&] {
        if (!params || (n > 0 && (!X || !Y)) || n < 0) throw Error(VSR_EINVAL, "bad argument");
        launch_mlp_forward(params, bf16, X, n, Y, nullptr);
        VSR_HIP(hipGetLastError());
        VSR_HIP(hipDeviceSynchronize());
    });
}

vsr_status vsr_mlp_gradient(const float *params, int32_t bf16, const float *X, const float *T, int64_t n, float *grad,
                            float *loss) {
    return run([&] {
        if (!params || !X || !T || !grad || n <= 0 || n > (1 << 30)) throw Error(VSR_EINVAL, "bad argument");
        int ntile = (int)((n + 15) / 16);
        DBuf<float> gpart((size_t)ntile * mlp_num_params()), lpart(ntile);
        launch_mlp_grad(params, bf16, X, T, nullptr, 0, (int)n, gpart.p, lpart.p, grad, loss, nullptr);
        VSR_HIP(hipGetLastError());
        VSR_HIP(hipDeviceSynchronize());
    });
}

vsr_status vsr_mlp_train(float *params, float *adam_m, float *adam_v, int32_t bf16, const float *X, const float *T,
                         int64_t n, const int32_t *order, int32_t batch, int32_t steps, int32_t step0, float lr,
                         float *loss) {
    return run([&] {
        if (!params || !adam_m || !adam_v || !X || !T || !order || batch <= 0 || steps < 0 || step0 < 0 || n <= 0)
            throw Error(VSR_EINVAL, "bad argument");
        int ntile = (batch + 15) / 16;
        DBuf<float> gpart((size_t)ntile * mlp_num_params()), lpart(ntile), grad(mlp_num_params());
        for (int s = 0; s < steps; ++s) {
            int t = step0 + s + 1;
            launch_mlp_grad(params, bf16, X, T, order, (int64_t)s * batch, batch, gpart.p, lpart.p, grad.p,
                            loss ? loss + s : nullptr, nullptr);
            launch_adam(params, adam_m, adam_v, grad.p, lr, (float)std::pow(0.9, t), (float)std::pow(0.999, t), nullptr);
        }
        VSR_HIP(hipGetLastError());
        VSR_HIP(hipDeviceSynchronize());
    });
}

vsr_status vsr_surrogate_scalings(int64_t ncell, const double *corners, const double *kappa, int32_t p, const float *params,
                                  int32_t bf16, double *mu_out, int32_t *learned) {
    return run([&] {
        check_cells(ncell, corners);
        if (!params || !mu_out) throw Error(VSR_EINVAL, "NULL argument");
        if (p < 2 || p > 15) throw Error(VSR_EINVAL, "p must be in [2, 15]");
        if (ncell == 0) return;
        DBuf<float> feat(74 * ncell), y(3 * ncell);
        std::vector<double> mu;
        features_and_mu(ncell, corners, kappa, p, feat.p, mu);
        launch_mlp_forward(params, bf16, feat.p, ncell, y.p, nullptr);
        VSR_HIP(hipGetLastError());
        std::vector<float> yh(3 * ncell);
        d2h(yh.data(), y.p, 3 * ncell);
        std::vector<double> mul(3 * ncell);
        for (int64_t i = 0; i < 3 * ncell; ++i) {
            double d = std::fmin(4.0, std::fmax(-4.0, (double)yh[i]));
            mul[i] = mu[i] * std::exp(d);
        }
        std::vector<double> r0(ncell), r1(ncell);
        DBuf<double> dc(24 * ncell), dm(3 * ncell), dr(ncell);
        h2d(dc.p, corners, 24 * ncell);
        h2d(dm.p, mu.data(), 3 * ncell);
        launch_ratio((int)ncell, dc.p, dm.p, dr.p, nullptr);
        d2h(r0.data(), dr.p, ncell);
        h2d(dm.p, mul.data(), 3 * ncell);
        launch_ratio((int)ncell, dc.p, dm.p, dr.p, nullptr);
        d2h(r1.data(), dr.p, ncell);
        VSR_HIP(hipGetLastError());
        for (int64_t e = 0; e < ncell; ++e) {
            bool use = r1[e] < r0[e];
            double k = kappa ? kappa[e] : 1.0;
            for (int j = 0; j < 3; ++j) mu_out[3 * e + j] = k * (use ? mul[3 * e + j] : mu[3 * e + j]);
            if (learned) learned[e] = use ? 1 : 0;
        }
    });
}

}  // extern "C"
