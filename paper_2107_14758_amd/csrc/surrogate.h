// Launch wrappers of the learned-surrogate kernels (surrogate.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vsr {

int mlp_num_params();
void launch_features(int ncell, const double *corners, const double *kappa, int q, const double *xq, const double *wq,
                     float *feat, double *mu_avg, hipStream_t s);
void launch_ratio(int ncell, const double *corners, const double *mu, double *ratio, hipStream_t s);
void launch_labels(int ncell, const double *corners, const double *mu_avg, double *delta, double *ratio, hipStream_t s);
void launch_mlp_forward(const float *P, int bf16, const float *X, int64_t n, float *Y, hipStream_t s);
void launch_mlp_grad(const float *P, int bf16, const float *X, const float *T, const int *idx, int64_t s_begin, int nbatch,
                     float *gpart, float *lpart, float *grad, float *loss, hipStream_t s);
void launch_adam(float *P, float *m, float *v, const float *g, float lr, float b1t, float b2t, hipStream_t s);

}  // namespace vsr
