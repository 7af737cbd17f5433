// Learned separable surrogate (extension of Sec. 2.7): per-cell geometry features,
// Theorem-1 spectral ratio of a diagonal scaling, minimax labels, and a small MLP
// (74 -> 64 -> 64 -> 3, GELU) with forward, backward and Adam kernels.
//
// Cells are given by their 8 corners, corner (a,b,c) in {0,1}^3 (x fastest) at
// corners[cell*24 + ((c*2+b)*2+a)*3 + coord].  The reference cell is [-1,1]^3.
#include <hip/hip_runtime.h>

#include <cmath>

#include "surrogate.h"
#include "vsr_internal.h"

namespace vsr {
namespace {

// DF at reference point (x, y, z): J[i][j] = dx_i / dxi_j for the trilinear map.
__device__ void jac(const double *X, double x, double y, double z, double J[3][3]) {
    double N[3][2] = {{0.5 * (1 - x), 0.5 * (1 + x)}, {0.5 * (1 - y), 0.5 * (1 + y)}, {0.5 * (1 - z), 0.5 * (1 + z)}};
    const double dN[2] = {-0.5, 0.5};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[i][j] = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const double *P = X + ((c * 2 + b) * 2 + a) * 3;
                double g0 = dN[a] * N[1][b] * N[2][c], g1 = N[0][a] * dN[b] * N[2][c], g2 = N[0][a] * N[1][b] * dN[c];
                for (int i = 0; i < 3; ++i) {
                    J[i][0] += g0 * P[i];
                    J[i][1] += g1 * P[i];
                    J[i][2] += g2 * P[i];
                }
            }
}

__device__ double det3(const double J[3][3]) {
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// |det J| J^{-1} J^{-T} = adj(J) adj(J)^T / |det J| (symmetric; g = xx, yy, zz, xy, xz, yz)
__device__ void metric(const double J[3][3], double g[6]) {
    double A[3][3];  // adjugate: J^{-1} = A / det
    A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    double d = fabs(det3(J));
    auto dot = [&](int r, int s) { return (A[r][0] * A[s][0] + A[r][1] * A[s][1] + A[r][2] * A[s][2]) / d; };
    g[0] = dot(0, 0);
    g[1] = dot(1, 1);
    g[2] = dot(2, 2);
    g[3] = dot(0, 1);
    g[4] = dot(0, 2);
    g[5] = dot(1, 2);
}

// Extreme eigenvalues of a symmetric 3x3 matrix by the trigonometric closed form.
__device__ void eig3_extremes(const double a[6], double &lmin, double &lmax) {
    double p1 = a[3] * a[3] + a[4] * a[4] + a[5] * a[5];
    if (p1 == 0.0) {
        lmin = fmin(a[0], fmin(a[1], a[2]));
        lmax = fmax(a[0], fmax(a[1], a[2]));
        return;
    }
    double q = (a[0] + a[1] + a[2]) / 3.0;
    double d0 = a[0] - q, d1 = a[1] - q, d2 = a[2] - q;
    double p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * p1;
    double p = sqrt(p2 / 6.0);
    double b0 = d0 / p, b1 = d1 / p, b2 = d2 / p, b3 = a[3] / p, b4 = a[4] / p, b5 = a[5] / p;
    double r = 0.5 * (b0 * (b1 * b2 - b5 * b5) - b3 * (b3 * b2 - b5 * b4) + b4 * (b3 * b5 - b1 * b4));
    r = fmin(1.0, fmax(-1.0, r));
    double phi = acos(r) / 3.0;
    lmax = q + 2.0 * p * cos(phi);
    lmin = q + 2.0 * p * cos(phi + 2.0943951023931957);
}

__device__ double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// ratio C/c of mu^{-1/2} G mu^{-1/2} over the 27 sample points held one per lane (lanes >= 27 idle)
__device__ void bounds_at(const double g[6], bool active, const double mu[3], double &c, double &C) {
    double lo = 1e300, hi = -1e300;
    if (active) {
        double s0 = 1.0 / sqrt(mu[0]), s1 = 1.0 / sqrt(mu[1]), s2 = 1.0 / sqrt(mu[2]);
        double m[6] = {g[0] * s0 * s0, g[1] * s1 * s1, g[2] * s2 * s2, g[3] * s0 * s1, g[4] * s0 * s2, g[5] * s1 * s2};
        eig3_extremes(m, lo, hi);
    }
    c = wave_min(lo);
    C = wave_max(hi);
}

// Per cell (one wavefront): features, the q-point average mu of diag(G) (kappa = 1), and the
// metric at the 27 sample points xi in {-1,0,1}^3.
__device__ void sample_metric(const double *X, int lane, double g[6]) {
    if (lane < 27) {
        double x = (lane % 3) - 1.0, y = ((lane / 3) % 3) - 1.0, z = (lane / 9) - 1.0;
        double J[3][3];
        jac(X, x, y, z, J);
        metric(J, g);
    } else {
        for (int i = 0; i < 6; ++i) g[i] = 0.0;
    }
}

// geometric features are centred on the undistorted cube and scaled to about unit spread
constexpr double kFeatureGain = 8.0;

__global__ void k_features(int ncell, const double *__restrict__ corners, const double *__restrict__ kappa, int q,
                           const double *__restrict__ xq, const double *__restrict__ wq, float *__restrict__ feat,
                           double *__restrict__ mu_avg) {
    const int lane = threadIdx.x & 63;
    const int cell = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (cell >= ncell) return;
    const double *X = corners + (int64_t)cell * 24;
    double J0[3][3];
    jac(X, 0.0, 0.0, 0.0, J0);
    double s = cbrt(fabs(det3(J0)));
    if (lane < 72) {
        int gp = lane / 9, ij = lane % 9;
        const double gg = 0.57735026918962576;
        double x = (gp & 1) ? gg : -gg, y = (gp & 2) ? gg : -gg, z = (gp & 4) ? gg : -gg;
        double J[3][3];
        jac(X, x, y, z, J);
        feat[(int64_t)cell * 74 + lane] = (float)(kFeatureGain * (J[ij / 3][ij % 3] / s - (ij % 4 == 0 ? 1.0 : 0.0)));
    }
    if (lane < 8) {  // the remaining 8 of the 72 entries (lanes 64..71 do not exist)
        int e = 64 + lane, gp = e / 9, ij = e % 9;
        const double gg = 0.57735026918962576;
        double x = (gp & 1) ? gg : -gg, y = (gp & 2) ? gg : -gg, z = (gp & 4) ? gg : -gg;
        double J[3][3];
        jac(X, x, y, z, J);
        feat[(int64_t)cell * 74 + e] = (float)(kFeatureGain * (J[ij / 3][ij % 3] / s - (ij % 4 == 0 ? 1.0 : 0.0)));
    }
    if (lane == 0) {
        feat[(int64_t)cell * 74 + 72] = (float)(kappa ? log(kappa[cell]) : 0.0);
        feat[(int64_t)cell * 74 + 73] = 0.0f;
    }
    // mu_avg = (1/8) sum_q w_q diag(G) over q^3 points, lanes stride the points
    double m0 = 0, m1 = 0, m2 = 0;
    int nq3 = q * q * q;
    for (int t = lane; t < nq3; t += 64) {
        int a = t % q, b = (t / q) % q, c = t / (q * q);
        double J[3][3], g[6];
        jac(X, xq[a], xq[b], xq[c], J);
        metric(J, g);
        double w = wq[a] * wq[b] * wq[c];
        m0 += w * g[0];
        m1 += w * g[1];
        m2 += w * g[2];
    }
    for (int off = 32; off > 0; off >>= 1) {
        m0 += __shfl_xor(m0, off, 64);
        m1 += __shfl_xor(m1, off, 64);
        m2 += __shfl_xor(m2, off, 64);
    }
    if (lane == 0) {
        mu_avg[3 * cell] = m0 / 8.0;
        mu_avg[3 * cell + 1] = m1 / 8.0;
        mu_avg[3 * cell + 2] = m2 / 8.0;
    }
}

__global__ void k_ratio(int ncell, const double *__restrict__ corners, const double *__restrict__ mu,
                        double *__restrict__ ratio) {
    const int lane = threadIdx.x & 63;
    const int cell = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (cell >= ncell) return;
    double g[6];
    sample_metric(corners + (int64_t)cell * 24, lane, g);
    double m[3] = {mu[3 * cell], mu[3 * cell + 1], mu[3 * cell + 2]};
    double c, C;
    bounds_at(g, lane < 27, m, c, C);
    if (lane == 0) ratio[cell] = C / c;
}

// Theorem-1 minimax label: minimise log(C/c) + 1e-6 |delta - mean(delta)|^2 (the small
// term only breaks ties where the ratio is flat) over delta = (a, b, 0) on a coarse-to-fine
// grid (17x17 of step 1/8, then twice 9x9 with the step divided by 4, first minimum in
// row-major order), then shift all components by log(c C)/2.
__global__ void k_labels(int ncell, const double *__restrict__ corners, const double *__restrict__ mu_avg,
                         double *__restrict__ delta, double *__restrict__ ratio) {
    const int lane = threadIdx.x & 63;
    const int cell = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (cell >= ncell) return;
    double g[6];
    sample_metric(corners + (int64_t)cell * 24, lane, g);
    const double m0 = mu_avg[3 * cell], m1 = mu_avg[3 * cell + 1], m2 = mu_avg[3 * cell + 2];
    double ba = 0.0, bb = 0.0, step = 0.125;
    int half = 8;
    for (int level = 0; level < 3; ++level) {
        if (level > 0) {
            step *= 0.25;
            half = 4;
        }
        double best_r = 1e300, na = ba, nb = bb;
        for (int ia = -half; ia <= half; ++ia)
            for (int ib = -half; ib <= half; ++ib) {
                double a = ba + ia * step, b = bb + ib * step;
                double mu[3] = {m0 * exp(a), m1 * exp(b), m2};
                double c, C;
                bounds_at(g, lane < 27, mu, c, C);
                double mm = (a + b) / 3.0;
                double r = log(C / c) + 1e-6 * ((a - mm) * (a - mm) + (b - mm) * (b - mm) + mm * mm);
                if (r < best_r) {
                    best_r = r;
                    na = a;
                    nb = b;
                }
            }
        ba = na;
        bb = nb;
    }
    double mu[3] = {m0 * exp(ba), m1 * exp(bb), m2};
    double c, C;
    bounds_at(g, lane < 27, mu, c, C);
    if (lane == 0) {
        double t = 0.5 * log(c * C);
        delta[3 * cell] = ba + t;
        delta[3 * cell + 1] = bb + t;
        delta[3 * cell + 2] = t;
        ratio[cell] = C / c;
    }
}

// ---------------------------------------------------------------- MLP
constexpr int NIN = 74, NH = 64, NOUT = 3, TILE = 16;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NOUT * NH,
              NPAR = OB3 + NOUT;

__device__ __forceinline__ float to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    return __uint_as_float(u);
}
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

struct MlpShared {
    float w[NPAR];
    float x[TILE * NIN];
    float z1[TILE * NH], h1[TILE * NH], z2[TILE * NH], h2[TILE * NH];
    float y[TILE * NOUT], dy[TILE * NOUT];
};

// forward of one tile of samples (rows idx[s] of X, or s0 + s when idx is NULL)
__device__ void mlp_tile_forward(MlpShared &S, const float *__restrict__ P, int bf16, const float *__restrict__ X,
                                 const int *__restrict__ idx, int64_t s0, int ns) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int j = tid; j < NPAR; j += nt) S.w[j] = bf16 ? to_bf16(P[j]) : P[j];
    for (int e = tid; e < TILE * NIN; e += nt) {
        int s = e / NIN, i = e % NIN;
        int64_t row = s < ns ? (idx ? idx[s0 + s] : s0 + s) : -1;
        S.x[e] = row >= 0 ? X[row * NIN + i] : 0.0f;
    }
    __syncthreads();
    for (int o = tid; o < TILE * NH; o += nt) {
        int s = o / NH, n = o % NH;
        float z = S.w[OB1 + n];
        for (int i = 0; i < NIN; ++i) z += S.w[OW1 + n * NIN + i] * S.x[s * NIN + i];
        S.z1[o] = z;
        S.h1[o] = gelu(z);
    }
    __syncthreads();
    for (int o = tid; o < TILE * NH; o += nt) {
        int s = o / NH, n = o % NH;
        float z = S.w[OB2 + n];
        for (int i = 0; i < NH; ++i) z += S.w[OW2 + n * NH + i] * S.h1[s * NH + i];
        S.z2[o] = z;
        S.h2[o] = gelu(z);
    }
    __syncthreads();
    for (int o = tid; o < TILE * NOUT; o += nt) {
        int s = o / NOUT, k = o % NOUT;
        float z = S.w[OB3 + k];
        for (int i = 0; i < NH; ++i) z += S.w[OW3 + k * NH + i] * S.h2[s * NH + i];
        S.y[o] = z;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_mlp_forward(const float *__restrict__ P, int bf16, const float *__restrict__ X,
                                                     int64_t n, float *__restrict__ Y) {
    extern __shared__ float smem[];
    MlpShared &S = *reinterpret_cast<MlpShared *>(smem);
    int64_t s0 = (int64_t)blockIdx.x * TILE;
    int ns = (int)min<int64_t>(TILE, n - s0);
    mlp_tile_forward(S, P, bf16, X, nullptr, s0, ns);
    for (int o = threadIdx.x; o < ns * NOUT; o += blockDim.x) Y[s0 * NOUT + o] = S.y[o];
}

// Per-tile gradient of the mean-squared loss over `nbatch` samples; writes the tile's
// partial gradient to gpart[tile * NPAR + j] and its partial loss to lpart[tile].
__global__ void __launch_bounds__(256) k_mlp_grad(const float *__restrict__ P, int bf16, const float *__restrict__ X,
                                                  const float *__restrict__ Tt, const int *__restrict__ idx, int64_t s_begin,
                                                  int nbatch, float *__restrict__ gpart, float *__restrict__ lpart) {
    extern __shared__ float smem[];
    MlpShared &S = *reinterpret_cast<MlpShared *>(smem);
    __shared__ float dz[TILE * NH];
    __shared__ float red[256];
    const int tid = threadIdx.x, nt = blockDim.x;
    int t0 = blockIdx.x * TILE;
    int ns = min(TILE, nbatch - t0);
    mlp_tile_forward(S, P, bf16, X, idx, s_begin + t0, ns);
    const float scale = 2.0f / (float)(nbatch * NOUT);
    float lsum = 0.0f;
    for (int o = tid; o < TILE * NOUT; o += nt) {
        int s = o / NOUT;
        float r = 0.0f;
        if (s < ns) {
            int64_t row = idx ? idx[s_begin + t0 + s] : s_begin + t0 + s;
            r = S.y[o] - Tt[row * NOUT + (o % NOUT)];
        }
        S.dy[o] = scale * r;
        lsum += r * r;
    }
    red[tid] = lsum;
    __syncthreads();
    float *g = gpart + (int64_t)blockIdx.x * NPAR;
    // layer 3
    for (int j = tid; j < NOUT * NH; j += nt) {
        int k = j / NH, m = j % NH;
        float a = 0.0f;
        for (int s = 0; s < TILE; ++s) a += S.dy[s * NOUT + k] * S.h2[s * NH + m];
        g[OW3 + j] = a;
    }
    for (int k = tid; k < NOUT; k += nt) {
        float a = 0.0f;
        for (int s = 0; s < TILE; ++s) a += S.dy[s * NOUT + k];
        g[OB3 + k] = a;
    }
    for (int o = tid; o < TILE * NH; o += nt) {
        int s = o / NH, m = o % NH;
        float a = 0.0f;
        for (int k = 0; k < NOUT; ++k) a += S.w[OW3 + k * NH + m] * S.dy[s * NOUT + k];
        dz[o] = a * gelu_d(S.z2[o]);
    }
    __syncthreads();
    // layer 2
    for (int j = tid; j < NH * NH; j += nt) {
        int nn = j / NH, m = j % NH;
        float a = 0.0f;
        for (int s = 0; s < TILE; ++s) a += dz[s * NH + nn] * S.h1[s * NH + m];
        g[OW2 + j] = a;
    }
    for (int nn = tid; nn < NH; nn += nt) {
        float a = 0.0f;
        for (int s = 0; s < TILE; ++s) a += dz[s * NH + nn];
        g[OB2 + nn] = a;
    }
    for (int o = tid; o < TILE * NH; o += nt) {   // dh1 -> z1 slot (z1 is no longer needed after)
        int s = o / NH, m = o % NH;
        float a = 0.0f;
        for (int nn = 0; nn < NH; ++nn) a += S.w[OW2 + nn * NH + m] * dz[s * NH + nn];
        S.h2[o] = a * gelu_d(S.z1[o]);             // h2 reused as dz1
    }
    __syncthreads();
    // layer 1
    for (int j = tid; j < NH * NIN; j += nt) {
        int m = j / NIN, i = j % NIN;
        float a = 0.0f;
        for (int s = 0; s < TILE; ++s) a += S.h2[s * NH + m] * S.x[s * NIN + i];
        g[OW1 + j] = a;
    }
    for (int m = tid; m < NH; m += nt) {
        float a = 0.0f;
        for (int s = 0; s < TILE; ++s) a += S.h2[s * NH + m];
        g[OB1 + m] = a;
    }
    if (tid == 0) {
        float a = 0.0f;
        for (int i = 0; i < nt; ++i) a += red[i];
        lpart[blockIdx.x] = a;
    }
}

// grad[j] = sum over tiles of gpart (fixed order); loss = sum(lpart) / (nbatch * NOUT)
__global__ void k_mlp_reduce(int ntile, int nbatch, const float *__restrict__ gpart, const float *__restrict__ lpart,
                             float *__restrict__ grad, float *__restrict__ loss) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < NPAR) {
        float a = 0.0f;
        for (int t = 0; t < ntile; ++t) a += gpart[(int64_t)t * NPAR + j];
        grad[j] = a;
    }
    if (j == 0 && loss) {
        float a = 0.0f;
        for (int t = 0; t < ntile; ++t) a += lpart[t];
        *loss = a / (float)(nbatch * NOUT);
    }
}

__global__ void k_adam(float *__restrict__ P, float *__restrict__ m, float *__restrict__ v, const float *__restrict__ g,
                       float lr, float b1t, float b2t) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NPAR) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float mj = b1 * m[j] + (1.0f - b1) * g[j];
    float vj = b2 * v[j] + (1.0f - b2) * g[j] * g[j];
    m[j] = mj;
    v[j] = vj;
    float mh = mj / (1.0f - b1t), vh = vj / (1.0f - b2t);
    P[j] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace

int mlp_num_params() { return NPAR; }

void launch_features(int ncell, const double *corners, const double *kappa, int q, const double *xq, const double *wq,
                     float *feat, double *mu_avg, hipStream_t s) {
    unsigned blocks = (unsigned)(((int64_t)ncell * 64 + 255) / 256);
    hipLaunchKernelGGL(k_features, dim3(blocks), dim3(256), 0, s, ncell, corners, kappa, q, xq, wq, feat, mu_avg);
}

void launch_ratio(int ncell, const double *corners, const double *mu, double *ratio, hipStream_t s) {
    unsigned blocks = (unsigned)(((int64_t)ncell * 64 + 255) / 256);
    hipLaunchKernelGGL(k_ratio, dim3(blocks), dim3(256), 0, s, ncell, corners, mu, ratio);
}

void launch_labels(int ncell, const double *corners, const double *mu_avg, double *delta, double *ratio, hipStream_t s) {
    unsigned blocks = (unsigned)(((int64_t)ncell * 64 + 255) / 256);
    hipLaunchKernelGGL(k_labels, dim3(blocks), dim3(256), 0, s, ncell, corners, mu_avg, delta, ratio);
}

void launch_mlp_forward(const float *P, int bf16, const float *X, int64_t n, float *Y, hipStream_t s) {
    if (n == 0) return;
    unsigned blocks = (unsigned)((n + TILE - 1) / TILE);
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(256), sizeof(MlpShared), s, P, bf16, X, n, Y);
}

void launch_mlp_grad(const float *P, int bf16, const float *X, const float *T, const int *idx, int64_t s_begin, int nbatch,
                     float *gpart, float *lpart, float *grad, float *loss, hipStream_t s) {
    int ntile = (nbatch + TILE - 1) / TILE;
    hipLaunchKernelGGL(k_mlp_grad, dim3(ntile), dim3(256), sizeof(MlpShared), s, P, bf16, X, T, idx, s_begin, nbatch, gpart,
                       lpart);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPAR + 255) / 256), dim3(256), 0, s, ntile, nbatch, gpart, lpart, grad, loss);
}

void launch_adam(float *P, float *m, float *v, const float *g, float lr, float b1t, float b2t, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((NPAR + 255) / 256), dim3(256), 0, s, P, m, v, g, lr, b1t, b2t);
}

}  // namespace vsr
