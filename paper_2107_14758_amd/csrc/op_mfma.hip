// General (trilinear) cell operator on the matrix cores (gfx950 MFMA 16x16x4, FP64 or FP32).
//
// y_K = (grad phi)^T G w (grad phi) x_K with the q^3 GLL rule (Sec. 2.1, 2.7), sum-factorized
// plane by plane along the reference z axis:
//   Z1 = I_z x, DZ1 = D_z x                 one quadrature plane c at a time, on the vector
//                                            units: thread (j, i) holds the cell's z-column
//                                            x[.][j][i] and its output column y[.][j][i]
//   T1 = Z1 I_x^T, T2 = Z1 D_x^T, T3 = DZ1 I_x^T          (j x a)   MFMA
//   ux = I_y T2, uy = D_y T1, uz = I_y T3                 (b x a)   MFMA
//   v = G(a, b, c) u at every point of the plane          vector units
//   S1 = I_y^T vx, S2 = D_y^T vy, S3 = I_y^T vz           (j x a)   MFMA
//   P1 = S1 D_x + S2 I_x, P2 = S3 I_x                     (j x i)   MFMA
//   y[k] += I_z[c][k] P1 + D_z[c][k] P2                   vector units
// The metric G = w kappa |det J| J^{-1} J^{-T} is evaluated in the kernel from the cell's
// corner edge differences (the same tables and formulas as the vector-unit kernel).  Every
// contraction of the x and y directions is a product of 16 x 16 tiles with K = 4 steps, the
// 1-D matrices I, D (q x (p+1)) zero-padded to whole tiles; the tiles pass through LDS.
#include "device_common.h"

namespace vsr {
namespace dev {
namespace {

typedef double mf64x4 __attribute__((ext_vector_type(4)));
typedef float mf32x4 __attribute__((ext_vector_type(4)));

// One 16x16x4 product-accumulate per wave.  Operands (measured on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; result register r of lane l is D[row(l, r)][l % 16]
// with row = l/16 + 4 r for FP64 and 4 (l/16) + r for FP32.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    using acc = mf64x4;
    static __device__ __forceinline__ acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    using acc = mf32x4;
    static __device__ __forceinline__ acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

constexpr int up4(int n) { return (n + 3) / 4 * 4; }

// C (16 x 16 tile) = sum over the NS steps k0 = 4 s of A(m, k) B(k, n), with A(m, k) =
// a[m sam + k sak] and B(k, n) = b[k sbk + n sbn]; C(m, n) is stored at c[m ldc + n].
template <typename T, int NS>
__device__ __forceinline__ void tile(const T *a, int sam, int sak, const T *b, int sbk, int sbn, T *c, int ldc, int lane) {
    using M = Mfma<T>;
    typename M::acc acc = {0, 0, 0, 0};
    const int lm = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int s = 0; s < NS; ++s) acc = M::mma(a[lm * sam + (4 * s + lk) * sak], b[(4 * s + lk) * sbk + lm * sbn], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) c[M::row(lane, r) * ldc + lm] = acc[r];
}

// Two tiles sharing B: C0 = A0 B and C1 = A1 B, interleaved (two independent chains).
template <typename T, int NS>
__device__ __forceinline__ void tile2(const T *a0, const T *a1, int sam, int sak, const T *b, int sbk, int sbn, T *c0,
                                      T *c1, int ldc, int lane) {
    using M = Mfma<T>;
    typename M::acc x0 = {0, 0, 0, 0}, x1 = {0, 0, 0, 0};
    const int lm = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const T bv = b[(4 * s + lk) * sbk + lm * sbn];
        x0 = M::mma(a0[lm * sam + (4 * s + lk) * sak], bv, x0);
        x1 = M::mma(a1[lm * sam + (4 * s + lk) * sak], bv, x1);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        c0[M::row(lane, r) * ldc + lm] = x0[r];
        c1[M::row(lane, r) * ldc + lm] = x1[r];
    }
}

// Six waves: wave w owns quantity g = w / 2 and the 16-wide a-tile h = w % 2 of both
// x-y passes, so each pass's second product reads only the tile its own wave stored.
constexpr int MW = 6, MTH = 64 * MW;

// S workgroups per cell split the quadrature planes; workgroup s writes its partial
// (p+1)^3 block to slot s of E.  Degrees 10 to 15 (q = 17 .. 24: two tiles along q).
template <typename T, int P, int S>
__global__ void __launch_bounds__(MTH) k_op_general_mfma(const double *__restrict__ gate, Dims d, const T *__restrict__ IDq,
                                                          const T *__restrict__ geo, const T *__restrict__ x, T *__restrict__ E) {
    if (gated(gate)) return;
    constexpr int N1 = P + 1, Q = QOF(P), QP = 32;
    constexpr int NK = up4(N1) / 4, QK = up4(Q) / 4;   // K steps along p + 1 and along q
    constexpr int QK1 = QK - 4;                          // K steps inside the second q-tile
    constexpr int LN = 17, LQ = QP + 1;                  // LDS row strides (odd: no bank conflicts)
    static_assert(N1 <= 16 && Q > 16 && Q <= QP, "degrees 10 to 15");
    // 1-D matrices [a][i] (I, D), zero beyond q rows and p + 1 columns
    __shared__ T sI[QP * LN], sD[QP * LN];
    __shared__ T sP[6 * 16 * LN];    // the six partial tiles of P1 (4) and P2 (2) [j][i]; the first
                                     // two also hold Z1, DZ1 of the next plane
    __shared__ T sT[3 * 16 * LQ];    // T1, T2, T3 [j][a]; then S1, S2, S3
    __shared__ T sU[3 * QP * LQ];    // ux, uy, uz [b][a]; then vx, vy, vz
    __shared__ T sE1[6 * Q], sE2[6 * Q], sA3[6 * Q], sW[Q], sX[Q];
    T *const sZ = sP;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = w >> 1, h = w & 1;
    const int64_t e = blockIdx.x / S;
    const int s = (int)(blockIdx.x % S);
    constexpr int CS = (Q + S - 1) / S;
    const int cb = s * CS, ce = min(Q, cb + CS);
    for (int t = tid; t < QP * LN; t += MTH) {
        const int a = t / LN, i = t % LN;
        const bool in = a < Q && i < N1;
        sI[t] = in ? IDq[a * N1 + i] : T(0);
        sD[t] = in ? IDq[Q * N1 + a * N1 + i] : T(0);
    }
    for (int t = tid; t < 2 * 16 * LN; t += MTH) sZ[t] = T(0);
    {
        const T *cg = geo + e * kGeoStride, *xq = IDq + 2 * Q * N1;
        for (int t = tid; t < 6 * Q; t += MTH) {
            const int r = t / Q, qq = t % Q, cc = r / 3, dd = r % 3;
            const T n0 = T(0.5) * (T(1) - xq[qq]), n1 = T(0.5) * (T(1) + xq[qq]);
            sE1[t] = n0 * cg[(cc * 2 + 0) * 3 + dd] + n1 * cg[(cc * 2 + 1) * 3 + dd];
            sE2[t] = n0 * cg[12 + (cc * 2 + 0) * 3 + dd] + n1 * cg[12 + (cc * 2 + 1) * 3 + dd];
            sA3[t] = n0 * cg[24 + (cc * 2 + 0) * 3 + dd] + n1 * cg[24 + (cc * 2 + 1) * 3 + dd];
        }
        for (int t = tid; t < Q; t += MTH) {
            sW[t] = IDq[2 * Q * N1 + Q + t];
            sX[t] = xq[t];
        }
    }
    const T kap = geo[e * kGeoStride + 36];
    const int ex = (int)(e % d.nx), ey = (int)((e / d.nx) % d.ny), ez = (int)(e / ((int64_t)d.nx * d.ny));
    // thread (j, i) of the cell's (p+1)^2 z-columns
    const bool colt = tid < N1 * N1;
    const int j = tid / N1, i = tid % N1;
    T xc[N1], yc[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        const int K = P * ez + k, J = P * ey + j, I = P * ex + i;
        xc[k] = (colt && is_free(d, K, J, I)) ? x[free_index(d, K, J, I)] : T(0);
        yc[k] = T(0);
    }
    // This wave's 1-D factors.  Forward: T_g = Z_(g == 2) Fx_g^T with Fx = (I, D, I), then
    // u = Fy_g T_g into u slot (1, 0, 2)[g] with Fy = (D, I, I).  Back: S_g = By_g^T v_g with
    // By = (I, D, I), then the partial P_gh = S_g[:, tile h] Bx_g[tile h, :] with Bx = (D, I, I).
    const T *Fx = g == 1 ? sD : sI, *Fy = g == 0 ? sD : sI, *By = g == 1 ? sD : sI, *Bx = g == 0 ? sD : sI;
    const int uslot = g == 0 ? 1 : (g == 1 ? 0 : 2), n0 = 16 * h;
    __syncthreads();
    for (int c = cb; c < ce; ++c) {
        // ---- vector units: the previous plane's z back-contraction, this plane's z contraction
        if (colt) {
            const int o = j * LN + i;
            if (c > cb) {
                const T p1 = (sP[o] + sP[16 * LN + o]) + (sP[2 * 16 * LN + o] + sP[3 * 16 * LN + o]);
                const T p2 = sP[4 * 16 * LN + o] + sP[5 * 16 * LN + o];
#pragma unroll
                for (int k = 0; k < N1; ++k) yc[k] += sI[(c - 1) * LN + k] * p1 + sD[(c - 1) * LN + k] * p2;
            }
            T z0 = 0, z1 = 0;
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                z0 += sI[c * LN + k] * xc[k];
                z1 += sD[c * LN + k] * xc[k];
            }
            sZ[o] = z0;
            sZ[16 * LN + o] = z1;
        }
        __syncthreads();
        // ---- forward x then y: T_g[:, h] = Z Fx_g^T, then u[:, h] = Fy_g T_g[:, h] (two b-tiles)
        {
            T *tg = sT + g * 16 * LQ + n0;
            tile<T, NK>(sZ + (g == 2 ? 16 * LN : 0), LN, 1, Fx + n0 * LN, 1, LN, tg, LQ, lane);
            __threadfence_block();
            T *ug = sU + uslot * QP * LQ + n0;
            tile2<T, NK>(Fy, Fy + 16 * LN, LN, 1, tg, LQ, 1, ug, ug + 16 * LQ, LQ, lane);
        }
        __syncthreads();
        // ---- metric at the plane's points: v = w kappa |det J| J^{-1} J^{-T} u  (Sec. 2.7);
        // rows of J^{-1} are cross products of J's columns over det J
        {
            const T zeta = sX[c], nc0 = T(0.5) * (T(1) - zeta), nc1 = T(0.5) * (T(1) + zeta);
            const T wc = kap * sW[c];
            for (int pt = tid; pt < Q * Q; pt += MTH) {
                const int b = pt / Q, a = pt % Q;
                const T eta = sX[b], nb0 = T(0.5) * (T(1) - eta), nb1 = T(0.5) * (T(1) + eta);
                T J1[3], J2[3], J3[3];
#pragma unroll
                for (int dd = 0; dd < 3; ++dd) {
                    J3[dd] = nb0 * sA3[dd * Q + a] + nb1 * sA3[(3 + dd) * Q + a];
                    J1[dd] = nc0 * sE1[dd * Q + b] + nc1 * sE1[(3 + dd) * Q + b];
                    J2[dd] = nc0 * sE2[dd * Q + a] + nc1 * sE2[(3 + dd) * Q + a];
                }
                const T c1[3] = {J2[1] * J3[2] - J2[2] * J3[1], J2[2] * J3[0] - J2[0] * J3[2], J2[0] * J3[1] - J2[1] * J3[0]};
                const T c2[3] = {J3[1] * J1[2] - J3[2] * J1[1], J3[2] * J1[0] - J3[0] * J1[2], J3[0] * J1[1] - J3[1] * J1[0]};
                const T c3[3] = {J1[1] * J2[2] - J1[2] * J2[1], J1[2] * J2[0] - J1[0] * J2[2], J1[0] * J2[1] - J1[1] * J2[0]};
                const T det = J1[0] * c1[0] + J1[1] * c1[1] + J1[2] * c1[2];
                const T sc = sW[a] * sW[b] * wc / det;
                const T gxx = sc * (c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2]);
                const T gyy = sc * (c2[0] * c2[0] + c2[1] * c2[1] + c2[2] * c2[2]);
                const T gzz = sc * (c3[0] * c3[0] + c3[1] * c3[1] + c3[2] * c3[2]);
                const T gxy = sc * (c1[0] * c2[0] + c1[1] * c2[1] + c1[2] * c2[2]);
                const T gxz = sc * (c1[0] * c3[0] + c1[1] * c3[1] + c1[2] * c3[2]);
                const T gyz = sc * (c2[0] * c3[0] + c2[1] * c3[1] + c2[2] * c3[2]);
                T *u = sU + b * LQ + a;
                const T ux = u[0], uy = u[QP * LQ], uz = u[2 * QP * LQ];
                u[0] = gxx * ux + gxy * uy + gxz * uz;
                u[QP * LQ] = gxy * ux + gyy * uy + gyz * uz;
                u[2 * QP * LQ] = gxz * ux + gyz * uy + gzz * uz;
            }
        }
        __syncthreads();
        // ---- back y then x: S_g[:, h] = By_g^T v_g[:, h], then P_gh = S_g[:, h] Bx_g[h, :]
        {
            T *sg = sT + g * 16 * LQ + n0;
            tile<T, QK>(By, 1, LN, sU + g * QP * LQ + n0, LQ, 1, sg, LQ, lane);
            __threadfence_block();
            if (h == 0) tile<T, 4>(sg, LQ, 1, Bx, LN, 1, sP + w * 16 * LN, LN, lane);
            else tile<T, QK1>(sg, LQ, 1, Bx + 16 * LN, LN, 1, sP + w * 16 * LN, LN, lane);
        }
        __syncthreads();
    }
    if (colt) {
        const int o = j * LN + i;
        if (ce > cb) {
            const T p1 = (sP[o] + sP[16 * LN + o]) + (sP[2 * 16 * LN + o] + sP[3 * 16 * LN + o]);
            const T p2 = sP[4 * 16 * LN + o] + sP[5 * 16 * LN + o];
#pragma unroll
            for (int k = 0; k < N1; ++k) yc[k] += sI[(ce - 1) * LN + k] * p1 + sD[(ce - 1) * LN + k] * p2;
        }
        T *Es = E + (int64_t)s * (d.nx * d.ny * d.nz) * (N1 * N1 * N1);
#pragma unroll
        for (int k = 0; k < N1; ++k) Es[elem_index<N1>(d, ex, ey, ez, k, j, i)] = yc[k];
    }
}

}  // namespace
}  // namespace dev

using namespace dev;

template <typename T>
int launch_op_general_mfma(const Dims &d, int split, const T *IDq, const T *geo, const T *x, T *E, const Exec &e) {
    const int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
    if (split != 1 && split != 2) throw Error(VSR_EINVAL, "operator split must be 1 or 2");
    if (d.p < 10) throw Error(VSR_EINVAL, "the matrix-core operator covers degrees 10 to 15");
#define CALLS(P, S) \
    hipLaunchKernelGGL((k_op_general_mfma<T, P, S>), dim3((unsigned)(ncell * S)), dim3(MTH), 0, e.s, e.gate, d, IDq, geo, x, E)
#define CALL(P)                                    \
    {                                              \
        if (split == 2) CALLS(P < 10 ? 10 : P, 2); \
        else CALLS(P < 10 ? 10 : P, 1);            \
    }
    VSR_P_SWITCH(d.p, CALL)
#undef CALL
#undef CALLS
    return split;
}

template int launch_op_general_mfma<double>(const Dims &, int, const double *, const double *, const double *, double *,
                                            const Exec &);
template int launch_op_general_mfma<float>(const Dims &, int, const float *, const float *, const float *, float *,
                                           const Exec &);

}  // namespace vsr
