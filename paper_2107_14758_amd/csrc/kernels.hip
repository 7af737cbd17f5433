// HIP kernels for gfx950 (CDNA4, wave64): operator and element-vector gather, load vector,
// patch assembly, dense coarse solve and the PCG vector kernels.  The patch solves live in
// patch_kernels.h, the lattice transfers in transfer.hip.
//
// Method references: Brubeck & Farrell, "A scalable and robust vertex-star relaxation for
// high-order FEM", Sec. 2.
#include "device_common.h"

#include <stdexcept>

namespace vsr {

namespace {
using namespace dev;

// Sum over a workgroup (valid in thread 0), wavefronts added in a fixed order.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[16];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) part[wv] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; ++i) s += part[i];
    return s;
}

// ====================================================================== operator

// Separable (Cartesian) cell operator, eq. (kron) of Sec. 2.2:
// A^K = mu1 B x B x A + mu2 B x A x B + mu3 A x B x B.  Thread (j, i) of a cell owns one
// z-column.  The cell's values are staged KC z-slabs at a time (one global round trip per
// chunk; all slabs at once where they fit); the x and y contractions run through LDS with
// this thread's rows of A and B in registers, and each slab's result is folded at once into
// the column's z contraction (A and B read there at wave-uniform addresses).  The cell's
// (p+1)^3 results go to its block of the element vector E with plain stores; k_gather sums
// the blocks that share a lattice node (no atomics).
template <int P, int BYTES>
constexpr int kron_chunk() {
    constexpr int N1 = P + 1, per = 3 * N1 * N1 * BYTES, kc = (48 * 1024) / per;
    return kc < 1 ? 1 : (kc > N1 ? N1 : kc);
}

// Epilogues of the Cartesian operator.  The residual of the V-cycle is only ever restricted:
// to FDM covectors (T^T) before a relaxation, to the Q1 space (P^T) before the coarse solve.
// Both maps act cell by cell on an assembled vector, T^T sum_K R_K^T y_K = sum_K R_K^T (That^T
// x3) y_K (Sec. 2.4: a node's value depends only on the FDM functions of its cell's closure;
// likewise for the Q1 interpolation), once the entries of y_K at Dirichlet nodes are dropped.
// EPI_FDM stores (That^T x3) y_K in place of y_K (assembled by k_gather into FDM covectors);
// EPI_Q1 stores the 8 corner values (N^T x3) y_K per cell (assembled by k_coarse_gather).
enum { EPI_NONE = 0, EPI_FDM = 1, EPI_Q1 = 2 };

template <typename T, int P, int CPW, int EPI = EPI_NONE>
__global__ void __launch_bounds__(256) k_op_kron(const double *__restrict__ gate, Dims d, const T *__restrict__ AB1d,
                                                 const T *__restrict__ mu, const T *__restrict__ x, T *__restrict__ E) {
    if (gated(gate)) return;
    constexpr int N1 = P + 1, N2 = N1 * N1, KC = kron_chunk<P, (int)sizeof(T) * CPW>(), NCH = (N1 + KC - 1) / KC;
    __shared__ T xs[CPW][KC * N2], as[CPW][KC * N2], bs[CPW][KC * N2];
    const int tid = threadIdx.x;
    // CPW cells per workgroup, N2 threads each
    const int sub = tid / N2, lt = tid - sub * N2;
    const int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
    const int64_t e = (int64_t)blockIdx.x * CPW + sub;
    const bool active = sub < CPW && e < ncell;
    const int64_t ec = active ? e : 0;
    const int ex = (int)(ec % d.nx), ey = (int)((ec / d.nx) % d.ny), ez = (int)(ec / ((int64_t)d.nx * d.ny));
    const T m0 = active ? mu[3 * ec] : T(0), m1 = active ? mu[3 * ec + 1] : T(0), m2 = active ? mu[3 * ec + 2] : T(0);
    const int j = lt / N1, i = lt % N1;
    const int sb = active ? sub : 0;
    const T *A1 = AB1d, *B1 = AB1d + N2;
    T Ai[N1], Bi[N1], Aj[N1], Bj[N1], acc[N1];
#pragma unroll
    for (int t = 0; t < N1; ++t) {
        Ai[t] = A1[i * N1 + t];
        Bi[t] = B1[i * N1 + t];
        Aj[t] = A1[j * N1 + t];
        Bj[t] = B1[j * N1 + t];
        acc[t] = T(0);
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int k0 = c * KC, kn = min(KC, N1 - k0);
        if (c > 0) __syncthreads();
        if (active) {
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const int K = P * ez + k0 + kk, J = P * ey + j, I = P * ex + i;
                if (kk < kn) xs[sb][kk * N2 + lt] = is_free(d, K, J, I) ? x[free_index(d, K, J, I)] : T(0);
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll 1
            for (int kk = 0; kk < kn; ++kk) {
                T a = 0, b = 0;
#pragma unroll
                for (int ii = 0; ii < N1; ++ii) {
                    const T v = xs[sb][kk * N2 + j * N1 + ii];
                    a += Ai[ii] * v;
                    b += Bi[ii] * v;
                }
                as[sb][kk * N2 + lt] = a;
                bs[sb][kk * N2 + lt] = b;
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll 1
            for (int kk = 0; kk < kn; ++kk) {
                T c1 = 0, c2 = 0, c3 = 0;
#pragma unroll
                for (int jj = 0; jj < N1; ++jj) {
                    const T va = as[sb][kk * N2 + jj * N1 + i], vb = bs[sb][kk * N2 + jj * N1 + i];
                    c1 += Bj[jj] * va;
                    c2 += Aj[jj] * vb;
                    c3 += Bj[jj] * vb;
                }
                const T w = m0 * c1 + m1 * c2, sv = m2 * c3;
#pragma unroll
                for (int k = 0; k < N1; ++k) acc[k] += B1[k * N1 + k0 + kk] * w + A1[k * N1 + k0 + kk] * sv;
            }
        }
    }
    if constexpr (EPI == EPI_NONE) {
        if (!active) return;
#pragma unroll
        for (int k = 0; k < N1; ++k) E[elem_index<N1>(d, ex, ey, ez, k, j, i)] = acc[k];
    } else {
        // drop the entries at Dirichlet nodes (the assembled vector has none there)
#pragma unroll
        for (int k = 0; k < N1; ++k)
            if (!active || !is_free(d, P * ez + k, P * ey + j, P * ex + i)) acc[k] = T(0);
        if constexpr (EPI == EPI_FDM) {
            // out(c, b, a) = sum That[k][c] That[j][b] That[i][a] y(k, j, i): z in registers, x
            // and y through LDS, KC slabs at a time; That = AB1d[2 N2 ..] (node x function)
            const T *Th = AB1d + 2 * N2;
            T az[N1];
#pragma unroll
            for (int c = 0; c < N1; ++c) {
                T sacc = 0;
#pragma unroll
                for (int k = 0; k < N1; ++k) sacc += Th[k * N1 + c] * acc[k];
                az[c] = sacc;
            }
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int c0 = ch * KC, cn = min(KC, N1 - c0);
                __syncthreads();
                if (active) {
#pragma unroll
                    for (int cc = 0; cc < KC; ++cc)
                        if (cc < cn) xs[sb][cc * N2 + lt] = az[c0 + cc];
                }
                __syncthreads();
                if (active) {
#pragma unroll 1
                    for (int cc = 0; cc < cn; ++cc) {
                        T sacc = 0;
#pragma unroll
                        for (int ii = 0; ii < N1; ++ii) sacc += Th[ii * N1 + i] * xs[sb][cc * N2 + j * N1 + ii];
                        as[sb][cc * N2 + lt] = sacc;
                    }
                }
                __syncthreads();
                if (active) {
#pragma unroll 1
                    for (int cc = 0; cc < cn; ++cc) {
                        T sacc = 0;
#pragma unroll
                        for (int jj = 0; jj < N1; ++jj) sacc += Th[jj * N1 + j] * as[sb][cc * N2 + jj * N1 + i];
                        E[elem_index<N1>(d, ex, ey, ez, c0 + cc, j, i)] = sacc;
                    }
                }
            }
        } else {
            // 8 corner values (c, b, a) in {0,1}^3: sum N_c(k) N_b(j) N_a(i) y(k, j, i) with the
            // linear hats at the GLL nodes, Nh = AB1d[3 N2 ..] ([corner side][node])
            const T *Nh = AB1d + 3 * N2;
            T m0 = 0, m1 = 0;
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                m0 += Nh[k] * acc[k];
                m1 += Nh[N1 + k] * acc[k];
            }
            const T wa[2] = {Nh[i], Nh[N1 + i]}, wb[2] = {Nh[j], Nh[N1 + j]};
            // reduce over the cell's N2 threads through LDS, KC corners at a time
#pragma unroll
            for (int q0 = 0; q0 < 8; q0 += KC) {
                __syncthreads();
                if (active) {
#pragma unroll
                    for (int qq = 0; qq < KC; ++qq) {
                        const int q = q0 + qq;
                        if (q < 8) xs[sb][qq * N2 + lt] = ((q >> 2) ? m1 : m0) * wb[(q >> 1) & 1] * wa[q & 1];
                    }
                }
                __syncthreads();
                if (active && lt < KC && q0 + lt < 8) {
                    T sacc = 0;
                    for (int t = 0; t < N2; ++t) sacc += xs[sb][lt * N2 + t];
                    E[ec * 8 + q0 + lt] = sacc;
                }
            }
        }
    }
}

// c3[v] = c0[v] - sum over the 8 cells around interior vertex v of their corner value at v
// (the Q1 restriction of an element vector summed per coarse vertex, fixed order).
template <typename T>
__global__ void __launch_bounds__(256) k_coarse_gather(const double *__restrict__ gate, Dims d, const T *__restrict__ c0,
                                                       const T *__restrict__ e8, T *__restrict__ c3) {
    if (gated(gate)) return;
    const int ux = d.nx - 1, uy = d.ny - 1, uz = d.nz - 1;
    const int64_t nv = (int64_t)ux * uy * uz;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int vx = (int)(v % ux) + 1, vy = (int)((v / ux) % uy) + 1, vz = (int)(v / ((int64_t)ux * uy)) + 1;
    T vals[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        // cell (vx - 1 + ax, ...) sees vertex v as its corner (1 - ax, 1 - ay, 1 - az)
        const int ax = q & 1, ay = (q >> 1) & 1, az = q >> 2;
        const int64_t cell = ((int64_t)(vz - 1 + az) * d.ny + (vy - 1 + ay)) * d.nx + (vx - 1 + ax);
        vals[q] = e8[cell * 8 + ((1 - az) * 2 + (1 - ay)) * 2 + (1 - ax)];
    }
    T sum = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) sum += vals[q];
    c3[v] = c0[v] - sum;
}

// Launch geometry of the general operator: S workgroups per cell, each with ceil(Q/S)
// b-rows of Q quadrature columns.
constexpr int opg_rows(int P, int S) { return (QOF(P) + S - 1) / S; }
constexpr int opg_threads(int P, int S) { return (opg_rows(P, S) * QOF(P) + 63) / 64 * 64; }
// z-slabs per chunk: as many as fit in about 60 KB of LDS in either chunked phase
constexpr int opg_chunk(int P, int S, int bytes) {
    const int N1 = P + 1, Q = QOF(P), BR = opg_rows(P, S);
    const int fwd = N1 * N1 + 2 * N1 * Q, bwd = 3 * BR * Q + 2 * N1 * Q;
    const int per = (fwd > bwd ? fwd : bwd) * bytes;
    const int kc = (60 * 1024 - (4 * Q * N1 + 19 * Q) * bytes) / per;
    return kc < 1 ? 1 : (kc > N1 ? N1 : kc);
}

// General trilinear cell: y_K = (grad phi)^T G w (grad phi) x_K with the q^3 GLL rule
// (Sec. 2.1, 2.7).  Thread (b, a) owns one z-column of quadrature points.  The x and y
// contractions run through LDS for a chunk of KC z-slabs at a time (three barriers per chunk
// and direction); the z contraction, the metric and the z back-contraction stay in the
// column's registers.  S workgroups share a cell, each owning a band of ceil(Q/S) b-rows of
// columns (with S = 2 the FP64 column state of p = 14, 15 fits in registers); each writes
// its partial (p+1)^3 block to its own slot of the element vector E, and k_gather sums the
// slots and the cells that share a node.
template <typename T, int P, int S>
__global__ void __launch_bounds__(opg_threads(P, S)) k_op_general(const double *__restrict__ gate, Dims d,
                                                                   const T *__restrict__ IDq, const T *__restrict__ geo,
                                                                   const T *__restrict__ x, T *__restrict__ E) {
    if (gated(gate)) return;
    constexpr int N1 = P + 1, Q = QOF(P), Q2 = Q * Q, Q3 = Q2 * Q, BR = opg_rows(P, S);
    constexpr int KC = opg_chunk(P, S, (int)sizeof(T)), NCH = (N1 + KC - 1) / KC;
    constexpr int FWD = N1 * N1 + 2 * N1 * Q, BWD = 3 * BR * Q + 2 * N1 * Q;
    constexpr int NTH = opg_threads(P, S), NX = KC * N1 * N1, NLX = (NX + NTH - 1) / NTH;
    // the 1D matrices row-major ([a][i]: read with i varying across lanes) and transposed
    // ([i][a]: read with a varying across lanes), so that no phase strides lanes by a row
    __shared__ T sI[Q * N1], sD[Q * N1], sIt[N1 * Q], sDt[N1 * Q];
    // Metric tables of the trilinear map (Sec. 2.7): the Jacobian columns along a quadrature
    // column (a, b) are dx/dxi = n0(zeta) E1[0][b] + n1(zeta) E1[1][b], dx/deta = n0(zeta)
    // E2[0][a] + n1(zeta) E2[1][a], and dx/dzeta = n0(eta) A3[0][a] + n1(eta) A3[1][a] (fixed):
    // the halved corner edge differences interpolated along the other reference axes.
    __shared__ T sE1[6 * Q], sE2[6 * Q], sA3[6 * Q], sW[Q];
    __shared__ T buf[KC * (FWD > BWD ? FWD : BWD)];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t e = blockIdx.x / S;
    for (int t = tid; t < Q * N1; t += nt) {
        const T vi = IDq[t], vd = IDq[Q * N1 + t];
        sI[t] = vi;
        sD[t] = vd;
        sIt[(t % N1) * Q + t / N1] = vi;
        sDt[(t % N1) * Q + t / N1] = vd;
    }
    {
        const T *cg = geo + e * kGeoStride, *xq = IDq + 2 * Q * N1;
        for (int t = tid; t < 6 * Q; t += nt) {
            const int r = t / Q, qq = t % Q, cc = r / 3, dd = r % 3;
            const T n0 = T(0.5) * (T(1) - xq[qq]), n1 = T(0.5) * (T(1) + xq[qq]);
            sE1[t] = n0 * cg[(cc * 2 + 0) * 3 + dd] + n1 * cg[(cc * 2 + 1) * 3 + dd];
            sE2[t] = n0 * cg[12 + (cc * 2 + 0) * 3 + dd] + n1 * cg[12 + (cc * 2 + 1) * 3 + dd];
            sA3[t] = n0 * cg[24 + (cc * 2 + 0) * 3 + dd] + n1 * cg[24 + (cc * 2 + 1) * 3 + dd];
        }
        for (int t = tid; t < Q; t += nt) sW[t] = IDq[2 * Q * N1 + Q + t];
    }
    const int b0 = (int)(blockIdx.x % S) * BR, nb = min(BR, Q - b0);
    const int ex = (int)(e % d.nx), ey = (int)((e / d.nx) % d.ny), ez = (int)(e / ((int64_t)d.nx * d.ny));
    const bool col = tid < nb * Q;
    const int b = b0 + tid / Q, a = tid % Q;
    T AA[N1], AB[N1], BA[N1];
    // ---- forward: x and y contractions, KC slabs at a time
    T *xs = buf, *X1 = buf + KC * N1 * N1, *DX1 = X1 + KC * N1 * Q;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int k0 = c * KC, kn = min(KC, N1 - k0);
        // the chunk's loads all in flight before the first LDS store
        T xv[NLX];
#pragma unroll
        for (int l = 0; l < NLX; ++l) {
            const int t = tid + l * NTH;
            const int kk = t / (N1 * N1), jj = (t / N1) % N1, ii = t % N1;
            const int K = P * ez + k0 + kk, J = P * ey + jj, I = P * ex + ii;
            xv[l] = (t < kn * N1 * N1 && is_free(d, K, J, I)) ? x[free_index(d, K, J, I)] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < NLX; ++l) {
            const int t = tid + l * NTH;
            if (t < kn * N1 * N1) xs[t] = xv[l];
        }
        __syncthreads();
        for (int t = tid; t < kn * N1 * Q; t += nt) {
            const int kj = t / Q, aa = t % Q;   // kj = kk N1 + jj
            T s0 = 0, s1 = 0;
#pragma unroll
            for (int ii = 0; ii < N1; ++ii) {
                s0 += sIt[ii * Q + aa] * xs[kj * N1 + ii];
                s1 += sDt[ii * Q + aa] * xs[kj * N1 + ii];
            }
            X1[t] = s0;
            DX1[t] = s1;
        }
        __syncthreads();
        if (col) {
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const int k = k0 + kk;
                if (k < N1) {
                    T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
                    for (int jj = 0; jj < N1; ++jj) {
                        const T xv = X1[(kk * N1 + jj) * Q + a], dv = DX1[(kk * N1 + jj) * Q + a];
                        s0 += sIt[jj * Q + b] * xv;
                        s1 += sDt[jj * Q + b] * xv;
                        s2 += sIt[jj * Q + b] * dv;
                    }
                    AA[k] = s0;
                    AB[k] = s1;
                    BA[k] = s2;
                }
            }
        }
    }
    // ---- quadrature columns: z contraction, metric, z back-contraction
    T AAo[N1], ABo[N1], BAo[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) AAo[k] = ABo[k] = BAo[k] = 0;
    if (col) {
        // The weighted metric w kappa |det J| J^{-1} J^{-T} (Sec. 2.7) at point (a, b, c) from
        // the tables above instead of a stream from memory.  Rows of J^{-1} are cross products
        // of J's columns over det J, so G_mn = w kappa (c_m . c_n) / det J (det J > 0 is checked
        // at setup).  The table reads in the loop are kept there (not held in registers).
        const T *xq = IDq + 2 * Q * N1;
        const T eta = xq[b], nb0 = T(0.5) * (T(1) - eta), nb1 = T(0.5) * (T(1) + eta);
        T J3[3];
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) J3[dd] = nb0 * sA3[dd * Q + a] + nb1 * sA3[(3 + dd) * Q + a];
        const T wab = sW[a] * sW[b] * geo[e * kGeoStride + 36];
        for (int c = 0; c < Q; ++c) {
            int ia = a, ib = b;
            asm volatile("" : "+v"(ia), "+v"(ib));
            const T zeta = xq[c], nc0 = T(0.5) * (T(1) - zeta), nc1 = T(0.5) * (T(1) + zeta);
            T J1[3], J2[3];
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) {
                J1[dd] = nc0 * sE1[dd * Q + ib] + nc1 * sE1[(3 + dd) * Q + ib];
                J2[dd] = nc0 * sE2[dd * Q + ia] + nc1 * sE2[(3 + dd) * Q + ia];
            }
            const T c1[3] = {J2[1] * J3[2] - J2[2] * J3[1], J2[2] * J3[0] - J2[0] * J3[2], J2[0] * J3[1] - J2[1] * J3[0]};
            const T c2[3] = {J3[1] * J1[2] - J3[2] * J1[1], J3[2] * J1[0] - J3[0] * J1[2], J3[0] * J1[1] - J3[1] * J1[0]};
            const T c3[3] = {J1[1] * J2[2] - J1[2] * J2[1], J1[2] * J2[0] - J1[0] * J2[2], J1[0] * J2[1] - J1[1] * J2[0]};
            const T det = J1[0] * c1[0] + J1[1] * c1[1] + J1[2] * c1[2];
            const T sc = wab * sW[c] / det;
            const T gxx = sc * (c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2]);
            const T gyy = sc * (c2[0] * c2[0] + c2[1] * c2[1] + c2[2] * c2[2]);
            const T gzz = sc * (c3[0] * c3[0] + c3[1] * c3[1] + c3[2] * c3[2]);
            const T gxy = sc * (c1[0] * c2[0] + c1[1] * c2[1] + c1[2] * c2[2]);
            const T gxz = sc * (c1[0] * c3[0] + c1[1] * c3[1] + c1[2] * c3[2]);
            const T gyz = sc * (c2[0] * c3[0] + c2[1] * c3[1] + c2[2] * c3[2]);
            T ux = 0, uy = 0, uz = 0;
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                ux += sI[c * N1 + k] * BA[k];
                uy += sI[c * N1 + k] * AB[k];
                uz += sD[c * N1 + k] * AA[k];
            }
            T vx = gxx * ux + gxy * uy + gxz * uz;
            T vy = gxy * ux + gyy * uy + gyz * uz;
            T vz = gxz * ux + gyz * uy + gzz * uz;
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                AAo[k] += sD[c * N1 + k] * vz;
                ABo[k] += sI[c * N1 + k] * vy;
                BAo[k] += sI[c * N1 + k] * vx;
            }
        }
    }
    // ---- backward: y and x back-contractions, KC slabs at a time
    T *S0 = buf, *S1 = S0 + KC * BR * Q, *S2 = S1 + KC * BR * Q, *Y1 = S2 + KC * BR * Q, *DY1 = Y1 + KC * N1 * Q;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int k0 = c * KC, kn = min(KC, N1 - k0);
        __syncthreads();
        if (col) {
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const int k = k0 + kk;
                if (k < N1) {
                    S0[kk * BR * Q + tid] = AAo[k];
                    S1[kk * BR * Q + tid] = ABo[k];
                    S2[kk * BR * Q + tid] = BAo[k];
                }
            }
        }
        __syncthreads();
        for (int t = tid; t < kn * N1 * Q; t += nt) {
            const int kk = t / (N1 * Q), jj = (t / Q) % N1, aa = t % Q;
            const T *s0p = S0 + kk * BR * Q, *s1p = S1 + kk * BR * Q, *s2p = S2 + kk * BR * Q;
            T s0 = 0, s1 = 0;
            for (int bb = 0; bb < nb; ++bb) {
                s0 += sIt[jj * Q + b0 + bb] * s0p[bb * Q + aa] + sDt[jj * Q + b0 + bb] * s1p[bb * Q + aa];
                s1 += sIt[jj * Q + b0 + bb] * s2p[bb * Q + aa];
            }
            Y1[t] = s0;
            DY1[t] = s1;
        }
        __syncthreads();
        for (int t = tid; t < kn * N1 * N1; t += nt) {
            const int kk = t / (N1 * N1), jj = (t / N1) % N1, ii = t % N1;
            const T *y1 = Y1 + (kk * N1 + jj) * Q, *dy1 = DY1 + (kk * N1 + jj) * Q;
            T s = 0;
            for (int aa = 0; aa < Q; ++aa) s += sI[aa * N1 + ii] * y1[aa] + sD[aa * N1 + ii] * dy1[aa];
            E[(int64_t)(blockIdx.x % S) * (d.nx * d.ny * d.nz) * (N1 * N1 * N1) +
              elem_index<N1>(d, ex, ey, ez, k0 + kk, jj, ii)] = s;
        }
    }
}

// Assembly of an element vector: every free lattice node sums the blocks of the (up to 8)
// cells that contain it, each with its S slots, in a fixed order.  r == nullptr: out = sum;
// else out = r - sum (the residual of the cycle, in T).  A workgroup covers XB consecutive
// free nodes in lattice order.
constexpr int XB = 128;

template <int P>
__device__ __forceinline__ int axis_cells(int g, int c[2], int l[2]) {
    const int q = g / P, rem = g - q * P;
    if (rem == 0) {   // on a cell face: the cell below (local P) and the one above (local 0)
        c[0] = q - 1; l[0] = P; c[1] = q; l[1] = 0;
        return 2;
    }
    c[0] = q; l[0] = rem; c[1] = q; l[1] = rem;
    return 1;
}

template <typename T, int P>
__global__ void __launch_bounds__(XB) k_gather(const double *__restrict__ gate, Dims d, int slots, const T *__restrict__ E,
                                                const double *__restrict__ r, T *__restrict__ out,
                                                const double *__restrict__ dotv, double *__restrict__ partials,
                                                const T *__restrict__ rT) {
    if (gated(gate)) return;
    constexpr int N1 = P + 1, N3 = N1 * N1 * N1;
    if (gridDim.y > 1) {   // independent components (rT, dotv unused): E, r and out per blockIdx.y
        const int64_t nf = (int64_t)d.Lx * d.Ly * d.Lz;
        E += (int64_t)blockIdx.y * slots * d.nx * d.ny * d.nz * N3;
        out += blockIdx.y * nf;
        if (r != nullptr) r += blockIdx.y * nf;
    }
    // the free nodes in lattice order, XB consecutive ones per workgroup (whole lines and
    // line ends together, so that short lines leave no thread idle)
    const int64_t nfree = (int64_t)d.Lx * d.Ly * d.Lz, g0 = (int64_t)blockIdx.x * XB + threadIdx.x;
    const bool live = g0 < nfree;
    const int64_t g = live ? g0 : nfree - 1, line = g / d.Lx;
    const int I = (int)(g - line * d.Lx) + 1, J = (int)(line % d.Ly) + 1, K = (int)(line / d.Ly) + 1;
    int cx[2], lx[2], cy[2], ly[2], cz[2], lz[2];
    const int mx = axis_cells<P>(I, cx, lx), my = axis_cells<P>(J, cy, ly), mz = axis_cells<P>(K, cz, lz);
    const int64_t slot = (int64_t)d.nx * d.ny * d.nz * N3, rowlen = (int64_t)d.nx * N1;
    const int x0 = cx[0] * N1 + lx[0];   // with two cells along x their entries are adjacent (x0, x0 + 1)
    // all candidate loads issued together (predicated), then summed in a fixed order
    T v[2][4][2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int zc = t >> 1, yc = t & 1;
            const bool ok = s < slots && zc < mz && yc < my;
            const T *row = E + (ok ? s * slot + ((((int64_t)cz[zc] * d.ny + cy[yc]) * N1 + lz[zc]) * N1 + ly[yc]) * rowlen + x0 : 0);
            v[s][t][0] = ok ? row[0] : T(0);
            v[s][t][1] = ok && mx == 2 ? row[1] : T(0);
        }
    T sum = T(0);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t) sum += v[s][t][0] + v[s][t][1];
    const int64_t idx = g;
    const T o = rT != nullptr ? rT[idx] - sum : (r == nullptr ? sum : (T)r[idx] - sum);
    if (live) out[idx] = o;
    if (dotv != nullptr) {   // partial sum of dotv . out for this workgroup
        const double prod = block_sum(live ? dotv[idx] * (double)o : 0.0);
        if (threadIdx.x == 0) partials[blockIdx.x] = prod;
    }
}

// Load vector (Sec. 2.1), cell part: E_K = (I x I x I)^T (w |det DF| f) into the cell's block
// of the element vector; k_gather sums the blocks that share a node in a fixed order.
template <int P>
__global__ void __launch_bounds__(1024) k_load_vector(const double *__restrict__ gate, Dims d, const double *__restrict__ IDq, const double *__restrict__ wdet,
                                                      const double *__restrict__ f, double *__restrict__ E) {
    if (gated(gate)) return;
    constexpr int N1 = P + 1, Q = QOF(P), Q2 = Q * Q, Q3 = Q2 * Q;
    __shared__ double sI[Q * N1], X1[N1 * Q], S0[Q2];
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int t = tid; t < Q * N1; t += nt) sI[t] = IDq[t];
    const int64_t e = blockIdx.x;
    const int ex = (int)(e % d.nx), ey = (int)((e / d.nx) % d.ny), ez = (int)(e / ((int64_t)d.nx * d.ny));
    const bool col = tid < Q2;
    double acc[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) acc[k] = 0;
    __syncthreads();
    if (col) {
        for (int c = 0; c < Q; ++c) {
            int64_t pt = e * Q3 + c * Q2 + tid;
            double g = f[pt] * wdet[pt];
#pragma unroll
            for (int k = 0; k < N1; ++k) acc[k] += sI[c * N1 + k] * g;
        }
    }
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        __syncthreads();
        if (col) S0[tid] = acc[k];
        __syncthreads();
        for (int t = tid; t < N1 * Q; t += nt) {
            int jj = t / Q, aa = t % Q;
            double s = 0;
            for (int bb = 0; bb < Q; ++bb) s += sI[bb * N1 + jj] * S0[bb * Q + aa];
            X1[t] = s;
        }
        __syncthreads();
        for (int t = tid; t < N1 * N1; t += nt) {
            int jj = t / N1, ii = t % N1;
            double s = 0;
            for (int aa = 0; aa < Q; ++aa) s += sI[aa * N1 + ii] * X1[jj * Q + aa];
            E[elem_index<N1>(d, ex, ey, ez, k, jj, ii)] = s;
        }
    }
}

// ====================================================================== patch assembly
// Additive Schwarz sum z_F = sum_j Rbar_j^T u_j (Sec. 2.5): each free lattice node sums the
// 8 vertex-parity vectors of the star boxes (star_box_sum).
template <typename T>
__global__ void __launch_bounds__(XB) k_patch_assemble(const double *__restrict__ gate, Dims d, const T *__restrict__ U,
                                                        T *__restrict__ zF) {
    if (gated(gate)) return;
    const int64_t n = (int64_t)d.Lx * d.Ly * d.Lz, i = (int64_t)blockIdx.x * XB + threadIdx.x;
    if (i >= n) return;
    if (gridDim.y > 1) {   // independent (U, zF) pairs: U holds 8 n values per pair
        U += blockIdx.y * 8 * n;
        zF += blockIdx.y * n;
    }
    zF[i] = star_box_sum<T>(U, n, i);
}

// ====================================================================== dense / vector
template <typename T>
__global__ void k_dense_gemv(const double *__restrict__ gate, int n, const T *__restrict__ A, const T *__restrict__ x, T *__restrict__ y, T alpha, T beta) {
    if (gated(gate)) return;
    const int lane = threadIdx.x & 63;
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (row >= n) return;
    const T *a = A + (int64_t)row * n;
    // four independent partial sums per lane: four row loads in flight per step
    T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int c = lane;
    for (; c + 192 < n; c += 256) {
        s0 += a[c] * x[c];
        s1 += a[c + 64] * x[c + 64];
        s2 += a[c + 128] * x[c + 128];
        s3 += a[c + 192] * x[c + 192];
    }
    for (; c < n; c += 64) s0 += a[c] * x[c];
    T s = wave_sum((s0 + s1) + (s2 + s3));
    if (lane == 0) y[row] = beta == T(0) ? alpha * s : alpha * s + beta * y[row];
}

template <typename Tin, typename Tout>
__global__ void k_cast(const double *__restrict__ gate, int64_t n, const Tin *__restrict__ x, Tout *__restrict__ y) {
    if (gated(gate)) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (Tout)x[i];
}

template <typename T>
__global__ void k_fill(const double *__restrict__ gate, int64_t n, T *__restrict__ x, T v) {
    if (gated(gate)) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}

constexpr int RED_BLOCKS = 1024;


// Scalar update of a PCG reduction s into scal (thread 0 of one workgroup).  mode: 0 plain,
// 1 p.q -> alpha (recorded), 2 r.z -> beta (recorded, and the shift), 3 initial r.z (empties the
// record of alphas and betas), 4 r.r, 5 r.r after an x update
// with the device stopping test (iteration count, DONE and STATUS); `mirror` (may be NULL)
// receives DONE for a host that polls it.
__device__ __forceinline__ void apply_mode(double *scal, double s, int mode, double *mirror) {
    if (mode == 0) {
        scal[SC_TMP] = s;
    } else if (mode == 1) {
        scal[SC_PQ] = s;
        const double alpha = scal[SC_RZ] / s;
        scal[SC_ALPHA] = alpha;
        const int k = (int)scal[SC_NA];
        if (k < (int)scal[SC_HCAP]) {
            scal[SC_N + 2 * k] = alpha;
            scal[SC_NA] = (double)(k + 1);
        }
    } else if (mode == 2) {
        scal[SC_RZNEW] = s;
        const double beta = s / scal[SC_RZ];
        scal[SC_BETA] = beta;
        scal[SC_RZ] = s;
        const int k = (int)scal[SC_NA];
        if (k >= 1) scal[SC_N + 2 * (k - 1) + 1] = beta;
    } else if (mode == 3) {
        scal[SC_RZ] = s;
        scal[SC_NA] = 0.0;
    } else if (mode == 4) {
        scal[SC_RR] = s;
    } else if (mode == 5) {
        scal[SC_RR] = s;
        const double it = scal[SC_IT] + 1.0;
        scal[SC_IT] = it;
        double since = 0.0;
        if (s < scal[SC_SFAC2] * scal[SC_REF]) scal[SC_REF] = s;
        else since = scal[SC_SINCE] + 1.0;
        scal[SC_SINCE] = since;
        if (!(s - s == 0.0)) {  // NaN or infinite
            scal[SC_STATUS] = 2.0;
            scal[SC_DONE] = 1.0;
        } else if (s <= scal[SC_RTOL2] * scal[SC_BB]) {
            scal[SC_STATUS] = 1.0;
            scal[SC_DONE] = 1.0;
        } else if (it >= scal[SC_MAXIT]) {
            scal[SC_STATUS] = 3.0;
            scal[SC_DONE] = 1.0;
        } else if (scal[SC_WIN] > 0.0 && since >= scal[SC_WIN]) {
            scal[SC_STATUS] = 4.0;
            scal[SC_DONE] = 1.0;
        }
        if (mirror) *mirror = scal[SC_DONE];
    }
}

// Partial sums of x.y, one per workgroup.
__global__ void k_dot_partial(const double *__restrict__ gate, int64_t n, const double *__restrict__ x,
                              const double *__restrict__ y, double *partials) {
    if (gated(gate)) return;
    double s = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) s += x[i] * y[i];
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// The partials added in index order (the same order on every run) and applied by `mode`.
// A separate launch: a last-workgroup reduction inside the producing kernel needs a device-
// scope release per workgroup, which writes back the L2 of its XCD each time.
// One workgroup of FIN_THREADS adds the nb partials: four independent loads in flight per
// thread, a fixed order throughout.
constexpr int FIN_THREADS = 1024;
__global__ void __launch_bounds__(FIN_THREADS) k_finalize(const double *__restrict__ gate, int nb,
                                                          const double *__restrict__ partials, double *scal, int mode,
                                                          double *mirror) {
    if (gated(gate)) return;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int i = threadIdx.x;
    for (; i + 3 * FIN_THREADS < nb; i += 4 * FIN_THREADS) {
        s0 += partials[i];
        s1 += partials[i + FIN_THREADS];
        s2 += partials[i + 2 * FIN_THREADS];
        s3 += partials[i + 3 * FIN_THREADS];
    }
    for (; i < nb; i += FIN_THREADS) s0 += partials[i];
    const double s = block_sum((s0 + s1) + (s2 + s3));
    if (threadIdx.x == 0) apply_mode(scal, s, mode, mirror);
}

// x += alpha p, r -= alpha q, partial sums of r.r.
__global__ void k_pcg_xr(const double *__restrict__ gate, int64_t n, double *__restrict__ x, double *__restrict__ r,
                         const double *__restrict__ p, const double *__restrict__ q, const double *__restrict__ scal,
                         double *partials) {
    if (gated(gate)) return;
    const double alpha = scal[SC_ALPHA];
    double s = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        double ri = r[i] - alpha * q[i];
        r[i] = ri;
        s += ri * ri;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_pcg_p(const double *__restrict__ gate, int64_t n, double *__restrict__ p, const double *__restrict__ z, const double *__restrict__ scal) {
    if (gated(gate)) return;
    const double beta = scal[SC_BETA];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + beta * p[i];
}

// out = r - Az, then Az = 0 (ready for the next operator apply); out must not alias Az.
// y = a x + b y in FP64; with dotv, the workgroup's partial sum of dotv . y into partials
template <typename T>
__global__ void k_axpby_to_double(const double *__restrict__ gate, int64_t n, double a, const T *__restrict__ x, double b,
                                  double *__restrict__ y, const double *__restrict__ dotv, double *__restrict__ partials) {
    if (gated(gate)) return;
    double s = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double yi = b == 0.0 ? a * (double)x[i] : a * (double)x[i] + b * y[i];
        y[i] = yi;
        if (dotv != nullptr) s += dotv[i] * yi;
    }
    if (dotv != nullptr) {
        s = block_sum(s);
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
}

__global__ void k_pcg_start(double *scal, double rtol, int max_iterations, int window, double factor, double *mirror) {
    if (threadIdx.x == 0) {
        const double bb = scal[SC_RR];
        scal[SC_BB] = bb;
        scal[SC_RTOL2] = rtol * rtol;
        scal[SC_IT] = 0.0;
        scal[SC_MAXIT] = (double)max_iterations;
        scal[SC_REF] = bb;
        scal[SC_SINCE] = 0.0;
        scal[SC_WIN] = (double)window;
        scal[SC_SFAC2] = factor * factor;
        const bool finite = bb - bb == 0.0;
        scal[SC_STATUS] = !finite ? 2.0 : (bb == 0.0 ? 1.0 : 0.0);
        scal[SC_DONE] = (!finite || bb == 0.0) ? 1.0 : 0.0;
        if (mirror) *mirror = scal[SC_DONE];
    }
}



}  // namespace

// ====================================================================== launchers
template <typename T>
void launch_op_kron(const Dims &d, const T *AB1d, const T *mu, const T *x, T *E, const Exec &e) {
    const int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
    int cpw = std::is_same<T, double>::value ? e.t.op_cpw64 : e.t.op_cpw32;
    if (cpw != 1 && cpw != 2 && cpw != 4) throw Error(VSR_EINVAL, "op cells per workgroup must be 1, 2 or 4");
    if ((d.p + 1) * (d.p + 1) > 64) cpw = 1;
#define CALLC(P, C)                                                                                                 \
    hipLaunchKernelGGL((k_op_kron<T, P, C>), dim3((unsigned)((ncell + C - 1) / C)), dim3(round64(C * (P + 1) * (P + 1))), \
                       0, e.s, e.gate, d, AB1d, mu, x, E)
#define CALL(P)                                                  \
    if constexpr ((P + 1) * (P + 1) <= 64) {                     \
        if (cpw == 4) CALLC(P, 4);                               \
        else if (cpw == 2) CALLC(P, 2);                          \
        else CALLC(P, 1);                                        \
    } else {                                                     \
        CALLC(P, 1);                                             \
    }
    VSR_P_SWITCH(d.p, CALL)
#undef CALL
#undef CALLC
}

template <typename T>
int launch_op_general(const Dims &d, const T *IDq, const T *geo, const T *x, T *E, const Exec &e) {
    int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
    const int split = std::is_same<T, double>::value ? e.t.opg_split64 : e.t.opg_split32;
    if (split != 0 && split != 1 && split != 2) throw Error(VSR_EINVAL, "operator split must be 0 (default), 1 or 2");
    if (std::is_same<T, double>::value && d.p >= kOpgMfmaMinP)
        return launch_op_general_mfma<T>(d, split ? split : 1, IDq, geo, x, E, e);
    int slots = 1;
#define CALLS(P, S) \
    hipLaunchKernelGGL((k_op_general<T, P, S>), dim3((unsigned)(ncell * S)), dim3(opg_threads(P, S)), 0, e.s, e.gate, d, IDq, geo, x, E)
#define CALL(P)                                                                                  \
    {                                                                                            \
        const int sp = split ? split : (sizeof(T) == 8 && opg_threads(P, 1) > 512 ? 2 : 1);     \
        slots = sp;                                                                              \
        if (sp == 2) CALLS(P, 2);                                                                \
        else CALLS(P, 1);                                                                        \
    }
    VSR_P_SWITCH(d.p, CALL)
#undef CALL
#undef CALLS
    return slots;
}



void launch_load_vector(const Dims &d, const double *IDq, const double *wdet, const double *f, double *E, const Exec &e) {
    int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
#define CALL(P) \
    hipLaunchKernelGGL((k_load_vector<P>), dim3((unsigned)ncell), dim3(round64(QOF(P) * QOF(P))), 0, e.s, e.gate, d, IDq, wdet, f, E)
    VSR_P_SWITCH(d.p, CALL)
#undef CALL
}


// one workgroup per XB nodes of an x-line
inline unsigned line_blocks(const Dims &d) { return (unsigned)(((int64_t)d.Lx * d.Ly * d.Lz + XB - 1) / XB); }

template <typename T>
void launch_patch_assemble(const Dims &d, const T *U, T *zF, const Exec &e, int ncomp) {
    const int64_t n = (int64_t)d.Lx * d.Ly * d.Lz;
    hipLaunchKernelGGL((k_patch_assemble<T>), dim3((unsigned)((n + XB - 1) / XB), (unsigned)ncomp), dim3(XB), 0, e.s, e.gate,
                       d, U, zF);
}

template <typename T>
void launch_gather(const Dims &d, int slots, const T *E, const double *r, T *out, const Exec &e, const double *dotv,
                   double *partials) {
#define CALL(P) \
    hipLaunchKernelGGL((k_gather<T, P>), dim3(line_blocks(d)), dim3(XB), 0, e.s, e.gate, d, slots, E, r, out, dotv, partials, \
                       (const T *)nullptr)
    VSR_P_SWITCH(d.p, CALL)
#undef CALL
}

template <typename T>
void launch_gather_components(const Dims &d, int ncomp, const T *E, T *out, const Exec &e, const double *r) {
#define CALL(P)                                                                                                   \
    hipLaunchKernelGGL((k_gather<T, P>), dim3(line_blocks(d), (unsigned)ncomp), dim3(XB), 0, e.s, e.gate, d, 1, E, r, \
                       out, (const double *)nullptr, (double *)nullptr, (const T *)nullptr)
    VSR_P_SWITCH(d.p, CALL)
#undef CALL
}

template <typename T>
void launch_gather_sub(const Dims &d, const T *E, const T *rT, T *out, const Exec &e) {
#define CALL(P)                                                                                                   \
    hipLaunchKernelGGL((k_gather<T, P>), dim3(line_blocks(d)), dim3(XB), 0, e.s, e.gate, d, 1, E, (const double *)nullptr, \
                       out, (const double *)nullptr, (double *)nullptr, rT)
    VSR_P_SWITCH(d.p, CALL)
#undef CALL
}

template <typename T>
void launch_op_kron_restrict(const Dims &d, int kind, const T *AB1d, const T *mu, const T *x, T *E, const Exec &e) {
    const int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
    int cpw = std::is_same<T, double>::value ? e.t.op_cpw64 : e.t.op_cpw32;
    if (cpw != 1 && cpw != 2 && cpw != 4) throw Error(VSR_EINVAL, "op cells per workgroup must be 1, 2 or 4");
    if (kind != EPI_FDM && kind != EPI_Q1) throw Error(VSR_EINVAL, "unknown operator restriction");
    if ((d.p + 1) * (d.p + 1) > 64) cpw = 1;
#define CALLE(P, C, K)                                                                                              \
    hipLaunchKernelGGL((k_op_kron<T, P, C, K>), dim3((unsigned)((ncell + C - 1) / C)), dim3(round64(C * (P + 1) * (P + 1))), \
                       0, e.s, e.gate, d, AB1d, mu, x, E)
#define CALLC(P, C)                        \
    if (kind == EPI_FDM) CALLE(P, C, EPI_FDM); \
    else CALLE(P, C, EPI_Q1)
#define CALL(P)                                                  \
    if constexpr ((P + 1) * (P + 1) <= 64) {                     \
        if (cpw == 4) { CALLC(P, 4); }                           \
        else if (cpw == 2) { CALLC(P, 2); }                      \
        else { CALLC(P, 1); }                                    \
    } else {                                                     \
        CALLC(P, 1);                                             \
    }
    VSR_P_SWITCH(d.p, CALL)
#undef CALL
#undef CALLC
#undef CALLE
}

template <typename T>
void launch_coarse_gather(const Dims &d, const T *c0, const T *e8, T *c3, const Exec &e) {
    const int64_t nv = (int64_t)(d.nx - 1) * (d.ny - 1) * (d.nz - 1);
    if (nv == 0) return;
    hipLaunchKernelGGL((k_coarse_gather<T>), dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, e.s, e.gate, d, c0, e8, c3);
}

int64_t gather_blocks(const Dims &d) { return line_blocks(d); }

void launch_finalize(int nb, const double *partials, double *scal, int mode, double *mirror, const Exec &e) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, e.s, e.gate, nb, partials, scal, mode, mirror);
}

template <typename T>
void launch_dense_gemv(int n, const T *A, const T *x, T *y, T alpha, T beta, const Exec &e) {
    if (n == 0) return;
    unsigned blocks = (unsigned)(((int64_t)n * 64 + 255) / 256);
    hipLaunchKernelGGL((k_dense_gemv<T>), dim3(blocks), dim3(256), 0, e.s, e.gate, n, A, x, y, alpha, beta);
}

template <typename Tin, typename Tout>
void launch_cast(int64_t n, const Tin *x, Tout *y, const Exec &e) {
    hipLaunchKernelGGL((k_cast<Tin, Tout>), dim3(grid_for(n)), dim3(256), 0, e.s, e.gate, n, x, y);
}

template <typename T>
void launch_fill(int64_t n, T *x, T v, const Exec &e) {
    hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n)), dim3(256), 0, e.s, e.gate, n, x, v);
}

void launch_dot(int64_t n, const double *x, const double *y, double *partials, double *scal, int mode, double *mirror,
                const Exec &e) {
    int nb = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(256), 0, e.s, e.gate, n, x, y, partials);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, e.s, e.gate, nb, partials, scal, mode, mirror);
}

void launch_pcg_start(double *scal, double rtol, int max_iterations, int window, double factor, double *mirror,
                      const Exec &e) {
    hipLaunchKernelGGL(k_pcg_start, dim3(1), dim3(64), 0, e.s, scal, rtol, max_iterations, window, factor, mirror);
}

void launch_pcg_xr(int64_t n, double *x, double *r, const double *p, const double *q, double *scal, double *partials, int mode,
                   double *mirror, const Exec &e) {
    int nb = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_pcg_xr, dim3(nb), dim3(256), 0, e.s, e.gate, n, x, r, p, q, scal, partials);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, e.s, e.gate, nb, partials, scal, mode, mirror);
}

void launch_pcg_p(int64_t n, double *p, const double *z, const double *scal, const Exec &e) {
    hipLaunchKernelGGL(k_pcg_p, dim3(grid_for(n)), dim3(256), 0, e.s, e.gate, n, p, z, scal);
}


template <typename T>
int launch_axpby_to_double(int64_t n, double a, const T *x, double b, double *y, const Exec &e, const double *dotv,
                           double *partials) {
    const unsigned nb = grid_for(n);
    hipLaunchKernelGGL((k_axpby_to_double<T>), dim3(nb), dim3(256), 0, e.s, e.gate, n, a, x, b, y, dotv, partials);
    return (int)nb;
}



// explicit instantiations
#define INST(T)                                                                                          \
    template void launch_op_kron<T>(const Dims &, const T *, const T *, const T *, T *, const Exec &);    \
    template int launch_op_general<T>(const Dims &, const T *, const T *, const T *, T *, const Exec &);  \
    template void launch_dense_gemv<T>(int, const T *, const T *, T *, T, T, const Exec &);               \
    template void launch_fill<T>(int64_t, T *, T, const Exec &);                                          \
    template void launch_gather<T>(const Dims &, int, const T *, const double *, T *, const Exec &, const double *, \
                                   double *);                                                                    \
    template void launch_gather_sub<T>(const Dims &, const T *, const T *, T *, const Exec &);                   \
    template void launch_gather_components<T>(const Dims &, int, const T *, T *, const Exec &, const double *);  \
    template void launch_patch_assemble<T>(const Dims &, const T *, T *, const Exec &, int);              \
    template void launch_op_kron_restrict<T>(const Dims &, int, const T *, const T *, const T *, T *, const Exec &); \
    template void launch_coarse_gather<T>(const Dims &, const T *, const T *, T *, const Exec &);              \
    template int launch_axpby_to_double<T>(int64_t, double, const T *, double, double *, const Exec &, const double *, \
                                           double *);
INST(float)
INST(double)
template void launch_cast<double, float>(int64_t, const double *, float *, const Exec &);
template void launch_cast<float, double>(int64_t, const float *, double *, const Exec &);
template void launch_cast<double, double>(int64_t, const double *, double *, const Exec &);

}  // namespace vsr
