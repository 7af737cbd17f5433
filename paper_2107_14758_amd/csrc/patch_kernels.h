// Vertex-star patch solves (Sec. 2.4-2.6) for gfx950: one workgroup per patch.  Included
// by one translation unit per precision.
#pragma once

#include "device_common.h"

namespace vsr {
namespace {
using namespace dev;

// ====================================================================== patches
// Box coordinates of a vertex star run over [0, 2m] per axis; the central plane is at m.
// A box position pos maps to the free lattice index p (v - 1) + pos.

__device__ __forceinline__ int la_(int a, int m) { return a < m ? a : a - 1; }
__device__ __forceinline__ int inv_la_(int c, int m) { return c < m ? c : c + 1; }

// interface index of the interior-class ordering (leaves, level-1 separators, top plane)
__device__ __forceinline__ int iface_interior(int ax, int ay, int az, int m, int w, int nl, int ns) {
    if (az == m) return nl + ns + ay * w + ax;
    if (ax == m) return nl + la_(az, m) * w + ay;
    if (ay == m) return la_(az, m) * 2 * m + la_(ax, m);
    return -1;
}

// Per-patch coefficients staged in LDS: the star's cell scalings mu[cz][cy][cx][3]
// (zero for absent cells), the interior eigenvalues lambda_1..m and the couplings
// A_F[t, vertex] of interior mode t to the vertex on the star's central plane
// (afc[0][.] for the cell below the plane, afc[1][.] above).
template <typename T, int M>
struct PatchCtx {
    Dims d;
    int vx, vy, vz;
    const T *rF;
    const T *mu, *lam, *afc;   // LDS
    __device__ int64_t gidx(int ax, int ay, int az) const {
        return ((int64_t)(P_() * (vz - 1) + az) * d.Ly + (P_() * (vy - 1) + ay)) * d.Lx + (P_() * (vx - 1) + ax);
    }
    __device__ static constexpr int P_() { return M + 1; }
    __device__ const T *cmu(const int c[3]) const { return mu + 3 * ((c[2] * 2 + c[1]) * 2 + c[0]); }
    // r_F at a face DOF minus the condensed interior lines of its two cells along axis dd:
    // g = r_G - A_GI A_II^{-1} r_I (Sec. 2.6), A_II = mu . lambda, A_GI = mu_dd A_F[interior, vertex].
    __device__ T condensed(const int pos[3], int dd) const {
        // both cells' interior lines are loaded before any arithmetic (one round of latency)
        T rv[2 * M + 1];
        load_line(pos, dd, rv);
        return condense_line(pos, dd, rv);
    }
    // the values condensed() reads: r at the face DOF, then the interior line of the cell
    // below it along dd and that of the cell above
    __device__ void load_line(const int pos[3], int dd, T *rv) const {
        rv[0] = rF[gidx(pos[0], pos[1], pos[2])];
#pragma unroll
        for (int cd = 0; cd < 2; ++cd) {
            int q[3] = {pos[0], pos[1], pos[2]};
#pragma unroll
            for (int t = 1; t <= M; ++t) {
                q[dd] = cd == 0 ? t - 1 : M + t;
                rv[1 + cd * M + t - 1] = rF[gidx(q[0], q[1], q[2])];
            }
        }
    }
    __device__ T condense_line(const int pos[3], int dd, const T *rl) const {
        const T g = rl[0];
        const T *rv[2] = {rl + 1, rl + 1 + M};
        int c[3], l[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = pos[a] > M;
            l[a] = c[a] ? pos[a] - M : pos[a] + 1;
        }
        T acc = 0;
#pragma unroll
        for (int cd = 0; cd < 2; ++cd) {
            c[dd] = cd;
            const T *mk = cmu(c);
            T base = 0;
            for (int a = 0; a < 3; ++a)
                if (a != dd) base += mk[a] * lam[l[a] - 1];
            const T mdd = mk[dd];
#pragma unroll
            for (int t = 1; t <= M; ++t) acc += mdd * afc[cd * M + t - 1] * rv[cd][t - 1] / (base + mdd * lam[t - 1]);
        }
        return g - acc;
    }
    // u_I = A_II^{-1}(r_I - A_IG u_G) at an interior DOF; face(a) gives the interface value
    template <typename F>
    __device__ T back_interior(const int pos[3], const bool full[3], F face) const {
        return back_interior_r(pos, full, rF[gidx(pos[0], pos[1], pos[2])], face);
    }
    // the same with r_I already loaded
    template <typename F>
    __device__ T back_interior_r(const int pos[3], const bool full[3], T r, F face) const {
        int c[3], l[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = pos[a] > M;
            l[a] = c[a] ? pos[a] - M : pos[a] + 1;
        }
        const T *mk = cmu(c);
        T D = mk[0] * lam[l[0] - 1] + mk[1] * lam[l[1] - 1] + mk[2] * lam[l[2] - 1];
        T u = r;
        for (int a = 0; a < 3; ++a)
            if (full[a]) u -= mk[a] * afc[c[a] * M + l[a] - 1] * face(a);
        return u / D;
    }
};

template <typename T, int M>
__device__ void stage_coefficients(const Dims &d, int vx, int vy, int vz, const int kind[3], const T *__restrict__ mu,
                                   const T *__restrict__ lam, const T *__restrict__ afc, T *smu, T *slam, T *safc) {
    const int tid = threadIdx.x;
    if (tid < 24) {
        int comp = tid % 3, cell = tid / 3, cx = cell & 1, cy = (cell >> 1) & 1, cz = cell >> 2;
        int cc[3] = {cx, cy, cz};
        bool ok = true;
        for (int a = 0; a < 3; ++a)
            if (kind[a] == AX_LOW ? cc[a] == 0 : (kind[a] == AX_HIGH ? cc[a] == 1 : false)) ok = false;
        int ex = vx - 1 + cx, ey = vy - 1 + cy, ez = vz - 1 + cz;
        smu[tid] = ok ? mu[3 * ((int64_t)ex + d.nx * ((int64_t)ey + d.ny * (int64_t)ez)) + comp] : T(0);
    }
    for (int t = tid; t < M; t += blockDim.x) slam[t] = lam[t];
    for (int t = tid; t < 2 * M; t += blockDim.x) safc[t] = afc[t];
}

// Triangular solves with the packed inverse Li of a lower Cholesky factor (column k holds
// rows k..nstore-1 of L^{-1} from offset k nstore - k (k - 1) / 2): y = L^{-1} b and
// y = L^{-T} b are matrix-vector products whose rows are independent, so a wavefront has
// no elimination chain.  Lane i returns row i (zero for i >= rows); b is in LDS, read as
// broadcasts; four partial sums per lane.  Entries outside the triangle or at or beyond
// `rows` are never loaded.
template <typename T>
__device__ __forceinline__ T tri_inv_mv(const T *__restrict__ Li, int nstore, int k0, int k1, int rows, int lane,
                                        const T *b) {
    T acc[4] = {T(0), T(0), T(0), T(0)};
    int off = k0 * nstore - k0 * (k0 - 1) / 2;   // start of column k0
    const bool live = lane < rows;
#pragma unroll 4
    for (int k = k0; k < k1; ++k) {
        const T v = (live && lane >= k) ? Li[off + lane - k] : T(0);
        acc[k & 3] += v * b[k];
        off += nstore - k;
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

template <typename T>
__device__ __forceinline__ T tri_inv_t_mv(const T *__restrict__ Li, int nstore, int k0, int k1, int rows, int lane,
                                          const T *b) {
    T acc[4] = {T(0), T(0), T(0), T(0)};
    const int base = lane * nstore - lane * (lane - 1) / 2 - lane;   // L^{-1}(k, lane) at base + k
    const bool live = lane < rows;
#pragma unroll 4
    for (int k = k0; k < k1; ++k) {
        const T v = (live && k >= lane) ? Li[base + k] : T(0);
        acc[k & 3] += v * b[k];
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Symmetric S stored as its packed lower triangle (column k holds rows k..nstore-1 from
// offset k nstore - k (k - 1) / 2): lane i returns sum over k in [k0, k1) of S(i, k) b[k]
// (zero for i >= rows), reading S(i, k) from column k below the diagonal and from column i
// above it; b in LDS, read as broadcasts.
template <typename T>
__device__ __forceinline__ T sym_packed_mv(const T *__restrict__ Sp, int nstore, int k0, int k1, int rows, int lane,
                                           const T *b) {
    T acc[4] = {T(0), T(0), T(0), T(0)};
    int off = k0 * nstore - k0 * (k0 - 1) / 2;                          // start of column k0
    const int base = lane * nstore - lane * (lane - 1) / 2 - lane;      // S(k, lane) at base + k, k >= lane
    const bool live = lane < rows;
#pragma unroll 4
    for (int k = k0; k < k1; ++k) {
        const T v = live ? (lane >= k ? Sp[off + lane - k] : Sp[base + k]) : T(0);
        acc[k & 3] += v * b[k];
        off += nstore - k;
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Value of v in lane k (k uniform across the wavefront).
template <typename T>
__device__ __forceinline__ T lane_value(T v, int k);
template <>
__device__ __forceinline__ float lane_value<float>(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
template <>
__device__ __forceinline__ double lane_value<double>(double v, int k) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k), hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

// tri_inv_t_mv over all `rows` columns with b held one entry per lane (lane k holds b[k]):
// the same products summed in the same order, no LDS round trip for b.
template <typename T>
__device__ __forceinline__ T tri_inv_t_mv_lanes(const T *__restrict__ Li, int nstore, int rows, int lane, T b) {
    T acc[4] = {T(0), T(0), T(0), T(0)};
    const int base = lane * nstore - lane * (lane - 1) / 2 - lane;
    const bool live = lane < rows;
#pragma unroll 4
    for (int k = 0; k < rows; ++k) {
        const T bk = lane_value(b, k);
        const T v = (live && k >= lane) ? Li[base + k] : T(0);
        acc[k & 3] += v * bk;
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

template <typename T>
struct Vec4 {
    T v[4];
};
template <typename T>
__device__ __forceinline__ Vec4<T> load4(const T *p);
template <>
__device__ __forceinline__ Vec4<float> load4<float>(const float *p) {
    float4 a = *reinterpret_cast<const float4 *>(p);
    return {{a.x, a.y, a.z, a.w}};
}
template <>
__device__ __forceinline__ Vec4<double> load4<double>(const double *p) {
    double2 a = *reinterpret_cast<const double2 *>(p);
    double2 b = *reinterpret_cast<const double2 *>(p + 2);
    return {{a.x, a.y, b.x, b.y}};
}

// y[r] -= sum_c M[c * ld + r] x[c] for r < nrows (ld multiple of 4, M 16-byte aligned);
// x, y in LDS.  Work split over (row quads) x (column chunks), accumulated with LDS atomics;
// each thread keeps U column loads in flight.  det: one chunk per row quad, so every sum is
// taken by one thread in column order (no atomics; bitwise repeatable, fewer threads busy).
template <typename T, int U, int NTH>
__device__ void panel_fwd(const T *__restrict__ M, int ld, int nrows, int ncols, const T *x, T *y, bool det) {
    const int tid = threadIdx.x;
    constexpr int nt = NTH;
    const int nq = (nrows + 3) / 4;
    if (nq == 0 || ncols == 0) return;
    int nch = det ? 1 : max(1, min((ncols + U - 1) / U, nt / nq));
    int chunk = (ncols + nch - 1) / nch;
    for (int task = tid; task < nq * nch; task += nt) {
        int rq = task % nq, ch = task / nq;
        int c0 = ch * chunk, c1 = min(ncols, c0 + chunk);
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        const T *base = M + 4 * rq;
        for (int c = c0; c < c1; c += U) {
            Vec4<T> v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (c + u < c1) v[u] = load4(base + (int64_t)(c + u) * ld);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (c + u < c1) {
                    T xc = x[c + u];
                    a0 += v[u].v[0] * xc;
                    a1 += v[u].v[1] * xc;
                    a2 += v[u].v[2] * xc;
                    a3 += v[u].v[3] * xc;
                }
            }
        }
        int r = 4 * rq;
        if (nch == 1) {
            if (r < nrows) y[r] -= a0;
            if (r + 1 < nrows) y[r + 1] -= a1;
            if (r + 2 < nrows) y[r + 2] -= a2;
            if (r + 3 < nrows) y[r + 3] -= a3;
        } else {
            if (r < nrows) atomicAdd(&y[r], -a0);
            if (r + 1 < nrows) atomicAdd(&y[r + 1], -a1);
            if (r + 2 < nrows) atomicAdd(&y[r + 2], -a2);
            if (r + 3 < nrows) atomicAdd(&y[r + 3], -a3);
        }
    }
}

// y[c] -= sum_r M[c * ld + r] x[r] for c < ncols.
// Long columns (at least 32 row quads): a wavefront takes G = min(U, 8) columns at a time
// and its lanes split their rows, so every load instruction reads whole cache lines; G
// loads in flight per lane; the G sums are reduced across the wavefront and stored by lane
// 0 (each column has one owner, no atomics).  Short columns: a thread streams one (column, row chunk) with
// U loads in flight; chunks of one column meet in an LDS atomic (det: one chunk per column,
// summed by one thread in row order).
template <typename T, int U, int NTH>
__device__ void panel_bwd(const T *__restrict__ M, int ld, int nrows, int ncols, const T *x, T *y, bool det) {
    const int tid = threadIdx.x;
    constexpr int nt = NTH, NW = NTH / 64;
    const int nq = (nrows + 3) / 4;
    if (nq == 0 || ncols == 0) return;
    if (nq >= 32) {
        constexpr int G = U > 8 ? 8 : U;   // columns per wavefront step
        const int lane = tid & 63, wv = tid >> 6;
        for (int c0 = wv * G; c0 < ncols; c0 += NW * G) {
            T acc[G];
#pragma unroll
            for (int g = 0; g < G; ++g) acc[g] = T(0);
            for (int q = lane; q < nq; q += 64) {
                const int r = 4 * q;
                const T x0 = x[r], x1 = r + 1 < nrows ? x[r + 1] : T(0), x2 = r + 2 < nrows ? x[r + 2] : T(0),
                        x3 = r + 3 < nrows ? x[r + 3] : T(0);
                Vec4<T> v[G];
#pragma unroll
                for (int g = 0; g < G; ++g)
                    if (c0 + g < ncols) v[g] = load4(M + (int64_t)(c0 + g) * ld + r);
#pragma unroll
                for (int g = 0; g < G; ++g)
                    if (c0 + g < ncols) acc[g] += (v[g].v[0] * x0 + v[g].v[1] * x1) + (v[g].v[2] * x2 + v[g].v[3] * x3);
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const T sg = wave_sum(acc[g]);
                if (lane == 0 && c0 + g < ncols) y[c0 + g] -= sg;
            }
        }
        return;
    }
    int nrc = det ? 1 : max(1, min((nq + U - 1) / U, nt / ncols));
    int chunk = (nq + nrc - 1) / nrc;
    for (int task = tid; task < ncols * nrc; task += nt) {
        int c = task % ncols, rc = task / ncols;
        int q0 = rc * chunk, q1 = min(nq, q0 + chunk);
        const T *col = M + (int64_t)c * ld;
        T s = 0;
        for (int q = q0; q < q1; q += U) {
            Vec4<T> v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (q + u < q1) v[u] = load4(col + 4 * (q + u));
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (q + u < q1) {
                    int r = 4 * (q + u);
                    s += v[u].v[0] * x[r];
                    if (r + 1 < nrows) s += v[u].v[1] * x[r + 1];
                    if (r + 2 < nrows) s += v[u].v[2] * x[r + 2];
                    if (r + 3 < nrows) s += v[u].v[3] * x[r + 3];
                }
            }
        }
        if (nrc == 1) y[c] -= s;
        else atomicAdd(&y[c], -s);
    }
}

// Lane move by a DPP control (row_mask and bank_mask select the lanes written; lanes whose
// source lies outside the row read 0).
template <int CTRL, int RM, int BM>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, RM, BM, true));
}
template <int CTRL, int RM, int BM>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, RM, BM, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, RM, BM, true);
    return __hiloint2double(hi, lo);
}

// Sum over the wavefront's 64 lanes, returned in every lane: DPP row shifts sum each 16-lane
// row into its lane 15, row broadcasts carry the row sums into lane 63, and a readlane
// returns it (vector ALU only; no LDS-routed shuffles).
template <typename T>
__device__ __forceinline__ T wave_total(T v) {
    T s = v + dpp_mov<0x111, 0xf, 0xf>(v) + dpp_mov<0x112, 0xf, 0xf>(v) + dpp_mov<0x113, 0xf, 0xf>(v);
    s += dpp_mov<0x114, 0xf, 0xe>(s);   // row_shr:4 into banks 1-3
    s += dpp_mov<0x118, 0xf, 0xc>(s);   // row_shr:8 into banks 2-3: lane 15 of a row holds its sum
    s += dpp_mov<0x142, 0xa, 0xf>(s);   // row_bcast:15 into rows 1 and 3
    s += dpp_mov<0x143, 0xc, 0xf>(s);   // row_bcast:31 into rows 2 and 3: lane 63 holds the total
    return lane_value(s, 63);
}

// One pass over a panel M of a symmetric matrix (column c holds rows r < nrows at
// M[c ld + r], ld a multiple of 4, 16-byte aligned) that applies it both ways:
// yB[r] -= sum_c M(r, c) xJ[c] for every row, and the return value of lane c (c < ncols) is
// this wavefront's share of sum_r M(r, c) xB[r] (the caller adds the wavefronts' shares).
// The NW wavefronts form NWR row groups times NW / NWR column groups; a lane owns up to RQ
// row quads of its group (its rows' sums stay in registers) and each column's sum is
// reduced across the wavefront, so every entry is loaded once.  With one column group every
// sum is taken in a fixed order and yB is written (assign: yB = -sum); with several, the
// groups' row sums meet in LDS atomics (yB must hold its start value).
template <typename T, int NTH, int RQ, int NWR>
__device__ T panel_sym(const T *__restrict__ M, int ld, int nrows, int ncols, const T *xJ, const T *xB, T *yB,
                       bool assign) {
    constexpr int NW = NTH / 64, NWC = NW / NWR, G = 4;   // G columns' loads in flight per step
    static_assert(NW % NWR == 0, "whole column groups");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, rg = wv % NWR, cg = wv / NWR;
    const int nq = (nrows + 3) / 4, per = (nq + NWR - 1) / NWR;
    const int qb = rg * per, qe = min(nq, qb + per);
    const int cper = (ncols + NWC - 1) / NWC, cb = cg * cper, ce = min(ncols, cb + cper);
    T a[RQ][4], xb[RQ][4];
#pragma unroll
    for (int t = 0; t < RQ; ++t) {
        const int q = qb + lane + 64 * t;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[t][u] = T(0);
            xb[t][u] = q < qe && 4 * q + u < nrows ? xB[4 * q + u] : T(0);
        }
    }
    T mine = T(0);
    for (int c0 = cb; c0 < ce; c0 += G) {
        Vec4<T> v[G][RQ];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int t = 0; t < RQ; ++t) {
                const int q = qb + lane + 64 * t;
                if (c0 + g < ce && q < qe) v[g][t] = load4(M + (int64_t)(c0 + g) * ld + 4 * q);
                else v[g][t] = Vec4<T>{{T(0), T(0), T(0), T(0)}};
            }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const T xc = c0 + g < ce ? xJ[c0 + g] : T(0);
            T s = 0;
#pragma unroll
            for (int t = 0; t < RQ; ++t) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[t][u] += v[g][t].v[u] * xc;
                    s += v[g][t].v[u] * xb[t][u];
                }
            }
            s = wave_total(s);
            if (lane == c0 + g) mine = s;
        }
    }
#pragma unroll
    for (int t = 0; t < RQ; ++t) {
        const int q = qb + lane + 64 * t;
        if (q < qe)
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (4 * q + u < nrows) {
                    if constexpr (NWC == 1) yB[4 * q + u] = (assign ? T(0) : yB[4 * q + u]) - a[t][u];
                    else atomicAdd(&yB[4 * q + u], -a[t][u]);
                }
    }
    return mine;
}

// Workgroup barrier that also stops the compiler from moving instructions between the
// phases it separates (interleaving phases raises register pressure and forces spills).
__device__ __forceinline__ void phase_sync() {
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
}

// Sum of the wavefronts' 64-row partials (pairwise for 4 and 8 wavefronts).
template <typename T>
__device__ __forceinline__ T sum_waves(const T *red, int nw, int lane) {
    if (nw == 4) return (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
    if (nw == 8)
        return ((red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane])) +
               ((red[256 + lane] + red[320 + lane]) + (red[384 + lane] + red[448 + lane]));
    T s = 0;
    for (int w = 0; w < nw; ++w) s += red[64 * w + lane];
    return s;
}

// Offset of top-plane tile J inside one interior-patch factor.  Every tile before it holds
// its diagonal block packed in 64 columns, then the panel of rows below it padded to a
// multiple of 4 (only the last tile, which has no panel, is packed in its own width).
__device__ __forceinline__ int64_t tile_offset(int64_t off_Ltop, int NT, int J) {
    int64_t o = off_Ltop;
    for (int j = 0; j < J; ++j) {
        int rows = NT - 64 * j - min(64, NT - 64 * j);
        o += 64 * 65 / 2 + (int64_t)64 * ((rows + 3) / 4 * 4);
    }
    return o;
}

// Interior-vertex patch solve, one workgroup per patch (Sec. 2.6): condensation of the
// diagonal interior block, then the nested-dissection Cholesky factor of the interface
// Schur complement (leaves, level-1 separator slices, dense top plane), forward and
// backward, then interior back-substitution.  Output: the patch box of (2m+1)^3 values.
template <typename T, int P, int UNR, int NTH>
__device__ __forceinline__ void patch_interior(const int pid, Dims d, PatchArgs A, const int *__restrict__ verts,
                                               const int *__restrict__ fidx, const T *__restrict__ factor, const T *__restrict__ mu,
                                               const T *__restrict__ lam, const T *__restrict__ afc,
                                               const T *__restrict__ rF, T *__restrict__ U) {
    constexpr int M = P - 1, W = 2 * M + 1, NL = 4 * M * M, NS = 2 * M * W, NT = W * W, NI = NL + NS + NT;
    constexpr int NTILE = (NT + 63) / 64;
    __shared__ T g[NI];
    __shared__ T smu[24], slam[M], safc[2 * M];
    __shared__ T tl[64 * 65 / 2];
    __shared__ T red[NTH];   // one 64-row partial per wavefront
    // level-1 and leaf work vectors of the top x level-1 coupling; while the top plane is
    // applied (neither is live then) the same memory holds -x_T (NS + NL >= NT)
    __shared__ T zw[NS + NL];
    T *const zs = zw, *const wl = zw + NS, *const xt = zw;
    // panel_sym's shape: row groups of at most 64 row quads of the tallest panel (whole
    // wavefronts' worth of lanes), the wavefronts left over split the columns; one row
    // group per wavefront (no atomics) in the deterministic mode
    constexpr int TOP_NQ = NT > 64 ? (NT - 64 + 3) / 4 : 1;
    constexpr int TOP_NWR0 = (TOP_NQ + 63) / 64 < NTH / 64 ? (TOP_NQ + 63) / 64 : NTH / 64;
    constexpr int TOP_NWR = TOP_NWR0 <= 1 ? 1 : (TOP_NWR0 <= 2 ? 2 : (TOP_NWR0 <= 4 ? 4 : NTH / 64));
    constexpr int TOP_RQ = (TOP_NQ + 64 * TOP_NWR - 1) / (64 * TOP_NWR);
    constexpr int TOP_RQD = (TOP_NQ + NTH - 1) / NTH;
    // the 2m slice inverses are applied four times (forward, the coupling, backward twice):
    // staged once in LDS while they fit in 9 KB (FP64 p=7 included: its registers already
    // hold it to 4 workgroups per CU, and the LDS fits 4), and in FP32 from degree 11 on
    // (18-49 KB: meshes at those degrees have few patches per CU, so the LDS costs no
    // residency), else read from the factor each time
    constexpr int LS = W * (W + 1) / 2, NSEP = 2 * M * LS;
    constexpr bool SEP_LDS = NSEP * sizeof(T) <= 9216 || (sizeof(T) == 4 && P >= 11);
    __shared__ T sL[SEP_LDS ? NSEP : 1];
    constexpr int nt = NTH, nw = NTH / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int kfull[3] = {AX_FULL, AX_FULL, AX_FULL};
    const int vx = verts[3 * pid], vy = verts[3 * pid + 1], vz = verts[3 * pid + 2];
    const T *F = factor + (int64_t)fidx[pid] * A.stride;
    if constexpr (SEP_LDS) {   // every load in flight before the first LDS store
        constexpr int RS = (NSEP + NTH - 1) / NTH;
        T sv[RS];
#pragma unroll
        for (int u = 0; u < RS; ++u) sv[u] = tid + nt * u < NSEP ? F[A.off_Lsep + tid + nt * u] : T(0);
#pragma unroll
        for (int u = 0; u < RS; ++u)
            if (tid + nt * u < NSEP) sL[tid + nt * u] = sv[u];
    }
    const T *Lsep = SEP_LDS ? (const T *)sL : F + A.off_Lsep;
    stage_coefficients<T, M>(d, vx, vy, vz, kfull, mu, lam, afc, smu, slam, safc);
    phase_sync();
    PatchCtx<T, M> C{d, vx, vy, vz, rF, smu, slam, safc};
    // the star box: up to degree kFusedScatterMaxP stored as the vertex's own box, above it
    // in the lattice vector of the star's vertex-parity class (boxes of one class do not
    // overlap) at the lattice nodes it covers (see launch_patch_all)
    constexpr bool PARITY = P > kFusedScatterMaxP;
    T *Uc = PARITY ? U + star_class(vx, vy, vz) * ((int64_t)d.Lx * d.Ly * d.Lz)
                   : U + ((int64_t)(vz * (d.ny + 1) + vy) * (d.nx + 1) + vx) * (int64_t)(W * W * W);
    const int X0 = vx * P - M, Y0 = vy * P - M, Z0 = vz * P - M;   // lattice node of box position 0

    // ---- condensation of the interior DOFs into the interface right-hand side
    auto iface_pos = [&](int idx, int pos[3]) {   // position of interface DOF idx; returns its axis
        if (idx < NL) {
            pos[2] = inv_la_(idx / (2 * M), M); pos[0] = inv_la_(idx % (2 * M), M); pos[1] = M;
        } else if (idx < NL + NS) {
            int t = idx - NL;
            pos[2] = inv_la_(t / W, M); pos[1] = t % W; pos[0] = M;
        } else {
            int t = idx - NL - NS;
            pos[1] = t / W; pos[0] = t % W; pos[2] = M;
        }
        return pos[0] == M ? 0 : (pos[1] == M ? 1 : 2);
    };
    // ---- forward: the leaves' diagonal block is applied as their values are condensed
    const T *invd = F + A.off_invd, *B1 = F + A.off_B1, *B2 = F + A.off_B2;
    for (int idx = tid; idx < NI; idx += nt) {
        int pos[3];
        const int dd = iface_pos(idx, pos);
        const int ncen = (pos[0] == M) + (pos[1] == M) + (pos[2] == M);
        const T dl = idx < NL ? invd[idx] : T(1);
        const T gv = ncen == 1 ? C.condensed(pos, dd) : rF[C.gidx(pos[0], pos[1], pos[2])];
        g[idx] = idx < NL ? gv * dl : gv;
    }
    phase_sync();
    // leaf columns update their level-1 slice (their top-plane update, g_T -= L_TL y_L, is
    // folded into the coupling below, which reads L_TL anyway: g_T is not used before it)
    for (int task = tid; task < NS; task += nt) {
        int s = task / W, r = task % W;
        T acc = 0;
#pragma unroll
        for (int c = 0; c < 2 * M; ++c) acc += B1[(int64_t)(s * 2 * M + c) * W + r] * g[s * 2 * M + c];
        g[NL + s * W + r] -= acc;
    }
    phase_sync();
    // level-1 separator slices, one wavefront per slice: the dense lower solve y_S, then at
    // once (from the lanes' registers) z = L_SS^{-T} y_S for the top x level-1 coupling below
    for (int s = wv; s < 2 * M; s += nw) {
        const T x = tri_inv_mv<T>(Lsep + s * LS, W, 0, W, W, lane, g + NL + s * W);
        if (lane < W) g[NL + s * W + lane] = x;
        const T zv = tri_inv_t_mv_lanes<T>(Lsep + s * LS, W, W, lane, x);
        if (lane < W) zs[s * W + lane] = zv;
    }
    // stage the first top-plane diagonal tile while the level-1 solves finish
    T *gt = g + NL + NS;
    // stage a packed diagonal block verbatim (column k holds rows k..ns-1 from offset
    // k ns - k (k - 1) / 2; ns = 64, or the last block's own width NBL); all loads in flight
    // before the first LDS store
    constexpr int NBL = NT - 64 * (NTILE - 1);
    auto tile_ns = [](int J) { return J + 1 < NTILE ? 64 : NBL; };
    auto stage_tile = [&](int J) {
        const T *D = F + tile_offset(A.off_Ltop, NT, J);
        const int ns = tile_ns(J), NP = ns * (ns + 1) / 2;
        constexpr int R = (64 * 65 / 2 + NTH - 1) / NTH;
        T v[R];
#pragma unroll
        for (int u = 0; u < R; ++u) v[u] = tid + nt * u < NP ? D[tid + nt * u] : T(0);
#pragma unroll
        for (int u = 0; u < R; ++u)
            if (tid + nt * u < NP) tl[tid + nt * u] = v[u];
    };
    stage_tile(0);
    phase_sync();
    // the level-1 solution updates the top plane: g_T -= L_TS y_S with L_TS = S''_TS L_SS^{-T}
    // and S''_TS = S_TS - L_TL L_SL^T (S_TS: the raw Schur block, y-diagonal and stored; the
    // leaf blocks and the slice inverses are the ones used above), so the dense panel is
    // never formed
    const T *Sy = F + A.off_Sy;
    for (int i = tid; i < NL; i += nt) {     // w_L = L_SL^T z (leaf (s, c) meets slice s)
        const int sl = i / (2 * M);
        T acc = 0;
#pragma unroll
        for (int r = 0; r < W; ++r) acc += B1[(int64_t)i * W + r] * zs[sl * W + r];
        wl[i] = acc;
    }
    phase_sync();
    for (int i = tid; i < NT; i += nt) {     // g_T -= L_TL y_L + S_TS z - L_TL w_L
        const int ay = i / W, ax = i % W;
        T acc = 0;
#pragma unroll
        for (int s = 0; s < 2 * M; ++s) acc += Sy[(int64_t)s * NT + i] * zs[s * W + ay];
        if (ax != M) {
            const int lx = la_(ax, M);
#pragma unroll
            for (int c = 0; c < 2 * M; ++c) acc += B2[(int64_t)(lx * 2 * M + c) * W + ay] * (g[c * 2 * M + lx] - wl[c * 2 * M + lx]);
        }
        gt[i] -= acc;
    }
    phase_sync();
    // dense top plane: x_T = S_T^{-1} g_T with the stored inverse of the top plane's Schur
    // complement (S_T = L_T L_T^T; one symmetric product instead of the two triangular
    // sweeps), 64-column tiles of its lower triangle, each read once: per tile the diagonal
    // block from LDS (the k-range split over the wavefronts) and the panel below it both ways.
    // xt accumulates -x_T (the first tile's products start it: tile 0's panel covers every
    // row below it).
    static_assert(NS + NL >= NT, "xt fits the coupling's work vectors");
    const bool top_atomic = !A.det && TOP_NWR < nw;   // column groups meet in LDS atomics
    if (top_atomic) {   // they need -x_T to start at zero (zs, wl are no longer read)
        for (int i = tid; i < NT; i += nt) xt[i] = T(0);
        phase_sync();
    }
    for (int J = 0; J < NTILE; ++J) {
        const int c0 = 64 * J, nb = min(64, NT - c0);
        const int kw = 64 / nw;
        T part = sym_packed_mv<T>(tl, tile_ns(J), min(kw * wv, nb), min(kw * wv + kw, nb), nb, lane, gt + c0);
        const T *D = F + tile_offset(A.off_Ltop, NT, J);
        const int rows = NT - c0 - nb;
        if (top_atomic)
            part += panel_sym<T, NTH, TOP_RQ, TOP_NWR>(D + 64 * 65 / 2, (rows + 3) / 4 * 4, rows, nb, gt + c0,
                                                       gt + c0 + nb, xt + c0 + nb, false);
        else
            part += panel_sym<T, NTH, TOP_RQD, NTH / 64>(D + 64 * 65 / 2, (rows + 3) / 4 * 4, rows, nb, gt + c0,
                                                         gt + c0 + nb, xt + c0 + nb, J == 0);
        red[tid] = part;
        phase_sync();
        if (wv == 0 && lane < nb) xt[c0 + lane] = (J == 0 && !top_atomic ? T(0) : xt[c0 + lane]) - sum_waves(red, nw, lane);
        if (J + 1 < NTILE) stage_tile(J + 1);
        phase_sync();
    }
    for (int i = tid; i < NT; i += nt) gt[i] = -xt[i];
    phase_sync();
    // y_S -= L_TS^T x_T = L_SS^{-1} (S_TS^T x_T - L_SL (L_TL^T x_T))
    for (int i = tid; i < NL; i += nt) {     // w_L = L_TL^T x_T (leaf (c, lx) meets top column lx)
        const int c = i / (2 * M), lx = i % (2 * M), ax = inv_la_(lx, M);
        T acc = 0;
#pragma unroll
        for (int ay = 0; ay < W; ++ay) acc += B2[(int64_t)(lx * 2 * M + c) * W + ay] * gt[ay * W + ax];
        wl[i] = acc;
    }
    phase_sync();
    if constexpr (W > 16) {   // h = S_TS^T x_T - L_SL w_L
        // S_TS^T x_T row by row: each half-wavefront reads one (s, r) row of W consecutive
        // entries (a thread per row would stride W through the block and thrash the L1),
        // RB rows in flight, then a butterfly sum within the half
        static_assert(W <= 32, "one row per half-wavefront");
        constexpr int RB = 16;
        const int half = lane >> 5, gl = lane & 31, a = gl < W ? gl : W - 1;
        for (int base = 2 * wv; base < NS; base += 2 * nw * RB) {
            T v[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int row = base + half + 2 * nw * u, rr = row < NS ? row : NS - 1;
                const int s = rr / W, r = rr % W;
                const T e = Sy[(int64_t)s * NT + r * W + a] * gt[r * W + a];
                v[u] = row < NS && gl < W ? e : T(0);
            }
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                T x = v[u];
#pragma unroll
                for (int off = 16; off > 0; off >>= 1) x += __shfl_xor(x, off, 32);
                const int row = base + half + 2 * nw * u;
                if (gl == 0 && row < NS) zs[row] = x;
            }
        }
        phase_sync();
        for (int i = tid; i < NS; i += nt) {
            const int s = i / W, r = i % W;
            T acc = zs[i];
#pragma unroll
            for (int c = 0; c < 2 * M; ++c) acc -= B1[(int64_t)(s * 2 * M + c) * W + r] * wl[s * 2 * M + c];
            zs[i] = acc;
        }
    } else {
        for (int i = tid; i < NS; i += nt) {
            const int s = i / W, r = i % W;
            T acc = 0;
#pragma unroll
            for (int ax = 0; ax < W; ++ax) acc += Sy[(int64_t)s * NT + r * W + ax] * gt[r * W + ax];
#pragma unroll
            for (int c = 0; c < 2 * M; ++c) acc -= B1[(int64_t)(s * 2 * M + c) * W + r] * wl[s * 2 * M + c];
            zs[i] = acc;
        }
    }
    phase_sync();
    for (int s = wv; s < 2 * M; s += nw) {   // y_S -= L_SS^{-1} h, then x_S = L_SS^{-T} y_S
        const T d = tri_inv_mv<T>(Lsep + s * LS, W, 0, W, W, lane, zs + s * W);
        const T y = lane < W ? g[NL + s * W + lane] - d : T(0);
        const T x = tri_inv_t_mv_lanes<T>(Lsep + s * LS, W, W, lane, y);
        if (lane < W) g[NL + s * W + lane] = x;
    }
    phase_sync();
    for (int i = tid; i < NL; i += nt) {     // y_L = D_L^{-1} (y_L - L_SL^T y_S - L_TL^T x_T); the last is w_L
        int s = i / (2 * M), c = i % (2 * M);
        T v = g[i] - wl[i];
#pragma unroll
        for (int r = 0; r < W; ++r) v -= B1[(int64_t)(s * 2 * M + c) * W + r] * g[NL + s * W + r];
        g[i] = v * invd[i];
    }
    phase_sync();
    // ---- interface values and interior back-substitution into the patch box, OB outputs
    // per thread at a time with their r values loaded first (one round of latency per OB):
    // the whole box in one round while that takes at most 12 per thread, else 8 at a time
    const bool full[3] = {true, true, true};
    constexpr int W3 = W * W * W, OB1 = (W3 + NTH - 1) / NTH, OB = OB1 <= 12 ? OB1 : 8;
    for (int base = tid; base < W3; base += nt * OB) {
        T rv[OB];
#pragma unroll
        for (int u = 0; u < OB; ++u) {
            const int idx = base + u * nt;
            rv[u] = idx < W3 ? rF[C.gidx(idx % W, (idx / W) % W, idx / (W * W))] : T(0);
        }
#pragma unroll
        for (int u = 0; u < OB; ++u) {
            const int idx = base + u * nt;
            if (idx >= W3) break;
            const int ax = idx % W, ay = (idx / W) % W, az = idx / (W * W);
            const int ii = iface_interior(ax, ay, az, M, W, NL, NS);
            T val;
            if (ii >= 0) {
                val = g[ii];
            } else {
                const int pos[3] = {ax, ay, az};
                val = C.back_interior_r(pos, full, rv[u], [&](int a) {
                    int q[3] = {ax, ay, az};
                    q[a] = M;
                    return g[iface_interior(q[0], q[1], q[2], M, W, NL, NS)];
                });
            }
            if constexpr (PARITY) Uc[free_index(d, Z0 + az, Y0 + ay, X0 + ax)] = val;
            else Uc[idx] = val;
        }
    }
}

// Boundary-vertex patches: their stars lose cells, and the interface Schur complement
// splits into independent dense slices (2 full axes: crosses of 4m+1 DOFs; 1 full axis:
// single DOFs).  desc: vx, vy, vz, kind_x, kind_y, kind_z, nslices, slice size.
template <typename T, int P, int NTH>
__device__ __forceinline__ void patch_boundary(const int pid, Dims d, const int *__restrict__ desc,
                                               const int64_t *__restrict__ off, const T *__restrict__ factor,
                                               const T *__restrict__ mu, const T *__restrict__ lam,
                                               const T *__restrict__ afc, const T *__restrict__ rF, T *__restrict__ U) {
    constexpr int M = P - 1, W = 2 * M + 1, MAXN = 4 * M + 1;
    __shared__ T g[M * MAXN > M * M ? M * MAXN : M * M];
    __shared__ T smu[24], slam[M], safc[2 * M];
    constexpr int nt = NTH, nw = NTH / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int *ds = desc + 8 * pid;
    const int kind[3] = {ds[3], ds[4], ds[5]};
    stage_coefficients<T, M>(d, ds[0], ds[1], ds[2], kind, mu, lam, afc, smu, slam, safc);
    __syncthreads();
    PatchCtx<T, M> C{d, ds[0], ds[1], ds[2], rF, smu, slam, safc};
    const int nslices = ds[6], ns = ds[7], n = nslices * ns;
    const bool full[3] = {kind[0] == AX_FULL, kind[1] == AX_FULL, kind[2] == AX_FULL};
    int fa = -1, fb = -1, hh = -1, hb = -1, hc = -1;
    for (int a = 0; a < 3; ++a) {
        if (full[a]) { if (fa < 0) fa = a; else fb = a; }
        else { if (hb < 0) hb = a; else hc = a; }
    }
    const int nfull = full[0] + full[1] + full[2];
    if (nfull == 2) hh = hb;
    auto spos = [&](int a, int t) { return kind[a] == AX_LOW ? M + 1 + t : t; };
    auto sidx = [&](int a, int pos) { return kind[a] == AX_LOW ? pos - M - 1 : pos; };
    auto decode = [&](int idx, int pos[3]) {
        if (nfull == 2) {
            int t = idx / ns, c = idx % ns;
            pos[hh] = spos(hh, t);
            if (c < 2 * M) { pos[fa] = M; pos[fb] = inv_la_(c, M); }
            else { pos[fb] = M; pos[fa] = c - 2 * M; }
        } else {  // one full axis
            int tb = idx % M, tc = idx / M;
            pos[fa] = M; pos[hb] = spos(hb, tb); pos[hc] = spos(hc, tc);
        }
    };
    auto encode = [&](const int pos[3]) -> int {
        if (nfull == 2) {
            int t = sidx(hh, pos[hh]);
            int c = (pos[fa] == M && pos[fb] != M) ? la_(pos[fb], M) : 2 * M + pos[fa];
            return t * ns + c;
        }
        return sidx(hb, pos[hb]) + M * sidx(hc, pos[hc]);
    };
    constexpr bool PARITY = P > kFusedScatterMaxP;   // the layouts of patch_interior
    T *Uc = PARITY ? U + star_class(ds[0], ds[1], ds[2]) * ((int64_t)d.Lx * d.Ly * d.Lz)
                   : U + ((int64_t)(ds[2] * (d.ny + 1) + ds[1]) * (d.nx + 1) + ds[0]) * (int64_t)(W * W * W);
    const int X0 = ds[0] * P - M, Y0 = ds[1] * P - M, Z0 = ds[2] * P - M;
    for (int idx = tid; idx < n; idx += nt) {
        int pos[3];
        decode(idx, pos);
        int ncen = 0, dd = 0;
        for (int a = 0; a < 3; ++a)
            if (full[a] && pos[a] == M) { ++ncen; dd = a; }
        g[idx] = ncen == 1 ? C.condensed(pos, dd) : rF[C.gidx(pos[0], pos[1], pos[2])];
    }
    __syncthreads();
    const T *F = factor + (n > 0 ? off[pid] : 0);
    if (ns == 1) {
        for (int t = tid; t < nslices; t += nt) g[t] *= F[t] * F[t];
    } else if (ns > 1) {
        for (int t = wv; t < nslices; t += nw) {
            const T *Ls = F + (int64_t)t * (ns * (ns + 1) / 2);
            const T y = tri_inv_mv<T>(Ls, ns, 0, ns, ns, lane, g + t * ns);
            if (lane < ns) g[t * ns + lane] = y;
            const T x = tri_inv_t_mv<T>(Ls, ns, 0, ns, ns, lane, g + t * ns);
            if (lane < ns) g[t * ns + lane] = x;
        }
    }
    __syncthreads();
    int lo[3], cnt[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = kind[a] == AX_LOW ? M + 1 : 0;
        cnt[a] = kind[a] == AX_FULL ? W : M;
    }
    const int tot = cnt[0] * cnt[1] * cnt[2];
    for (int idx = tid; idx < tot; idx += nt) {
        int pos[3] = {lo[0] + idx % cnt[0], lo[1] + (idx / cnt[0]) % cnt[1], lo[2] + idx / (cnt[0] * cnt[1])};
        bool iface = (full[0] && pos[0] == M) || (full[1] && pos[1] == M) || (full[2] && pos[2] == M);
        T val;
        if (iface) {
            val = g[encode(pos)];
        } else {
            val = C.back_interior(pos, full, [&](int a) {
                int q[3] = {pos[0], pos[1], pos[2]};
                q[a] = M;
                return g[encode(q)];
            });
        }
        if constexpr (PARITY) Uc[free_index(d, Z0 + pos[2], Y0 + pos[1], X0 + pos[0])] = val;
        else Uc[(pos[2] * W + pos[1]) * W + pos[0]] = val;
    }
}


// Every patch of one relaxation in one launch: the interior-vertex stars first, then the
// boundary-vertex stars, whose short solves fill the CUs that the last round of interior
// patches leaves idle.
// Waves per SIMD the compiler must leave room for: 8 (64 VGPRs) for the 256-thread FP32
// kernels up to degree 7 with panel unroll 4, whose solves are latency-bound and gain
// more from the extra resident patch than they lose to the tighter register budget.
template <typename T, int P, int UNR, int NTH>
constexpr int patch_min_waves() { return sizeof(T) == 4 && P <= 7 && UNR <= 4 && NTH == 256 ? 8 : 1; }

template <typename T, int P, int UNR, int NTH>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(patch_min_waves<T, P, UNR, NTH>())))
k_patch_all(const double *__restrict__ gate, Dims d, PatchArgs A, int n_int,
                                                   const int *__restrict__ verts, const int *__restrict__ fidx,
                                                   const T *__restrict__ fint,
                                                   const int *__restrict__ desc, const int64_t *__restrict__ off,
                                                   const T *__restrict__ fbnd, const T *__restrict__ mu,
                                                   const T *__restrict__ lam, const T *__restrict__ afc,
                                                   const T *__restrict__ rF, T *__restrict__ U, CompStrides cs) {
    if (gated(gate)) return;
    if (gridDim.y > 1) {   // independent problems of one structure: blockIdx.y selects one
        const int64_t c = blockIdx.y;
        fint += c * cs.fint;
        fbnd += c * cs.fbnd;
        mu += c * cs.mu;
        rF += c * cs.rF;
        U += c * cs.U;
    }
    if ((int)blockIdx.x < n_int) patch_interior<T, P, UNR, NTH>(blockIdx.x, d, A, verts, fidx, fint, mu, lam, afc, rF, U);
    else patch_boundary<T, P, NTH>(blockIdx.x - n_int, d, desc, off, fbnd, mu, lam, afc, rF, U);
}

}  // namespace

template <typename T>
void launch_patch_all(const Dims &d, const PatchArgs &a, int n_int, const int *verts, const int *fidx, const T *fint, int n_bnd,
                      const int *desc, const int64_t *off, const T *fbnd, const T *mu, const T *lam, const T *afc,
                      const T *rF, T *U, const Exec &e, int ncomp, CompStrides cs) {
    if (n_int + n_bnd == 0) return;
    if (ncomp < 1 || ncomp > 65535) throw Error(VSR_EINVAL, "patch launch: bad problem count");
    const int unr = e.t.patch_unroll, nth = e.t.patch_threads;
    if (unr != 4 && unr != 8 && unr != 16) throw Error(VSR_EINVAL, "patch_unroll must be 4, 8 or 16");
    if (nth != 256 && nth != 512 && nth != 1024) throw Error(VSR_EINVAL, "patch_threads must be 256, 512 or 1024");
    if (nth == 1024 && unr == 16) throw Error(VSR_EINVAL, "1024 patch threads take an unroll of 4 or 8");
#define CALLT(P, UU, NN)                                                                                          \
    hipLaunchKernelGGL((k_patch_all<T, P, UU, NN>), dim3(n_int + n_bnd, ncomp), dim3(NN), 0, e.s, e.gate, d, a, n_int, verts, \
                       fidx, fint, desc, off, fbnd, mu, lam, afc, rF, U, cs)
#define CALLU(P, UU)                                       \
    if (nth == 512) CALLT(P, UU, 512);                      \
    else if (nth == 1024) {                                 \
        if constexpr (UU < 16) CALLT(P, UU, 1024);          \
    } else CALLT(P, UU, 256)
#define CALL(P)                          \
    if (unr == 4) { CALLU(P, 4); }       \
    else if (unr == 8) { CALLU(P, 8); }  \
    else { CALLU(P, 16); }
    VSR_P_SWITCH(d.p, CALL)
#undef CALL
#undef CALLU
#undef CALLT
}

}  // namespace vsr

#define VSR_INSTANTIATE_PATCH(T)                                                                                     \
    namespace vsr {                                                                                                  \
    template void launch_patch_all<T>(const Dims &, const PatchArgs &, int, const int *, const int *, const T *, int,   \
                                      const int *,                                                                   \
                                      const int64_t *, const T *, const T *, const T *, const T *, const T *, T *,   \
                                      const Exec &, int, CompStrides);                                              \
    }
