// Host-side setup in FP64: one-dimensional GLL/FDM data, geometry, vertex-star
// patch factorization, Q1 coarse matrix, lattice transfer tables.
//
// References are to Brubeck & Farrell, "A scalable and robust vertex-star
// relaxation for high-order FEM", Sec. 2.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "kernels.h"
#include "vsr_internal.h"

namespace vsr {

// ============================================================ one-dimensional data
// GLL nodes of order n = N+1: +-1 and the zeros of (1 - x^2) P_N'(x) = N (P_{N-1} - x P_N),
// whose derivative is -N(N+1) P_N (Legendre's equation), giving the Newton step
// x += (P_{N-1} - x P_N) / ((N+1) P_N).  Weights 2 / (N(N+1) P_N(x)^2).
static void legendre_pair(int N, double x, double &PN, double &PNm1) {
    double a = 1.0, b = x;  // P_0, P_1
    if (N == 0) { PN = 1.0; PNm1 = 0.0; return; }
    for (int k = 1; k < N; ++k) {
        double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
        a = b;
        b = c;
    }
    PN = b;
    PNm1 = a;
}

static void gll(int n, std::vector<double> &x, std::vector<double> &w) {
    int N = n - 1;
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    x[0] = -1.0;
    x[N] = 1.0;
    for (int k = 1; k < N; ++k) {
        double t = -std::cos(M_PI * k / N);
        for (int it = 0; it < 100; ++it) {
            double PN, PNm1;
            legendre_pair(N, t, PN, PNm1);
            double dt = (PNm1 - t * PN) / ((N + 1) * PN);
            t += dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        x[k] = t;
    }
    std::sort(x.begin(), x.end());
    for (int k = 0; k < n; ++k) {
        double PN, PNm1;
        legendre_pair(N, x[k], PN, PNm1);
        w[k] = 2.0 / (N * (N + 1) * PN * PN);
    }
}

// Lagrange basis on `nodes` evaluated at `pts` by the barycentric formula:
// l_j(x) = (c_j / (x - xi_j)) / sum_k c_k / (x - xi_k),  c_j = 1 / prod_{k != j} (xi_j - xi_k),
// l_j'(x) = l_j(x) sum_{k != j} 1 / (x - xi_k); at a node xi_i, l_j'(xi_i) = (c_j/c_i)/(xi_i - xi_j)
// and l_i'(xi_i) = -sum_{j != i} l_j'(xi_i).
static void lagrange_bary(const std::vector<double> &nodes, const std::vector<double> &pts,
                          std::vector<double> &V, std::vector<double> &D) {
    int n = (int)nodes.size(), np = (int)pts.size();
    std::vector<double> c(n, 1.0);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k)
            if (k != j) c[j] /= (nodes[j] - nodes[k]);
    V.assign((size_t)np * n, 0.0);
    D.assign((size_t)np * n, 0.0);
    for (int a = 0; a < np; ++a) {
        double x = pts[a];
        int hit = -1;
        for (int k = 0; k < n; ++k)
            if (std::fabs(x - nodes[k]) < 1e-14) hit = k;
        if (hit >= 0) {
            V[(size_t)a * n + hit] = 1.0;
            double s = 0.0;
            for (int j = 0; j < n; ++j) {
                if (j == hit) continue;
                double d = (c[j] / c[hit]) / (nodes[hit] - nodes[j]);
                D[(size_t)a * n + j] = d;
                s += d;
            }
            D[(size_t)a * n + hit] = -s;
            continue;
        }
        double den = 0.0;
        for (int k = 0; k < n; ++k) den += c[k] / (x - nodes[k]);
        for (int j = 0; j < n; ++j) {
            double l = (c[j] / (x - nodes[j])) / den;
            double s = 0.0;
            for (int k = 0; k < n; ++k)
                if (k != j) s += 1.0 / (x - nodes[k]);
            V[(size_t)a * n + j] = l;
            D[(size_t)a * n + j] = l * s;
        }
    }
}

// Cyclic Jacobi rotations for a symmetric matrix (row-major n x n): eigenvalues in
// `ev`, eigenvectors as the columns of Q.
static void jacobi_eig(int n, std::vector<double> A, std::vector<double> &ev, std::vector<double> &Q) {
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[(size_t)i * n + j] * A[(size_t)i * n + j];
                if (i != j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = cs * akp - sn * akq;
                    A[(size_t)k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = cs * apk - sn * aqk;
                    A[(size_t)q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double qkp = Q[(size_t)k * n + p], qkq = Q[(size_t)k * n + q];
                    Q[(size_t)k * n + p] = cs * qkp - sn * qkq;
                    Q[(size_t)k * n + q] = sn * qkp + cs * qkq;
                }
            }
    }
    ev.resize(n);
    for (int i = 0; i < n; ++i) ev[i] = A[(size_t)i * n + i];
}

// Inverse of the leading n x n block of a row-major lower-triangular L (leading dimension
// lda), packed column-major into nstore columns: column k holds rows k..nstore-1 from offset
// k nstore - k (k - 1) / 2; rows or columns at or beyond n are zero.  The inverse of a lower
// triangle is lower triangular, so it takes the storage of the factor itself; the solves
// become triangular matrix-vector products with independent rows (no elimination chain).
static void pack_lower_inverse(int n, const double *L, int lda, int nstore, double *out) {
    std::vector<double> x((size_t)n);
    size_t e = 0;
    for (int k = 0; k < nstore; ++k) {
        if (k < n) {   // column k of L^{-1}: forward substitution of L x = e_k
            for (int i = k; i < n; ++i) {
                double v = i == k ? 1.0 : 0.0;
                for (int j = k; j < i; ++j) v -= L[(size_t)i * lda + j] * x[j];
                x[i] = v / L[(size_t)i * lda + i];
            }
        }
        for (int i = k; i < nstore; ++i, ++e) out[e] = (k < n && i < n) ? x[i] : 0.0;
    }
}

// sum_k a[k] b[k] over k < n with eight independent partial sums, so that the dense setup
// loops (Schur updates, Cholesky, inverses) are not serialized on the latency of one add
static inline double dot8(const double *a, const double *b, int n) {
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int k = 0;
    for (; k + 8 <= n; k += 8)
        for (int u = 0; u < 8; ++u) s[u] += a[k + u] * b[k + u];
    for (; k < n; ++k) s[0] += a[k] * b[k];
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Lower triangle of a symmetric n x n block A (row-major, lda) packed like pack_lower_inverse
// (column k holds rows k..nstore-1 from offset k nstore - k (k - 1) / 2; zero beyond n).
static void pack_lower(int n, const double *A, int lda, int nstore, double *out) {
    size_t e = 0;
    for (int k = 0; k < nstore; ++k)
        for (int i = k; i < nstore; ++i, ++e) out[e] = (k < n && i < n) ? A[(size_t)i * lda + k] : 0.0;
}

// S^{-1} = L^{-T} L^{-1} from the lower Cholesky factor L of S (row-major, lda): the columns
// of L^{-1} by forward substitution (C[j][i] = (L^{-1})[i][j], i >= j), then the lower
// triangle of their Gram matrix, (S^{-1})[i][j] = sum_{k >= i} C[i][k] C[j][k] for i >= j.
static void inverse_from_cholesky(int n, const double *L, int lda, std::vector<double> &Sinv) {
    std::vector<double> C((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double *x = &C[(size_t)j * n];
        for (int i = j; i < n; ++i) {
            const double *li = L + (size_t)i * lda;
            const double v = (i == j ? 1.0 : 0.0) - dot8(li + j, x + j, i - j);
            x[i] = v / li[i];
        }
    }
    Sinv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) {
        const double *ci = &C[(size_t)i * n];
        for (int j = 0; j <= i; ++j) {
            const double *cj = &C[(size_t)j * n];
            Sinv[(size_t)i * n + j] = dot8(ci + i, cj + i, n - i);
        }
    }
}

// Dense Cholesky in place (row-major, lower), returns false on a non-positive pivot.
static bool cholesky_lower(int n, double *a, int lda) {
    for (int j = 0; j < n; ++j) {
        double d = a[(size_t)j * lda + j] - dot8(a + (size_t)j * lda, a + (size_t)j * lda, j);
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        a[(size_t)j * lda + j] = d;
        double inv = 1.0 / d;
        for (int i = j + 1; i < n; ++i) {
            const double *ri = a + (size_t)i * lda, *rj = a + (size_t)j * lda;
            a[(size_t)i * lda + j] = (a[(size_t)i * lda + j] - dot8(ri, rj, j)) * inv;
        }
    }
    return true;
}

OneD make_1d(int p, int q) {
    OneD d;
    d.p = p;
    d.q = q;
    std::vector<double> wn;
    gll(p + 1, d.xi, wn);
    gll(q, d.xq, d.wq);
    lagrange_bary(d.xi, d.xq, d.Iq, d.Dq);
    int n = p + 1;
    d.A.assign((size_t)n * n, 0.0);
    d.B.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double a = 0, b = 0;
            for (int k = 0; k < q; ++k) {
                a += d.wq[k] * d.Dq[(size_t)k * n + i] * d.Dq[(size_t)k * n + j];
                b += d.wq[k] * d.Iq[(size_t)k * n + i] * d.Iq[(size_t)k * n + j];
            }
            d.A[(size_t)i * n + j] = a;
            d.B[(size_t)i * n + j] = b;
        }
    // interior generalized eigenproblem A_II S = B_II S Lambda, S^T B_II S = I (Sec. 2.3)
    int m = p - 1;
    std::vector<double> L((size_t)m * m), Ai((size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            L[(size_t)i * m + j] = d.B[(size_t)(i + 1) * n + j + 1];
            Ai[(size_t)i * m + j] = d.A[(size_t)(i + 1) * n + j + 1];
        }
    if (!cholesky_lower(m, L.data(), m)) throw Error(VSR_EINVAL, "interior mass matrix not SPD");
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j) L[(size_t)i * m + j] = 0.0;
    // C = L^{-1} A_II L^{-T}: solve L X = A_II, then L C^T = X^T
    std::vector<double> X = Ai;
    for (int c = 0; c < m; ++c)
        for (int i = 0; i < m; ++i) {
            double s = X[(size_t)i * m + c];
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * m + k] * X[(size_t)k * m + c];
            X[(size_t)i * m + c] = s / L[(size_t)i * m + i];
        }
    std::vector<double> C((size_t)m * m);
    for (int r = 0; r < m; ++r)         // row r of C = (L^{-1} row r of X^T)...: C = X L^{-T}
        for (int j = 0; j < m; ++j) {
            double s = X[(size_t)r * m + j];
            for (int k = 0; k < j; ++k) s -= C[(size_t)r * m + k] * L[(size_t)j * m + k];
            C[(size_t)r * m + j] = s / L[(size_t)j * m + j];
        }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < i; ++j) {
            double s = 0.5 * (C[(size_t)i * m + j] + C[(size_t)j * m + i]);
            C[(size_t)i * m + j] = C[(size_t)j * m + i] = s;
        }
    std::vector<double> ev, Q;
    jacobi_eig(m, C, ev, Q);
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return ev[a] < ev[b]; });
    // S = L^{-T} Q (back substitution with L^T), columns in ascending eigenvalue order
    std::vector<double> S((size_t)m * m);
    for (int jj = 0; jj < m; ++jj) {
        int j = order[jj];
        for (int i = m - 1; i >= 0; --i) {
            double s = Q[(size_t)i * m + j];
            for (int k = i + 1; k < m; ++k) s -= L[(size_t)k * m + i] * S[(size_t)k * m + jj];
            S[(size_t)i * m + jj] = s / L[(size_t)i * m + i];
        }
        if (S[jj] < 0)
            for (int i = 0; i < m; ++i) S[(size_t)i * m + jj] = -S[(size_t)i * m + jj];
    }
    d.lam.resize(m);
    for (int jj = 0; jj < m; ++jj) d.lam[jj] = ev[order[jj]];
    // FDM basis (Sec. 2.4): columns of T are GLL coefficients of the basis dual to
    // {u(-1), u(+1), int u s_k}: interior columns S; vertex columns l_0, l_p corrected by
    // -B_II^{-1} B_I0, -B_II^{-1} B_Ip.
    d.T.assign((size_t)n * n, 0.0);
    d.T[0] = 1.0;
    d.T[(size_t)p * n + p] = 1.0;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) d.T[(size_t)(i + 1) * n + j + 1] = S[(size_t)i * m + j];
    for (int e = 0; e < 2; ++e) {
        int col = e == 0 ? 0 : p;
        std::vector<double> rhs(m);
        for (int i = 0; i < m; ++i) rhs[i] = -d.B[(size_t)(i + 1) * n + col];
        for (int i = 0; i < m; ++i) {  // L y = rhs
            double s = rhs[i];
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * m + k] * rhs[k];
            rhs[i] = s / L[(size_t)i * m + i];
        }
        for (int i = m - 1; i >= 0; --i) {  // L^T x = y
            double s = rhs[i];
            for (int k = i + 1; k < m; ++k) s -= L[(size_t)k * m + i] * rhs[k];
            rhs[i] = s / L[(size_t)i * m + i];
        }
        for (int i = 0; i < m; ++i) d.T[(size_t)(i + 1) * n + col] = rhs[i];
    }
    // A_F = T^T A T, B_F = T^T B T, with the zeros the construction guarantees imposed exactly
    d.Af.assign((size_t)n * n, 0.0);
    d.Bf.assign((size_t)n * n, 0.0);
    std::vector<double> AT((size_t)n * n), BT((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double a = 0, b = 0;
            for (int k = 0; k < n; ++k) {
                a += d.A[(size_t)i * n + k] * d.T[(size_t)k * n + j];
                b += d.B[(size_t)i * n + k] * d.T[(size_t)k * n + j];
            }
            AT[(size_t)i * n + j] = a;
            BT[(size_t)i * n + j] = b;
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double a = 0, b = 0;
            for (int k = 0; k < n; ++k) {
                a += d.T[(size_t)k * n + i] * AT[(size_t)k * n + j];
                b += d.T[(size_t)k * n + i] * BT[(size_t)k * n + j];
            }
            d.Af[(size_t)i * n + j] = a;
            d.Bf[(size_t)i * n + j] = b;
        }
    for (int i = 1; i < p; ++i) {
        for (int j = 1; j < p; ++j) {
            d.Af[(size_t)i * n + j] = (i == j) ? d.lam[i - 1] : 0.0;
            d.Bf[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
        }
        d.Bf[(size_t)i * n + 0] = d.Bf[(size_t)0 * n + i] = 0.0;
        d.Bf[(size_t)i * n + p] = d.Bf[(size_t)p * n + i] = 0.0;
    }
    return d;
}

// ============================================================ geometry (Sec. 2.7)
Geometry make_geometry(int nx, int ny, int nz, const double *V, const double *kappa, const OneD &od,
                       bool keep_metric) {
    Geometry g;
    int q = od.q;
    int64_t ncell = (int64_t)nx * ny * nz, nq3 = (int64_t)q * q * q;
    auto vid = [&](int i, int j, int k) { return 3 * ((int64_t)i + (nx + 1) * ((int64_t)j + (ny + 1) * (int64_t)k)); };
    // Cartesian test: every cell an axis-aligned box
    bool cart = true;
    for (int k = 0; k < nz && cart; ++k)
        for (int j = 0; j < ny && cart; ++j)
            for (int i = 0; i < nx && cart; ++i)
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            const double *X = V + vid(i + a, j + b, k + c);
                            double h = std::fabs(V[vid(i + 1, j, k)] - V[vid(i, j, k)]) + 1e-300;
                            if (std::fabs(X[0] - V[vid(i + a, j, k)]) > 1e-13 * h ||
                                std::fabs(X[1] - V[vid(i, j + b, k) + 1]) > 1e-13 * h ||
                                std::fabs(X[2] - V[vid(i, j, k + c) + 2]) > 1e-13 * h)
                                cart = false;
                        }
    g.cartesian = cart;
    g.mu.assign(ncell * 3, 0.0);
    g.wdet.assign(ncell * nq3, 0.0);
    if (!cart || keep_metric) g.Gw.assign(ncell * 6 * nq3, 0.0);
    bool store = !g.Gw.empty();
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t e = 0; e < ncell; ++e) {
        int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((int64_t)nx * ny));
        double X[2][2][2][3];
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a)
                    for (int d = 0; d < 3; ++d) X[c][b][a][d] = V[vid(i + a, j + b, k + c) + d];
        double kap = kappa ? kappa[e] : 1.0;
        double mu0 = 0, mu1 = 0, mu2 = 0;
        for (int c = 0; c < q; ++c)
            for (int b = 0; b < q; ++b)
                for (int a = 0; a < q; ++a) {
                    double xs[3] = {od.xq[a], od.xq[b], od.xq[c]};
                    double N[3][2], dN[3][2];
                    for (int d = 0; d < 3; ++d) {
                        N[d][0] = 0.5 * (1 - xs[d]);
                        N[d][1] = 0.5 * (1 + xs[d]);
                        dN[d][0] = -0.5;
                        dN[d][1] = 0.5;
                    }
                    double J[3][3] = {{0}};
                    for (int cc = 0; cc < 2; ++cc)
                        for (int bb = 0; bb < 2; ++bb)
                            for (int aa = 0; aa < 2; ++aa) {
                                double g0 = dN[0][aa] * N[1][bb] * N[2][cc];
                                double g1 = N[0][aa] * dN[1][bb] * N[2][cc];
                                double g2 = N[0][aa] * N[1][bb] * dN[2][cc];
                                for (int d = 0; d < 3; ++d) {
                                    J[d][0] += g0 * X[cc][bb][aa][d];
                                    J[d][1] += g1 * X[cc][bb][aa][d];
                                    J[d][2] += g2 * X[cc][bb][aa][d];
                                }
                            }
                    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                    if (!(det > 0)) {
                        bad += 1;
                        continue;
                    }
                    // adjugate / det = J^{-1}
                    double Ji[3][3];
                    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
                    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
                    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
                    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
                    double G[3][3];
                    for (int r = 0; r < 3; ++r)
                        for (int s = 0; s < 3; ++s) {
                            double t = 0;
                            for (int u = 0; u < 3; ++u) t += Ji[r][u] * Ji[s][u];
                            G[r][s] = kap * det * t;
                        }
                    double w = od.wq[a] * od.wq[b] * od.wq[c];
                    int64_t pt = ((int64_t)c * q + b) * q + a;
                    g.wdet[e * nq3 + pt] = w * det;
                    mu0 += w * G[0][0];
                    mu1 += w * G[1][1];
                    mu2 += w * G[2][2];
                    if (store) {
                        double *o = &g.Gw[(e * 6) * nq3 + pt];
                        o[0 * nq3] = w * G[0][0];
                        o[1 * nq3] = w * G[1][1];
                        o[2 * nq3] = w * G[2][2];
                        o[3 * nq3] = w * G[0][1];
                        o[4 * nq3] = w * G[0][2];
                        o[5 * nq3] = w * G[1][2];
                    }
                }
        g.mu[e * 3 + 0] = mu0 / 8.0;
        g.mu[e * 3 + 1] = mu1 / 8.0;
        g.mu[e * 3 + 2] = mu2 / 8.0;
    }
    if (bad) throw Error(VSR_EMESH, "det(DF) <= 0 at " + std::to_string(bad) + " quadrature points");
    return g;
}

// ============================================================ patches (Sec. 2.5, 2.6)
static inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

InteriorLayout interior_layout(int p) {
    InteriorLayout L;
    int m = p - 1, w = 2 * m + 1;
    L.m = m;
    L.w = w;
    L.n_leaf = 4 * m * m;
    L.n_sep = 2 * m * w;
    L.n_top = w * w;
    L.n_iface = L.n_leaf + L.n_sep + L.n_top;
    L.top_pad = (int)round_up(L.n_top, 4);
    int64_t o = 0;
    L.off_invd = o; o += L.n_leaf;
    o = round_up(o, 4);
    L.off_B1 = o; o += (int64_t)2 * m * 2 * m * w;
    L.off_B2 = o; o += (int64_t)2 * m * 2 * m * w;
    o = round_up(o, 4);
    L.off_Lsep = o; o += (int64_t)2 * m * (w * (w + 1) / 2);
    o = round_up(o, 4);
    // raw top-plane x level-1 Schur block, y-diagonal: Sy[s][ay][ax] couples top (ax, ay) with
    // separator (s, ay) (it replaces the dense panel L_TS = (S_TS - L_TL L_SL^T) L_SS^{-T})
    L.off_Sy = o; o += (int64_t)w * w * 2 * m;
    o = round_up(o, 4);
    L.off_Ltop = o;
    L.ntiles = (L.n_top + 63) / 64;
    for (int J = 0; J < L.ntiles; ++J) {
        int c0 = 64 * J, nb = std::min(64, L.n_top - c0);
        int rows = L.n_top - c0 - nb;
        int rp = (int)round_up(rows, 4);
        L.tile_off.push_back(o);
        L.tile_rows_pad.push_back(rp);
        // the diagonal block is packed in 64 columns; the last (possibly narrower) block in its own width
        const int ns = J + 1 < L.ntiles ? 64 : nb;
        o += ns * (ns + 1) / 2 + (int64_t)64 * rp;
    }
    L.stride = round_up(o, 64);
    return L;
}

namespace {

struct Star {
    int kind[3];           // per axis (x, y, z)
    const double *mu[2][2][2];  // [cz][cy][cx] cell scalings, NULL if the cell is absent
};

inline bool cell_exists(int kind, int c) { return kind == AX_FULL || (kind == AX_LOW ? c == 1 : c == 0); }
inline int la(int a, int m) { return a < m ? a : a - 1; }

// Interface index of box coordinates (-1 if interior).  Interior class: leaves, level-1
// separators, top plane; boundary classes: slice-major cross / plane layout.
struct IfaceMap {
    int m, w, cls;          // cls: 3 full axes (interior), 2 (face), 1 (edge), 0 (corner)
    int kind[3];
    int full_a = -1, full_b = -1, half_h = -1;   // face class axes
    int ns = 0, nslices = 0, n = 0;
    int slice_pos(int ax, int pos) const { return kind[ax] == AX_LOW ? pos - m - 1 : pos; }
    int operator()(const int pos[3]) const {
        if (cls == 3) {
            int ax = pos[0], ay = pos[1], az = pos[2];
            int n_leaf = 4 * m * m, n_sep = 2 * m * w;
            if (az == m) return n_leaf + n_sep + ay * w + ax;
            if (ax == m) return n_leaf + la(az, m) * w + ay;
            if (ay == m) return la(az, m) * 2 * m + la(ax, m);
            return -1;
        }
        if (cls == 2) {
            int pa = pos[full_a], pb = pos[full_b];
            if (pa != m && pb != m) return -1;
            int t = slice_pos(half_h, pos[half_h]);
            int c = (pa == m && pb != m) ? la(pb, m) : 2 * m + pa;
            return t * ns + c;
        }
        if (cls == 1) {
            int a = -1, b = -1, c = -1;
            for (int d = 0; d < 3; ++d)
                if (kind[d] == AX_FULL) a = d;
            for (int d = 0; d < 3; ++d)
                if (d != a) { if (b < 0) b = d; else c = d; }
            if (pos[a] != m) return -1;
            return slice_pos(b, pos[b]) + m * slice_pos(c, pos[c]);
        }
        return -1;
    }
};

IfaceMap make_map(int p, const int kind[3]) {
    IfaceMap M;
    M.m = p - 1;
    M.w = 2 * M.m + 1;
    int nfull = 0;
    for (int d = 0; d < 3; ++d) {
        M.kind[d] = kind[d];
        nfull += kind[d] == AX_FULL;
    }
    M.cls = nfull;
    int m = M.m;
    if (nfull == 3) {
        M.n = 4 * m * m + 2 * m * M.w + M.w * M.w;
    } else if (nfull == 2) {
        for (int d = 0; d < 3; ++d) {
            if (kind[d] == AX_FULL) { if (M.full_a < 0) M.full_a = d; else M.full_b = d; }
            else M.half_h = d;
        }
        M.ns = 4 * m + 1;
        M.nslices = m;
        M.n = M.ns * m;
    } else if (nfull == 1) {
        M.ns = 1;
        M.nslices = m * m;
        M.n = m * m;
    } else {
        M.n = 0;
    }
    return M;
}

// Dense interface Schur complement S = A_GG - A_GI A_II^{-1} A_IG of the FDM-basis patch
// matrix of the separable surrogate (Sec. 2.4, 2.6, 2.7), row-major n x n.
void assemble_schur(const OneD &od, const Star &st, const IfaceMap &M, std::vector<double> &S) {
    int p = od.p, m = p - 1, n1 = p + 1;
    int n = M.n;
    S.assign((size_t)n * n, 0.0);
    const double *Af = od.Af.data(), *Bf = od.Bf.data();
    // 1D partners: the j with A_F[i][j] or B_F[i][j] nonzero (an interior FDM function
    // couples to itself and the two vertex functions only).  A pair of cell nodes couples
    // only if it is a partner pair along every axis (each term of the Kronecker sum has an
    // A_F or B_F factor per axis), so only those pairs are visited.
    std::vector<std::vector<int>> partner(n1);
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j)
            if (Af[i * n1 + j] != 0.0 || Bf[i * n1 + j] != 0.0) partner[i].push_back(j);
    std::vector<int> ids, lz, ly, lx, cell_node((size_t)n1 * n1 * n1);
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const double *mu = st.mu[cz][cy][cx];
                if (!mu) continue;
                int cc[3] = {cx, cy, cz};
                int lo[3], hi[3];
                for (int d = 0; d < 3; ++d) {
                    lo[d] = cc[d] == 0 ? 0 : m;
                    hi[d] = cc[d] == 0 ? m : 2 * m;
                    // on a half axis the star's central plane is the Dirichlet boundary
                    if (st.kind[d] != AX_FULL) {
                        if (cc[d] == 1) lo[d] = m + 1;
                        else hi[d] = m - 1;
                    }
                }
                ids.clear(); lz.clear(); ly.clear(); lx.clear();
                for (int az = lo[2]; az <= hi[2]; ++az)
                    for (int ay = lo[1]; ay <= hi[1]; ++ay)
                        for (int ax = lo[0]; ax <= hi[0]; ++ax) {
                            int pos[3] = {ax, ay, az};
                            int id = M(pos);
                            if (id < 0) continue;
                            ids.push_back(id);
                            lx.push_back(ax + 1 - cx * p);
                            ly.push_back(ay + 1 - cy * p);
                            lz.push_back(az + 1 - cz * p);
                        }
                int nc = (int)ids.size();
                std::fill(cell_node.begin(), cell_node.end(), -1);
                for (int s = 0; s < nc; ++s) cell_node[((size_t)lz[s] * n1 + ly[s]) * n1 + lx[s]] = s;
                for (int s = 0; s < nc; ++s)
                    for (int jz : partner[lz[s]])
                        for (int jy : partner[ly[s]])
                            for (int jx : partner[lx[s]]) {
                                const int t = cell_node[((size_t)jz * n1 + jy) * n1 + jx];
                                if (t < 0) continue;
                                double bz = Bf[lz[s] * n1 + jz], by = Bf[ly[s] * n1 + jy], bx = Bf[lx[s] * n1 + jx];
                                double az_ = Af[lz[s] * n1 + jz], ay_ = Af[ly[s] * n1 + jy], ax_ = Af[lx[s] * n1 + jx];
                                double v = mu[0] * bz * by * ax_ + mu[1] * bz * ay_ * bx + mu[2] * az_ * by * bx;
                                if (v != 0.0) S[(size_t)ids[s] * n + ids[t]] += v;
                            }
                // condensation of the cell's interior DOFs
                int e[3];
                for (int d = 0; d < 3; ++d) e[d] = cc[d] == 0 ? p : 0;
                for (int az = lo[2]; az <= hi[2]; ++az)
                    for (int ay = lo[1]; ay <= hi[1]; ++ay)
                        for (int ax = lo[0]; ax <= hi[0]; ++ax) {
                            if (ax == m || ay == m || az == m) continue;
                            int pos[3] = {ax, ay, az};
                            int l[3] = {ax + 1 - cx * p, ay + 1 - cy * p, az + 1 - cz * p};
                            double D = mu[0] * od.lam[l[0] - 1] + mu[1] * od.lam[l[1] - 1] + mu[2] * od.lam[l[2] - 1];
                            int fid[3];
                            double cf[3];
                            int nf = 0;
                            for (int d = 0; d < 3; ++d) {
                                if (st.kind[d] != AX_FULL) continue;
                                int q[3] = {pos[0], pos[1], pos[2]};
                                q[d] = m;
                                fid[nf] = M(q);
                                cf[nf] = mu[d] * Af[l[d] * n1 + e[d]];
                                ++nf;
                            }
                            for (int s = 0; s < nf; ++s)
                                for (int t = 0; t < nf; ++t) S[(size_t)fid[s] * n + fid[t]] -= cf[s] * cf[t] / D;
                        }
            }
}

// Structured Cholesky of the interior-class Schur complement in the nested-dissection
// order leaves / level-1 separators / top plane (Sec. 2.6): writes one patch factor.
bool factor_interior(const InteriorLayout &L, std::vector<double> &S, double *out, bool check) {
    int m = L.m, w = L.w, n = L.n_iface, nl = L.n_leaf, ns = L.n_sep, nt = L.n_top;
    auto leaf = [&](int s, int c) { return s * 2 * m + c; };          // slice s = la(az), c = la(ax)
    auto sep = [&](int s, int r) { return nl + s * w + r; };          // r = ay
    auto top = [&](int ay, int ax) { return nl + ns + ay * w + ax; };
    auto inv_la = [&](int c) { return c < m ? c : c + 1; };
    double *Sd = S.data();
    auto at = [&](int i, int j) -> double & { return Sd[(size_t)i * n + j]; };
    if (check) {
        // every nonzero lies in a block the factorization visits
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double v = at(i, j);
                if (v == 0.0 || i == j) continue;
                bool li = i < nl, lj = j < nl, si = i >= nl && i < nl + ns, sj = j >= nl && j < nl + ns;
                bool ok = true;
                if (li && lj) ok = false;
                if (si && sj) ok = (i - nl) / w == (j - nl) / w;
                if ((li && sj) || (si && lj)) {
                    int a = li ? i : j, b = li ? j : i;
                    ok = a / (2 * m) == (b - nl) / w;
                }
                if ((li && !lj && !sj) || (lj && !li && !si)) {
                    int a = li ? i : j, b = li ? j : i;
                    ok = inv_la(a % (2 * m)) == (b - nl - ns) % w;
                }
                if (!ok) return false;
            }
    }
    // leaves: diagonal
    std::vector<double> invd(nl);
    for (int i = 0; i < nl; ++i) {
        double d = at(i, i);
        if (!(d > 0)) return false;
        invd[i] = 1.0 / std::sqrt(d);
        out[L.off_invd + i] = invd[i];
    }
    // B1[s][c][r] = S[sep(s,r)][leaf(s,c)] / d ; B2[lx][c][r] = S[top(r,ax)][leaf(c,lx)] / d
    std::vector<double> B1((size_t)2 * m * 2 * m * w), B2((size_t)2 * m * 2 * m * w);
    for (int s = 0; s < 2 * m; ++s)
        for (int c = 0; c < 2 * m; ++c)
            for (int r = 0; r < w; ++r) B1[((size_t)s * 2 * m + c) * w + r] = at(sep(s, r), leaf(s, c)) * invd[leaf(s, c)];
    for (int lx = 0; lx < 2 * m; ++lx)
        for (int c = 0; c < 2 * m; ++c)
            for (int r = 0; r < w; ++r)
                B2[((size_t)lx * 2 * m + c) * w + r] = at(top(r, inv_la(lx)), leaf(c, lx)) * invd[leaf(c, lx)];
    std::memcpy(out + L.off_B1, B1.data(), B1.size() * sizeof(double));
    std::memcpy(out + L.off_B2, B2.data(), B2.size() * sizeof(double));
    // the raw top x separator block before the leaves update it: it couples top (ax, ay) only
    // with separators (s, ay) (both sides' 1D factors meet in one interior line)
    for (int ay = 0; ay < w; ++ay)
        for (int ax = 0; ax < w; ++ax)
            for (int s = 0; s < 2 * m; ++s) {
                for (int r = 0; r < w; ++r)
                    if (r != ay && at(top(ay, ax), sep(s, r)) != 0.0) return false;
                out[L.off_Sy + ((int64_t)s * w + ay) * w + ax] = at(top(ay, ax), sep(s, ay));
            }
    // Schur updates by the leaves
    for (int s = 0; s < 2 * m; ++s)
        for (int r1 = 0; r1 < w; ++r1)
            for (int r2 = 0; r2 < w; ++r2) {
                double t = 0;
                for (int c = 0; c < 2 * m; ++c) t += B1[((size_t)s * 2 * m + c) * w + r1] * B1[((size_t)s * 2 * m + c) * w + r2];
                at(sep(s, r1), sep(s, r2)) -= t;
            }
    for (int s = 0; s < 2 * m; ++s)        // leaf (s, lx) couples sep slice s with top line lx
        for (int lx = 0; lx < 2 * m; ++lx) {
            const double *b1 = &B1[((size_t)s * 2 * m + lx) * w];
            const double *b2 = &B2[((size_t)lx * 2 * m + s) * w];
            int ax = inv_la(lx);
            for (int ay = 0; ay < w; ++ay)
                for (int r = 0; r < w; ++r) at(top(ay, ax), sep(s, r)) -= b2[ay] * b1[r];
        }
    for (int lx = 0; lx < 2 * m; ++lx) {
        int ax = inv_la(lx);
        for (int a1 = 0; a1 < w; ++a1)
            for (int a2 = 0; a2 < w; ++a2) {
                double t = 0;
                for (int c = 0; c < 2 * m; ++c) t += B2[((size_t)lx * 2 * m + c) * w + a1] * B2[((size_t)lx * 2 * m + c) * w + a2];
                at(top(a1, ax), top(a2, ax)) -= t;
            }
    }
    // level-1 separators: Cholesky per slice, panel P_s = S[top, sep_s] L_s^{-T}
    std::vector<double> Ls((size_t)w * w), Pall((size_t)nt * 2 * m * w);   // Pall row-major [row][col]
    int ncol = 2 * m * w;
    for (int s = 0; s < 2 * m; ++s) {
        for (int i = 0; i < w; ++i)
            for (int j = 0; j < w; ++j) Ls[(size_t)i * w + j] = at(sep(s, i), sep(s, j));
        if (!cholesky_lower(w, Ls.data(), w)) return false;
        pack_lower_inverse(w, Ls.data(), w, w, out + L.off_Lsep + (int64_t)s * (w * (w + 1) / 2));
        for (int r = 0; r < nt; ++r) {
            double *pr = &Pall[(size_t)r * ncol + s * w];
            for (int j = 0; j < w; ++j) {
                const double v = at(nl + ns + r, sep(s, j)) - dot8(pr, Ls.data() + (size_t)j * w, j);
                pr[j] = v / Ls[(size_t)j * w + j];
            }
        }
    }
    // (Pall itself is not stored: the solve applies it as (S_TS - L_TL L_SL^T) L_SS^{-T})
    // top plane: S_top -= Pall Pall^T (lower triangle), then dense Cholesky
    std::vector<double> T((size_t)nt * nt);
    for (int i = 0; i < nt; ++i)
        for (int j = 0; j <= i; ++j) T[(size_t)i * nt + j] = at(nl + ns + i, nl + ns + j);
    const int BS = 64;
    for (int ib = 0; ib < nt; ib += BS)
        for (int jb = 0; jb <= ib; jb += BS)
            for (int kb = 0; kb < ncol; kb += 256) {
                int ie = std::min(nt, ib + BS), je = std::min(nt, jb + BS), ke = std::min(ncol, kb + 256);
                for (int i = ib; i < ie; ++i) {
                    const double *pi = &Pall[(size_t)i * ncol];
                    int jmax = std::min(je, i + 1);
                    for (int j = jb; j < jmax; ++j) {
                        const double *pj = &Pall[(size_t)j * ncol];
                        T[(size_t)i * nt + j] -= dot8(pi + kb, pj + kb, ke - kb);
                    }
                }
            }
    if (!cholesky_lower(nt, T.data(), nt)) return false;
    // the solve applies the top plane's S_T^{-1} = L^{-T} L^{-1} (symmetric) in one pass
    // instead of the two triangular sweeps: its lower triangle in 64-column tiles
    std::vector<double> Si;
    inverse_from_cholesky(nt, T.data(), nt, Si);
    for (int J = 0; J < L.ntiles; ++J) {
        int c0 = 64 * J, nb = std::min(64, nt - c0);
        double *D = out + L.tile_off[J];   // diagonal block, packed in 64 columns (the last in nb)
        pack_lower(nb, Si.data() + (size_t)c0 * nt + c0, nt, J + 1 < L.ntiles ? 64 : nb, D);
        int rp = L.tile_rows_pad[J], r0 = c0 + nb;
        double *Pn = D + 64 * 65 / 2;
        for (int k = 0; k < 64; ++k)
            for (int rr = 0; rr < rp; ++rr) {
                int r = r0 + rr;
                Pn[(size_t)k * rp + rr] = (k < nb && r < nt) ? Si[(size_t)r * nt + c0 + k] : 0.0;
            }
    }
    return true;
}

// Boundary classes: independent dense slices (packed inverses of their Cholesky factors).
bool factor_slices(const IfaceMap &M, std::vector<double> &S, double *out) {
    int n = M.n, ns = M.ns;
    std::vector<double> Ls((size_t)ns * ns);
    for (int t = 0; t < M.nslices; ++t) {
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j) Ls[(size_t)i * ns + j] = S[(size_t)(t * ns + i) * n + t * ns + j];
        if (!cholesky_lower(ns, Ls.data(), ns)) return false;
        pack_lower_inverse(ns, Ls.data(), ns, ns, out + (int64_t)t * (ns * (ns + 1) / 2));
    }
    return true;
}

}  // namespace

PatchSet make_patches(int nx, int ny, int nz, const OneD &od, const double *mu, bool interior_only, bool share) {
    PatchSet P;
    int p = od.p, m = p - 1;
    P.L = interior_layout(p);
    int nv[3] = {nx, ny, nz};
    auto kind_of = [&](int v, int ncell) { return v == 0 ? AX_LOW : (v == ncell ? AX_HIGH : AX_FULL); };
    for (int vz = 0; vz <= nz; ++vz)
        for (int vy = 0; vy <= ny; ++vy)
            for (int vx = 0; vx <= nx; ++vx) {
                int v[3] = {vx, vy, vz};
                int kind[3], nfull = 0;
                for (int d = 0; d < 3; ++d) {
                    kind[d] = kind_of(v[d], nv[d]);
                    nfull += kind[d] == AX_FULL;
                }
                if (nfull == 3) {
                    P.interior_vertices.insert(P.interior_vertices.end(), {vx, vy, vz});
                    continue;
                }
                if (interior_only) continue;
                int kk[3] = {kind[0], kind[1], kind[2]};
                IfaceMap M = make_map(p, kk);
                P.boundary_desc.insert(P.boundary_desc.end(), {vx, vy, vz, kind[0], kind[1], kind[2], M.nslices, M.ns});
            }
    int64_t ni = (int64_t)P.interior_vertices.size() / 3, nb = (int64_t)P.boundary_desc.size() / 8;
    auto star_of = [&](int vx, int vy, int vz, Star &st) {
        int v[3] = {vx, vy, vz};
        for (int d = 0; d < 3; ++d) st.kind[d] = kind_of(v[d], nv[d]);
        for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                    bool ok = cell_exists(st.kind[0], cx) && cell_exists(st.kind[1], cy) && cell_exists(st.kind[2], cz);
                    int ex = vx - 1 + cx, ey = vy - 1 + cy, ez = vz - 1 + cz;
                    st.mu[cz][cy][cx] = ok ? mu + 3 * ((int64_t)ex + nx * ((int64_t)ey + ny * (int64_t)ez)) : nullptr;
                }
    };
    // A star's patch matrix depends only on its class and its cells' scalings.  The key of a
    // star is its class and those scalings to 11 significant digits: the cell averages of
    // equal cells differ in the last bits with the cell's position, so stars that agree to
    // that precision (every interior star of a uniform Cartesian mesh with constant kappa)
    // share the factor of the first of them.  Without sharing every star gets its own factor.
    auto key_of = [&](const int32_t *v, const int *kind) {
        Star st;
        star_of(v[0], v[1], v[2], st);
        std::string k = std::to_string(kind[0]) + "," + std::to_string(kind[1]) + "," + std::to_string(kind[2]);
        char buf[32];
        for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx)
                    for (int c = 0; c < 3; ++c) {
                        const double *m3 = st.mu[cz][cy][cx];
                        std::snprintf(buf, sizeof buf, ",%.10e", m3 ? m3[c] : 0.0);
                        k += buf;
                    }
        return k;
    };
    std::vector<int64_t> int_rep;   // a representative interior patch per factor
    P.interior_factor_of.assign((size_t)ni, 0);
    {
        std::map<std::string, int32_t> seen;
        const int kf[3] = {AX_FULL, AX_FULL, AX_FULL};
        for (int64_t i = 0; i < ni; ++i) {
            int32_t f = (int32_t)int_rep.size();
            if (share) {
                auto ins = seen.emplace(key_of(&P.interior_vertices[3 * i], kf), f);
                f = ins.first->second;
                if (!ins.second) {
                    P.interior_factor_of[(size_t)i] = f;
                    continue;
                }
            }
            P.interior_factor_of[(size_t)i] = f;
            int_rep.push_back(i);
        }
    }
    P.n_interior_factors = (int64_t)int_rep.size();
    std::vector<int64_t> bnd_rep;   // boundary patches that own their factor
    P.boundary_off.assign((size_t)nb, 0);
    {
        std::map<std::string, int64_t> seen;
        for (int64_t i = 0; i < nb; ++i) {
            const int32_t *dsc = &P.boundary_desc[8 * i];
            const int64_t entries = (int64_t)dsc[6] * (dsc[7] * (dsc[7] + 1) / 2);
            if (share) {
                const int kind[3] = {dsc[3], dsc[4], dsc[5]};
                auto ins = seen.emplace(key_of(dsc, kind), P.boundary_entries);
                if (!ins.second) {
                    P.boundary_off[(size_t)i] = ins.first->second;
                    continue;
                }
            }
            P.boundary_off[(size_t)i] = P.boundary_entries;
            P.boundary_entries += entries;
            bnd_rep.push_back(i);
        }
    }
    P.interior_factor.assign((size_t)(P.n_interior_factors * P.L.stride), 0.0);
    P.boundary_factor.assign((size_t)std::max<int64_t>(P.boundary_entries, 1), 0.0);
    int failed = 0;
    int kfull[3] = {AX_FULL, AX_FULL, AX_FULL};
    IfaceMap Mi = make_map(p, kfull);
    const int64_t nfi = P.n_interior_factors, nfb = (int64_t)bnd_rep.size();
#pragma omp parallel
    {
        std::vector<double> S;
#pragma omp for schedule(dynamic, 1) reduction(+ : failed)
        for (int64_t f = 0; f < nfi; ++f) {
            Star st;
            const int32_t *v = &P.interior_vertices[3 * int_rep[(size_t)f]];
            star_of(v[0], v[1], v[2], st);
            assemble_schur(od, st, Mi, S);
            if (!factor_interior(P.L, S, &P.interior_factor[(size_t)(f * P.L.stride)], f == 0)) failed += 1;
        }
#pragma omp for schedule(dynamic, 4) reduction(+ : failed)
        for (int64_t r = 0; r < nfb; ++r) {
            const int64_t i = bnd_rep[(size_t)r];
            const int32_t *dsc = &P.boundary_desc[8 * i];
            Star st;
            star_of(dsc[0], dsc[1], dsc[2], st);
            if (dsc[6] == 0) continue;
            IfaceMap M = make_map(p, st.kind);
            assemble_schur(od, st, M, S);
            if (!factor_slices(M, S, &P.boundary_factor[(size_t)P.boundary_off[(size_t)i]])) failed += 1;
        }
    }
    if (failed) throw Error(VSR_ENOTSPD, "patch Cholesky failed on " + std::to_string(failed) + " patches");
    (void)m;
    return P;
}

// Per-cell data from which the operator kernels evaluate the metric of the trilinear map
// (Sec. 2.7) at any point: the halved edge differences of the 8 corners along each reference
// axis and the cell's kappa, kGeoStride values per cell (layout in kernels.h).
std::vector<double> make_cell_geometry(int nx, int ny, int nz, const double *V, const double *kappa) {
    const int64_t ncell = (int64_t)nx * ny * nz;
    std::vector<double> out((size_t)ncell * kGeoStride, 0.0);
    auto vid = [&](int i, int j, int k) { return 3 * ((int64_t)i + (nx + 1) * ((int64_t)j + (ny + 1) * (int64_t)k)); };
    for (int64_t e = 0; e < ncell; ++e) {
        const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((int64_t)nx * ny));
        double X[2][2][2][3];
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a)
                    for (int d = 0; d < 3; ++d) X[c][b][a][d] = V[vid(i + a, j + b, k + c) + d];
        double *o = &out[(size_t)e * kGeoStride];
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v)
                for (int d = 0; d < 3; ++d) {
                    o[(u * 2 + v) * 3 + d] = 0.5 * (X[u][v][1][d] - X[u][v][0][d]);        // d/dxi: (c, b)
                    o[12 + (u * 2 + v) * 3 + d] = 0.5 * (X[u][1][v][d] - X[u][0][v][d]);   // d/deta: (c, a)
                    o[24 + (u * 2 + v) * 3 + d] = 0.5 * (X[1][u][v][d] - X[0][u][v][d]);   // d/dzeta: (b, a)
                }
        o[36] = kappa ? kappa[e] : 1.0;
    }
    return out;
}

// ============================================================ coarse space (Sec. 2.5)
// Q1 reference gradients at the q^3 quadrature points: gr[(pt * 8 + corner) * 3 + axis].
static std::vector<double> q1_gradients(const OneD &od) {
    const int q = od.q;
    const int64_t nq3 = (int64_t)q * q * q;
    std::vector<double> gr((size_t)nq3 * 8 * 3);
    for (int c = 0; c < q; ++c)
        for (int b = 0; b < q; ++b)
            for (int a = 0; a < q; ++a) {
                double xs[3] = {od.xq[a], od.xq[b], od.xq[c]};
                for (int cc = 0; cc < 2; ++cc)
                    for (int bb = 0; bb < 2; ++bb)
                        for (int aa = 0; aa < 2; ++aa) {
                            double N[3] = {aa ? 0.5 * (1 + xs[0]) : 0.5 * (1 - xs[0]), bb ? 0.5 * (1 + xs[1]) : 0.5 * (1 - xs[1]),
                                           cc ? 0.5 * (1 + xs[2]) : 0.5 * (1 - xs[2])};
                            double dN[3] = {aa ? 0.5 : -0.5, bb ? 0.5 : -0.5, cc ? 0.5 : -0.5};
                            int64_t pt = ((int64_t)c * q + b) * q + a;
                            int loc = (cc * 2 + bb) * 2 + aa;
                            gr[(pt * 8 + loc) * 3 + 0] = dN[0] * N[1] * N[2];
                            gr[(pt * 8 + loc) * 3 + 1] = N[0] * dN[1] * N[2];
                            gr[(pt * 8 + loc) * 3 + 2] = N[0] * N[1] * dN[2];
                        }
            }
    return gr;
}

// Q1 element matrix of cell e under the operator's quadrature (corners x fastest).
static void q1_element(const OneD &od, const Geometry &g, const std::vector<double> &gr, int64_t e, double K[8][8]) {
    const int q = od.q;
    const int64_t nq3 = (int64_t)q * q * q;
    for (int s = 0; s < 8; ++s)
        for (int t = 0; t < 8; ++t) K[s][t] = 0.0;
    for (int64_t pt = 0; pt < nq3; ++pt) {
        double G[3][3];
        if (!g.Gw.empty()) {
            const double *o = &g.Gw[(e * 6) * nq3 + pt];
            G[0][0] = o[0]; G[1][1] = o[nq3]; G[2][2] = o[2 * nq3];
            G[0][1] = G[1][0] = o[3 * nq3]; G[0][2] = G[2][0] = o[4 * nq3]; G[1][2] = G[2][1] = o[5 * nq3];
        } else {
            int a = (int)(pt % q), b = (int)((pt / q) % q), c = (int)(pt / ((int64_t)q * q));
            double w = od.wq[a] * od.wq[b] * od.wq[c];
            for (int r = 0; r < 3; ++r)
                for (int s2 = 0; s2 < 3; ++s2) G[r][s2] = r == s2 ? w * g.mu[e * 3 + r] : 0.0;
        }
        for (int s = 0; s < 8; ++s) {
            const double *gs = &gr[(pt * 8 + s) * 3];
            double Gg[3];
            for (int r = 0; r < 3; ++r) Gg[r] = G[r][0] * gs[0] + G[r][1] * gs[1] + G[r][2] * gs[2];
            for (int t = 0; t < 8; ++t) {
                const double *gt = &gr[(pt * 8 + t) * 3];
                K[t][s] += gt[0] * Gg[0] + gt[1] * Gg[1] + gt[2] * Gg[2];
            }
        }
    }
}

std::vector<double> make_coarse_inverse(int nx, int ny, int nz, const OneD &od, const Geometry &g) {
    int cx = nx - 1, cy = ny - 1, cz = nz - 1;
    int64_t nc = (int64_t)cx * cy * cz;
    if (nc == 0) return {};
    int64_t bw = (int64_t)cx * cy + cx + 1;   // half bandwidth in lexicographic order
    // banded lower storage: Ab[i][k] = A0(i, i - bw + k), k in [0, bw]
    std::vector<double> Ab((size_t)nc * (bw + 1), 0.0);
    auto add = [&](int64_t i, int64_t j, double v) {
        if (j > i || i - j > bw) return;
        Ab[(size_t)i * (bw + 1) + (j - i + bw)] += v;
    };
    const std::vector<double> gr = q1_gradients(od);
    int64_t ncell = (int64_t)nx * ny * nz;
    for (int64_t e = 0; e < ncell; ++e) {
        int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((int64_t)nx * ny));
        double K[8][8];
        q1_element(od, g, gr, e, K);
        int64_t id[8];
        for (int cc = 0; cc < 2; ++cc)
            for (int bb = 0; bb < 2; ++bb)
                for (int aa = 0; aa < 2; ++aa) {
                    int vx = i + aa, vy = j + bb, vz = k + cc;
                    bool inner = vx >= 1 && vx <= cx && vy >= 1 && vy <= cy && vz >= 1 && vz <= cz;
                    id[(cc * 2 + bb) * 2 + aa] = inner ? ((int64_t)(vx - 1) + cx * ((int64_t)(vy - 1) + cy * (int64_t)(vz - 1))) : -1;
                }
        for (int s = 0; s < 8; ++s)
            for (int t = 0; t < 8; ++t)
                if (id[s] >= 0 && id[t] >= 0) add(id[s], id[t], K[s][t]);
    }
    // banded Cholesky
    for (int64_t j = 0; j < nc; ++j) {
        double *rj = &Ab[(size_t)j * (bw + 1)];
        int64_t k0 = std::max<int64_t>(0, j - bw);
        double d = rj[bw];
        for (int64_t k = k0; k < j; ++k) d -= rj[k - j + bw] * rj[k - j + bw];
        if (!(d > 0)) throw Error(VSR_ENOTSPD, "coarse matrix is not positive definite");
        d = std::sqrt(d);
        rj[bw] = d;
        for (int64_t i = j + 1; i <= std::min(nc - 1, j + bw); ++i) {
            double *ri = &Ab[(size_t)i * (bw + 1)];
            int64_t kk0 = std::max<int64_t>(0, i - bw);
            double s = ri[j - i + bw];
            for (int64_t k = std::max(k0, kk0); k < j; ++k) s -= ri[k - i + bw] * rj[k - j + bw];
            ri[j - i + bw] = s / d;
        }
    }
    std::vector<double> inv((size_t)nc * nc);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t col = 0; col < nc; ++col) {
        std::vector<double> x(nc, 0.0);
        x[col] = 1.0;
        for (int64_t i = col; i < nc; ++i) {
            double s = x[i];
            for (int64_t k = std::max<int64_t>(col, i - bw); k < i; ++k) s -= Ab[(size_t)i * (bw + 1) + k - i + bw] * x[k];
            x[i] = s / Ab[(size_t)i * (bw + 1) + bw];
        }
        for (int64_t i = nc - 1; i >= 0; --i) {
            double s = x[i];
            for (int64_t k = i + 1; k <= std::min(nc - 1, i + bw); ++k) s -= Ab[(size_t)k * (bw + 1) + i - k + bw] * x[k];
            x[i] = s / Ab[(size_t)i * (bw + 1) + bw];
        }
        for (int64_t i = 0; i < nc; ++i) inv[(size_t)i * nc + col] = x[i];
    }
    return inv;
}

// ============================================================ Q1 geometric multigrid (Sec. 2.8)
// The p-coarse problem solved by geometric multigrid: level 0 is the Q1 Galerkin matrix of the
// mesh over its interior vertices, stored as a 27-point stencil per vertex; each next level
// merges 2 x 2 x 2 cells (while every axis has an even number of at least 4 cells) and is the
// Galerkin product P^T A P with the trilinear index-space interpolation P (fine vertex 2I takes
// coarse vertex I, fine vertex 2I +- 1 half of I and half of its neighbour; Dirichlet zeros on
// the boundary).
std::vector<double> q1_stencil(int nx, int ny, int nz, const OneD &od, const Geometry &g) {
    const int cx = nx - 1, cy = ny - 1, cz = nz - 1;
    const int64_t nv = (int64_t)cx * cy * cz;
    std::vector<double> st((size_t)27 * nv, 0.0);
    if (nv == 0) return st;
    const std::vector<double> gr = q1_gradients(od);
    const int64_t ncell = (int64_t)nx * ny * nz;
    for (int64_t e = 0; e < ncell; ++e) {
        const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((int64_t)nx * ny));
        double K[8][8];
        q1_element(od, g, gr, e, K);
        for (int s = 0; s < 8; ++s) {
            const int sx = i + (s & 1), sy = j + ((s >> 1) & 1), sz = k + (s >> 2);
            if (sx < 1 || sx > cx || sy < 1 || sy > cy || sz < 1 || sz > cz) continue;
            const int64_t row = (sx - 1) + (int64_t)cx * ((sy - 1) + (int64_t)cy * (sz - 1));
            for (int t = 0; t < 8; ++t) {
                const int tx = i + (t & 1), ty = j + ((t >> 1) & 1), tz = k + (t >> 2);
                if (tx < 1 || tx > cx || ty < 1 || ty > cy || tz < 1 || tz > cz) continue;
                const int sidx = (tz - sz + 1) * 9 + (ty - sy + 1) * 3 + (tx - sx + 1);
                st[(size_t)sidx * nv + row] += K[s][t];
            }
        }
    }
    return st;
}

static bool mg_coarsenable(int cx, int cy, int cz) {
    return cx % 2 == 0 && cy % 2 == 0 && cz % 2 == 0 && cx >= 4 && cy >= 4 && cz >= 4;
}

// A_c = P^T A_f P for the stencil A_f of a level with (cx, cy, cz) cells.
static MGLevelHost galerkin_coarsen(const MGLevelHost &f) {
    MGLevelHost c;
    c.cx = f.cx / 2; c.cy = f.cy / 2; c.cz = f.cz / 2;
    const int fx = f.cx - 1, fy = f.cy - 1, fz = f.cz - 1;          // fine interior extents
    const int ux = c.cx - 1, uy = c.cy - 1, uz = c.cz - 1;          // coarse interior extents
    const int64_t nvf = (int64_t)fx * fy * fz, nvc = (int64_t)ux * uy * uz;
    c.st.assign((size_t)27 * nvc, 0.0);
    // 1D interpolation weights of fine index i (1..f-1) from coarse J: J = i/2 (weight 1) for
    // even i, J = (i -+ 1)/2 (weights 1/2) for odd i; coarse boundary vertices are dropped
    auto parents = [](int i, int nc_cells, int J[2], double w[2]) {
        if (i % 2 == 0) {
            J[0] = i / 2; w[0] = 1.0; J[1] = -1; w[1] = 0.0;
        } else {
            J[0] = (i - 1) / 2; w[0] = 0.5; J[1] = (i + 1) / 2; w[1] = 0.5;
        }
        for (int t = 0; t < 2; ++t)
            if (J[t] < 1 || J[t] > nc_cells - 1) { J[t] = -1; w[t] = 0.0; }
    };
#pragma omp parallel for schedule(static)
    for (int64_t I = 0; I < nvc; ++I) {
        const int Ix = 1 + (int)(I % ux), Iy = 1 + (int)((I / ux) % uy), Iz = 1 + (int)(I / ((int64_t)ux * uy));
        double acc[27] = {0};
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    // fine vertex i in the support of coarse vertex I, with P[i, I]
                    const int ix = 2 * Ix + dx, iy = 2 * Iy + dy, iz = 2 * Iz + dz;
                    const double wi = (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0);
                    const int64_t row = (ix - 1) + (int64_t)fx * ((iy - 1) + (int64_t)fy * (iz - 1));
                    for (int ez = -1; ez <= 1; ++ez)
                        for (int ey = -1; ey <= 1; ++ey)
                            for (int ex = -1; ex <= 1; ++ex) {
                                const int jx = ix + ex, jy = iy + ey, jz = iz + ez;
                                if (jx < 1 || jx > fx || jy < 1 || jy > fy || jz < 1 || jz > fz) continue;
                                const double a = f.st[(size_t)((ez + 1) * 9 + (ey + 1) * 3 + (ex + 1)) * nvf + row];
                                if (a == 0.0) continue;
                                int Jx[2], Jy[2], Jz[2];
                                double wx[2], wy[2], wz[2];
                                parents(jx, c.cx, Jx, wx);
                                parents(jy, c.cy, Jy, wy);
                                parents(jz, c.cz, Jz, wz);
                                for (int a3 = 0; a3 < 2; ++a3)
                                    for (int a2 = 0; a2 < 2; ++a2)
                                        for (int a1 = 0; a1 < 2; ++a1) {
                                            if (Jx[a1] < 0 || Jy[a2] < 0 || Jz[a3] < 0) continue;
                                            const int sidx = (Jz[a3] - Iz + 1) * 9 + (Jy[a2] - Iy + 1) * 3 + (Jx[a1] - Ix + 1);
                                            acc[sidx] += wi * a * wx[a1] * wy[a2] * wz[a3];
                                        }
                            }
                }
        for (int s = 0; s < 27; ++s) c.st[(size_t)s * nvc + I] = acc[s];
    }
    return c;
}

// Dense inverse of a level's matrix from its stencil (dense Cholesky; small levels only).
static std::vector<double> stencil_inverse(const MGLevelHost &L) {
    const int ux = L.cx - 1, uy = L.cy - 1, uz = L.cz - 1;
    const int64_t n = (int64_t)ux * uy * uz;
    std::vector<double> A((size_t)n * n, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        const int x = (int)(i % ux), y = (int)((i / ux) % uy), z = (int)(i / ((int64_t)ux * uy));
        for (int s = 0; s < 27; ++s) {
            const int jx = x + s % 3 - 1, jy = y + (s / 3) % 3 - 1, jz = z + s / 9 - 1;
            if (jx < 0 || jx >= ux || jy < 0 || jy >= uy || jz < 0 || jz >= uz) continue;
            A[(size_t)i * n + jx + (int64_t)ux * (jy + (int64_t)uy * jz)] = L.st[(size_t)s * n + i];
        }
    }
    // symmetrize the rounding of the Galerkin products, then L L^T
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
    for (int64_t j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int64_t k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(d > 0)) throw Error(VSR_ENOTSPD, "coarsest multigrid matrix is not positive definite");
        d = std::sqrt(d);
        A[(size_t)j * n + j] = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double s = A[(size_t)i * n + j];
            for (int64_t k = 0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = s / d;
        }
    }
    std::vector<double> inv((size_t)n * n);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t col = 0; col < n; ++col) {
        std::vector<double> x(n, 0.0);
        x[col] = 1.0;
        for (int64_t i = col; i < n; ++i) {
            double s = x[i];
            for (int64_t k = col; k < i; ++k) s -= A[(size_t)i * n + k] * x[k];
            x[i] = s / A[(size_t)i * n + i];
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = x[i];
            for (int64_t k = i + 1; k < n; ++k) s -= A[(size_t)k * n + i] * x[k];
            x[i] = s / A[(size_t)i * n + i];
        }
        for (int64_t i = 0; i < n; ++i) inv[(size_t)i * n + col] = x[i];
    }
    return inv;
}

MGHierarchyHost make_mg_hierarchy(int nx, int ny, int nz, const OneD &od, const Geometry &g) {
    MGHierarchyHost H;
    MGLevelHost L0;
    L0.cx = nx; L0.cy = ny; L0.cz = nz;
    L0.st = q1_stencil(nx, ny, nz, od, g);
    H.levels.push_back(std::move(L0));
    while (mg_coarsenable(H.levels.back().cx, H.levels.back().cy, H.levels.back().cz))
        H.levels.push_back(galerkin_coarsen(H.levels.back()));
    // a single level is the direct solve: its inverse is the one of the dense coarse path
    H.coarsest_inverse = H.levels.size() == 1 ? make_coarse_inverse(nx, ny, nz, od, g) : stencil_inverse(H.levels.back());
    return H;
}

// ============================================================ lattice transfers
// Cell blocks of the FDM transfers T^T and T (Sec. 2.4: T maps FDM coefficients to GLL
// values; column b of the reference T holds the GLL values of FDM function b) and of the Q1
// transfers P^T and P (Sec. 2.5).  Free lattice positions along an axis are P = 1 .. p n - 1;
// cell e owns P = e p + 1 .. e p + p (its interior nodes and its high vertex), a = P - e p - 1.
std::vector<double> transfer_block(int kind, const OneD &od) {
    const int p = od.p, n1 = p + 1;
    auto Tm = [&](int i, int j) { return od.T[(size_t)i * n1 + j]; };
    std::vector<double> M;
    if (kind == XFER_FDM_RESTRICT) {
        // inputs P = e p + 1 + s, s < 2p - 1: this cell's interior, its high vertex, the next cell's interior
        const int K = 2 * p - 1;
        M.assign((size_t)p * K, 0.0);
        for (int a = 0; a < p - 1; ++a)
            for (int s = 0; s < p - 1; ++s) M[(size_t)a * K + s] = Tm(s + 1, a + 1);
        for (int s = 0; s < p - 1; ++s) M[(size_t)(p - 1) * K + s] = Tm(s + 1, p);
        M[(size_t)(p - 1) * K + p - 1] = 1.0;
        for (int s = p; s < K; ++s) M[(size_t)(p - 1) * K + s] = Tm(s - p + 1, 0);
    } else if (kind == XFER_FDM_PROLONG) {
        // inputs P = e p + s, s <= p: the cell's closure
        const int K = p + 1;
        M.assign((size_t)p * K, 0.0);
        for (int a = 0; a < p - 1; ++a)
            for (int s = 0; s < K; ++s) M[(size_t)a * K + s] = Tm(a + 1, s);
        M[(size_t)(p - 1) * K + p] = 1.0;
    } else if (kind == XFER_COARSE_RESTRICT) {
        // the coarse vertex e + 1 from the fine positions P = e p + 1 + s around it
        const int K = 2 * p - 1;
        M.assign((size_t)K, 0.0);
        for (int s = 0; s < p - 1; ++s) M[s] = 0.5 * (1 + od.xi[s + 1]);
        M[p - 1] = 1.0;
        for (int s = p; s < K; ++s) M[s] = 0.5 * (1 - od.xi[s - p + 1]);
    } else if (kind == XFER_COARSE_PROLONG) {
        // inputs: the coarse vertices e and e + 1
        M.assign((size_t)p * 2, 0.0);
        for (int a = 0; a < p - 1; ++a) {
            M[(size_t)a * 2] = 0.5 * (1 - od.xi[a + 1]);
            M[(size_t)a * 2 + 1] = 0.5 * (1 + od.xi[a + 1]);
        }
        M[(size_t)(p - 1) * 2 + 1] = 1.0;
    } else {
        throw Error(VSR_EINVAL, "unknown transfer kind");
    }
    return M;
}

// ============================================================ Sturm bisection
static int sturm_count(const std::vector<double> &d, const std::vector<double> &e, double x) {
    int cnt = 0;
    double q = 1.0;
    for (size_t i = 0; i < d.size(); ++i) {
        double off = i ? e[i - 1] * e[i - 1] : 0.0;
        q = d[i] - x - (i ? off / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0) ++cnt;
    }
    return cnt;
}

void tridiag_extremes(const std::vector<double> &d, const std::vector<double> &e, double &lmin, double &lmax) {
    int n = (int)d.size();
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < n; ++i) {
        double r = (i ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    auto kth = [&](int k) {  // k-th smallest (0-based)
        double a = lo, b = hi;
        for (int it = 0; it < 200 && b - a > 1e-15 * std::max(std::fabs(a), std::fabs(b)); ++it) {
            double c = 0.5 * (a + b);
            if (sturm_count(d, e, c) > k) b = c; else a = c;
        }
        return 0.5 * (a + b);
    };
    lmin = kth(0);
    lmax = kth(n - 1);
}


// ------------------------------------------------------------------ linear elasticity (Sec. 3.1)
std::vector<double> spd_inverse(int n, const std::vector<double> &A) {
    std::vector<double> L(A);
    if (!cholesky_lower(n, L.data(), n)) throw Error(VSR_ENOTSPD, "non-positive pivot in a dense Cholesky factor");
    std::vector<double> Si;
    inverse_from_cholesky(n, L.data(), n, Si);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) Si[(size_t)j * n + i] = Si[(size_t)i * n + j];
    return Si;
}

std::vector<double> elasticity_q1_matrix(const std::vector<double> &X, const std::vector<double> &Y,
                                         const std::vector<double> &Z, const OneD &od, double mu, double lam) {
    const int nx = (int)X.size() - 1, ny = (int)Y.size() - 1, nz = (int)Z.size() - 1;
    const int ux = nx - 1, uy = ny - 1, uz = nz - 1, nc = ux * uy * uz, N = 3 * nc;
    std::vector<double> A0((size_t)N * N, 0.0);
    if (nc == 0) return A0;
    // 1-D Q1 matrices on [-1, 1] with the operator's q-point rule: K = int N' N', M = int N N,
    // G[t][u] = int N_t' N_u (test function differentiated)
    double K1[2][2] = {}, M1[2][2] = {}, G1[2][2] = {};
    for (size_t k = 0; k < od.xq.size(); ++k) {
        const double x = od.xq[k], w = od.wq[k];
        const double Nv[2] = {0.5 * (1 - x), 0.5 * (1 + x)}, dN[2] = {-0.5, 0.5};
        for (int t = 0; t < 2; ++t)
            for (int u = 0; u < 2; ++u) {
                K1[t][u] += w * dN[t] * dN[u];
                M1[t][u] += w * Nv[t] * Nv[u];
                G1[t][u] += w * dN[t] * Nv[u];
            }
    }
    const double *coords[3] = {X.data(), Y.data(), Z.data()};
    for (int ez = 0; ez < nz; ++ez)
        for (int ey = 0; ey < ny; ++ey)
            for (int ex = 0; ex < nx; ++ex) {
                const int e3[3] = {ex, ey, ez};
                double h[3];
                for (int a = 0; a < 3; ++a) h[a] = coords[a][e3[a] + 1] - coords[a][e3[a]];
                const double vol = h[0] * h[1] * h[2] / 8.0;
                // I_ij(a, b) = int d_i phi_a d_j phi_b: per axis K (i = j = axis), G (test
                // derivative), G^T (trial derivative) or M
                auto Iij = [&](int i, int j, const int ta[3], const int tb[3]) {
                    double v = vol;
                    for (int ax = 0; ax < 3; ++ax) {
                        const int t = ta[ax], u = tb[ax];
                        if (ax == i && ax == j) v *= K1[t][u] * (2 / h[ax]) * (2 / h[ax]);
                        else if (ax == i) v *= G1[t][u] * (2 / h[ax]);
                        else if (ax == j) v *= G1[u][t] * (2 / h[ax]);
                        else v *= M1[t][u];
                    }
                    return v;
                };
                for (int a = 0; a < 8; ++a)
                    for (int b = 0; b < 8; ++b) {
                        const int ta[3] = {a & 1, (a >> 1) & 1, a >> 2}, tb[3] = {b & 1, (b >> 1) & 1, b >> 2};
                        const int va[3] = {ex + ta[0], ey + ta[1], ez + ta[2]}, vb[3] = {ex + tb[0], ey + tb[1], ez + tb[2]};
                        bool inner = true;
                        for (int ax = 0; ax < 3; ++ax) {
                            const int nn = ax == 0 ? nx : (ax == 1 ? ny : nz);
                            inner = inner && va[ax] >= 1 && va[ax] <= nn - 1 && vb[ax] >= 1 && vb[ax] <= nn - 1;
                        }
                        if (!inner) continue;
                        const int ia = ((va[2] - 1) * uy + (va[1] - 1)) * ux + (va[0] - 1);
                        const int ib = ((vb[2] - 1) * uy + (vb[1] - 1)) * ux + (vb[0] - 1);
                        const double lap = Iij(0, 0, ta, tb) + Iij(1, 1, ta, tb) + Iij(2, 2, ta, tb);
                        for (int c = 0; c < 3; ++c)
                            for (int e = 0; e < 3; ++e) {
                                // mu (delta_ce grad.grad + d_e phi_a d_c phi_b) + lam d_c phi_a d_e phi_b
                                double v = mu * Iij(e, c, ta, tb) + lam * Iij(c, e, ta, tb);
                                if (c == e) v += mu * lap;
                                A0[(size_t)(c * nc + ia) * N + e * nc + ib] += v;
                            }
                    }
            }
    return A0;
}
}  // namespace vsr
