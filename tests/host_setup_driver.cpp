// Host-only driver of the solver's setup code (1D data, geometry, patch factors, coarse
// inverse, multigrid hierarchy, transfer blocks, tridiagonal eigenvalue bounds), built with g++ and the address
// and undefined-behaviour sanitizers by tests/test_host_sanitizers.py.  It checks that the
// host setup reads and writes only inside its buffers on small meshes of every patch class.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2107_14758_amd/csrc/vsr_internal.h"

using namespace vsr;

static std::vector<double> cube(int nx, int ny, int nz, double jitter, unsigned seed) {
    std::vector<double> v(3 * (size_t)(nx + 1) * (ny + 1) * (nz + 1));
    unsigned s = seed;
    auto uni = [&]() { s = s * 1664525u + 1013904223u; return ((s >> 8) / 16777216.0) * 2.0 - 1.0; };
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double *c = &v[3 * (i + (size_t)(nx + 1) * (j + (size_t)(ny + 1) * k))];
                c[0] = (double)i / nx; c[1] = (double)j / ny; c[2] = (double)k / nz;
                const bool interior = i > 0 && i < nx && j > 0 && j < ny && k > 0 && k < nz;
                if (interior) {
                    c[0] += jitter * uni() / nx; c[1] += jitter * uni() / ny; c[2] += jitter * uni() / nz;
                }
            }
    return v;
}

int main() {
    struct Case { int nx, ny, nz, p; double jitter; bool interior_only, share; };
    const Case cases[] = {{2, 2, 2, 2, 0.0, false, false}, {3, 2, 4, 3, 0.15, false, false},
                          {2, 3, 2, 5, 0.2, true, false},  {3, 3, 3, 4, 0.0, false, true},
                          {2, 2, 3, 7, 0.15, false, false}, {8, 4, 4, 2, 0.15, false, false},
                          {8, 8, 8, 2, 0.0, false, true}};
    for (const Case &c : cases) {
        const int q = (3 * (c.p + 1) + 1) / 2;
        OneD od = make_1d(c.p, q);
        std::vector<double> V = cube(c.nx, c.ny, c.nz, c.jitter, 7u + c.p);
        std::vector<double> kappa((size_t)c.nx * c.ny * c.nz);
        for (size_t e = 0; e < kappa.size(); ++e) kappa[e] = 1.0 + 0.5 * std::sin(1.0 + e);
        Geometry g = make_geometry(c.nx, c.ny, c.nz, V.data(), kappa.data(), od, true);
        double sum = 0;
        PatchSet S = make_patches(c.nx, c.ny, c.nz, od, g.mu.data(), c.interior_only, c.share);
        std::vector<double> A0 = make_coarse_inverse(c.nx, c.ny, c.nz, od, g);
        MGHierarchyHost H = make_mg_hierarchy(c.nx, c.ny, c.nz, od, g);
        for (double x : H.coarsest_inverse) sum += 1e-6 * x;
        for (int k = 0; k < 4; ++k)
            for (double x : transfer_block(k, od)) sum += x;
        std::vector<double> d(od.lam.begin(), od.lam.end()), e(d.size() > 0 ? d.size() - 1 : 0, 0.1);
        double lmin = 0, lmax = 0;
        if (!d.empty()) tridiag_extremes(d, e, lmin, lmax);
        std::printf("case %dx%dx%d p=%d: %zu interior + %zu boundary stars, %zu factor entries, coarse %zu, "
                    "%zu multigrid levels, lambda [%.3f, %.3f], check %.6f\n",
                    c.nx, c.ny, c.nz, c.p, S.interior_vertices.size() / 3, S.boundary_off.size(),
                    S.interior_factor.size() + S.boundary_factor.size(), A0.size(), H.levels.size(), lmin, lmax, sum);
        if (!std::isfinite(sum) || !std::isfinite(lmin) || !std::isfinite(lmax)) return 1;
    }
    std::printf("host setup ok\n");
    return 0;
}
