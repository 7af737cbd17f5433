// Internal declarations shared by the host setup, the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/vsr.h"

namespace vsr {

// Error carrying a vsr_status across internal C++ code; the C ABI converts it.
struct Error : std::runtime_error {
    vsr_status status;
    Error(vsr_status s, const std::string &msg) : std::runtime_error(msg), status(s) {}
};

#define VSR_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            throw ::vsr::Error(VSR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ 1D data (host, FP64)
struct OneD {
    int p = 0, q = 0;
    std::vector<double> xi, xq, wq;   // GLL nodes (p+1), quadrature points/weights (q)
    std::vector<double> Iq, Dq;       // q x (p+1) row-major: l_j(x_a), l_j'(x_a)
    std::vector<double> A, B;         // (p+1)^2 row-major reference stiffness / mass
    std::vector<double> lam;          // p-1 interior eigenvalues, ascending
    std::vector<double> T;            // (p+1)^2 row-major: GLL coefficients of the FDM basis (columns)
    std::vector<double> Af, Bf;       // (p+1)^2 FDM-basis matrices with structural zeros imposed
};
OneD make_1d(int p, int q);

// ------------------------------------------------------------------ geometry (host, FP64)
struct Geometry {
    bool cartesian = false;
    std::vector<double> mu;     // ncell * 3 surrogate scalings (or the Cartesian closed form)
    std::vector<double> Gw;     // ncell * 6 * q^3 (xx, yy, zz, xy, xz, yz), w_q folded in; empty if cartesian
    std::vector<double> wdet;   // ncell * q^3 : w_q |det DF|
};
Geometry make_geometry(int nx, int ny, int nz, const double *vertices, const double *kappa,
                       const OneD &od, bool keep_metric);
// Halved corner edge differences and kappa per cell, for the operator's on-the-fly metric.
std::vector<double> make_cell_geometry(int nx, int ny, int nz, const double *vertices, const double *kappa);

// ------------------------------------------------------------------ patches
// Box coordinates of a patch run over [0, 2m] per axis (m = p-1); the star's
// central plane is at m.  Axis kinds: FULL (interior vertex), LOW (vertex at 0:
// valid positions m+1..2m), HIGH (vertex at N: valid positions 0..m-1).
enum AxisKind : int { AX_FULL = 0, AX_LOW = 1, AX_HIGH = 2 };

// Layout of the interior-vertex patch factor (all interior patches share it).
struct InteriorLayout {
    int m = 0, w = 0;           // w = 2m+1
    int n_leaf = 0, n_sep = 0, n_top = 0, n_iface = 0;
    int top_pad = 0;            // top-plane size padded to a multiple of 4
    int64_t off_invd = 0, off_B1 = 0, off_B2 = 0, off_Lsep = 0, off_Sy = 0, off_Ltop = 0;
    int ntiles = 0;
    std::vector<int64_t> tile_off;   // offset of tile J (diag block 64x64 then panel below)
    std::vector<int> tile_rows_pad;  // padded row count of the panel below tile J
    int64_t stride = 0;              // entries per patch (multiple of 64)
};
InteriorLayout interior_layout(int p);

struct PatchSet {
    // interior class
    InteriorLayout L;
    std::vector<int32_t> interior_vertices;   // 3 ints per patch (vx, vy, vz)
    std::vector<int32_t> interior_factor_of;  // per interior patch: index of its factor
    int64_t n_interior_factors = 0;
    // boundary classes: per patch vx,vy,vz, kind(x,y,z), nslices, slice size, factor offset
    std::vector<int32_t> boundary_desc;       // 8 ints per patch
    std::vector<int64_t> boundary_off;        // factor offset per boundary patch
    int64_t boundary_entries = 0;
    // factors (FP64 on the host; converted to the device precision on upload)
    std::vector<double> interior_factor;      // n_interior_factors * L.stride
    std::vector<double> boundary_factor;
};
// share: stars with the same class and bit-identical cell scalings (every interior star of a
// uniform Cartesian mesh with constant kappa) are factored once and share the factor.
PatchSet make_patches(int nx, int ny, int nz, const OneD &od, const double *mu, bool interior_only, bool share = false);

// ------------------------------------------------------------------ coarse space
// Dense inverse of the Q1 Galerkin matrix over interior vertices (row-major, nc x nc).
std::vector<double> make_coarse_inverse(int nx, int ny, int nz, const OneD &od, const Geometry &g);

// ------------------------------------------------------------------ Q1 geometric multigrid
// Levels of the p-coarse (Q1) problem (Sec. 2.8): level 0 is the Q1 Galerkin matrix of the mesh
// over its interior vertices; each next level merges 2 x 2 x 2 cells while every axis has an
// even number of at least 4 cells, and is the Galerkin product P^T A P with trilinear
// index-space interpolation.  Stencils hold 27 coefficients per interior vertex, stored
// [s][vertex] with s = (dz+1) 9 + (dy+1) 3 + (dx+1) and vertices x fastest.
struct MGLevelHost {
    int cx = 0, cy = 0, cz = 0;   // cells per axis; (cx-1)(cy-1)(cz-1) interior vertices
    std::vector<double> st;       // 27 x nv
};
struct MGHierarchyHost {
    std::vector<MGLevelHost> levels;
    std::vector<double> coarsest_inverse;   // dense inverse of the last level, row-major
};
std::vector<double> q1_stencil(int nx, int ny, int nz, const OneD &od, const Geometry &g);
MGHierarchyHost make_mg_hierarchy(int nx, int ny, int nz, const OneD &od, const Geometry &g);

// Cell block of a lattice transfer (row-major OA x K) for launch_transfer: along an axis,
// cell e maps inputs e*in_step + in_off + s to outputs e*out_step + a.
//   XFER_FDM_RESTRICT   T^T: OA = p, K = 2p-1 (in_step p, in_off 0, out_step p)
//   XFER_FDM_PROLONG    T:   OA = p, K = p+1  (p, -1, p)
//   XFER_COARSE_RESTRICT P^T: OA = 1, K = 2p-1 (p, 0, 1)
//   XFER_COARSE_PROLONG P:   OA = p, K = 2    (1, -1, p)
enum { XFER_FDM_RESTRICT = 0, XFER_FDM_PROLONG = 1, XFER_COARSE_RESTRICT = 2, XFER_COARSE_PROLONG = 3 };
std::vector<double> transfer_block(int kind, const OneD &od);

// Device address (on the current device) of the library's static workspace, for callers
// that cannot allocate; VSR_EINVAL if `bytes` exceeds its size (static_workspace_bytes()).
void *static_workspace(size_t bytes);
size_t static_workspace_bytes();

// Symmetric tridiagonal extreme eigenvalues by Sturm bisection.
void tridiag_extremes(const std::vector<double> &d, const std::vector<double> &e, double &lmin, double &lmax);

// Linear elasticity (Sec. 3.1): the inverse of a dense SPD matrix (row-major, symmetric
// output; throws on a non-positive pivot), and the Q1 Galerkin matrix of a(v, u) = int 2 mu
// eps(v):eps(u) + lam div v div u on the tensor grid of box cells with vertex coordinates X, Y,
// Z (one per axis), over the interior vertices, rows [component][vertex] (x fastest), the
// 1-D integrals taken with od's quadrature.
std::vector<double> spd_inverse(int n, const std::vector<double> &A);
std::vector<double> elasticity_q1_matrix(const std::vector<double> &X, const std::vector<double> &Y,
                                         const std::vector<double> &Z, const OneD &od, double mu, double lam);

}  // namespace vsr
