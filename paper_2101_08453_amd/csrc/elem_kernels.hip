// Element-level kernels of the finite element formulation (Sec. 2 of Mandel
// et al.): geometry check, stiffness stencil assembly, the matrix-free
// element-by-element stiffness apply with 2x2x2 Gauss quadrature, the
// one-point right-hand side -int grad(mu).u0, the weak divergence check,
// the centre-gradient recovery u = u0 + A^-1 grad(lambda), and the adjoints
// of the recovery and of the right-hand side.
//
// Element geometry without forming shape-function gradients: on the reference
// cube the trilinear map has d x / d xi_1 = 1/2 * bilinear interpolation, in
// (xi_2, xi_3), of the four x-directed edge vectors x_{1bc} - x_{0bc} (and
// likewise for xi_2, xi_3).  At the 2x2x2 Gauss points each Jacobian column
// therefore takes only four distinct values.  With the Jacobian columns c_m,
// the rows of J^{-1} are r_m / det J with r_0 = c_1 x c_2, r_1 = c_2 x c_0,
// r_2 = c_0 x c_1, det J = c_0 . r_0.  For a nodal field v with reference
// gradient g = grad_xi v, the physical gradient is (sum_m g_m r_m) / det J.
//
// Local node a = ax + 2 ay + 4 az sits at reference corner (2ax-1, 2ay-1, 2az-1).
#include <algorithm>

#include "mcw_internal.hpp"

namespace mcw {
namespace {

constexpr double GQ = 0.57735026918962576451;  // Gauss abscissa 1/sqrt(3)
constexpr double WP = 0.5 * (1.0 + GQ);        // 1D linear shape value at the near Gauss point
constexpr double WM = 0.5 * (1.0 - GQ);        // ... at the far Gauss point

// Bilinear interpolation of four corner values v[b + 2c] (b, c in {0,1}) to
// the four Gauss points (s1, s2): out[s1 + 2 s2] = sum w(b,s1) w(c,s2) v[b+2c],
// w(b,s) = WP if b == s else WM.  The weight matrix is symmetric, so the same
// routine is its own transpose (used to spread Gauss-point values to edges).
__device__ __forceinline__ void bil4(const double v[4], double out[4]) {
  const double t00 = WP * v[0] + WM * v[1];
  const double t10 = WM * v[0] + WP * v[1];
  const double t01 = WP * v[2] + WM * v[3];
  const double t11 = WM * v[2] + WP * v[3];
  out[0] = WP * t00 + WM * t01;
  out[1] = WP * t10 + WM * t11;
  out[2] = WM * t00 + WP * t01;
  out[3] = WM * t10 + WP * t11;
}

// Differences of a nodal scalar along the edges of direction m, indexed by
// the pair of the other two local coordinates (in increasing axis order).
__device__ __forceinline__ void edge_diffs(const double v[8], double e[3][4]) {
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int b = p & 1, c = p >> 1;
    e[0][p] = v[1 + 2 * b + 4 * c] - v[0 + 2 * b + 4 * c];  // pair (ay, az)
    e[1][p] = v[b + 2 + 4 * c] - v[b + 4 * c];              // pair (ax, az)
    e[2][p] = v[b + 2 * c + 4] - v[b + 2 * c];              // pair (ax, ay)
  }
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Jacobian columns at the Gauss points: Jg[m][d][pair] for column m,
// coordinate d, pair index of the two other Gauss coordinates.
__device__ __forceinline__ void gauss_jacobian(const double xe[3][8], double Jg[3][3][4]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double e[3][4];
    edge_diffs(xe[d], e);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      double o[4];
      bil4(e[m], o);
#pragma unroll
      for (int p = 0; p < 4; ++p) Jg[m][d][p] = 0.5 * o[p];
    }
  }
}

// Jacobian columns at the element centre: c[m][d] = 1/8 sum of the 4 edges.
__device__ __forceinline__ void centre_jacobian(const double xe[3][8], double c[3][3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double e[3][4];
    edge_diffs(xe[d], e);
#pragma unroll
    for (int m = 0; m < 3; ++m) c[m][d] = 0.125 * (e[m][0] + e[m][1] + e[m][2] + e[m][3]);
  }
}

// Reference gradient of a nodal scalar at the centre.
__device__ __forceinline__ void centre_ref_grad(const double v[8], double g[3]) {
  double e[3][4];
  edge_diffs(v, e);
#pragma unroll
  for (int m = 0; m < 3; ++m) g[m] = 0.125 * (e[m][0] + e[m][1] + e[m][2] + e[m][3]);
}

// Rows r_m of the adjugate and det J from Jacobian columns.
__device__ __forceinline__ double adjugate(const double c0[3], const double c1[3], const double c2[3],
                                           double r[3][3]) {
  cross3(c1, c2, r[0]);
  cross3(c2, c0, r[1]);
  cross3(c0, c1, r[2]);
  return dot3(c0, r[0]);
}

// Gauss point (sx, sy, sz): pair indices of the three Jacobian columns.
#define GP_PAIRS(sx, sy, sz) const int p0 = (sy) + 2 * (sz), p1 = (sx) + 2 * (sz), p2 = (sx) + 2 * (sy)

// y += K_e v for one element (2x2x2 Gauss, coefficient diag(c)).
__device__ __forceinline__ void element_apply(const double Jg[3][3][4], const double v[8],
                                              const double c[3], double y[8]) {
  double ev[3][4], G[3][4];
  edge_diffs(v, ev);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    bil4(ev[m], G[m]);
#pragma unroll
    for (int p = 0; p < 4; ++p) G[m][p] *= 0.5;
  }
  double Acc[3][4] = {};
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    const int sx = g & 1, sy = (g >> 1) & 1, sz = g >> 2;
    GP_PAIRS(sx, sy, sz);
    const double c0[3] = {Jg[0][0][p0], Jg[0][1][p0], Jg[0][2][p0]};
    const double c1[3] = {Jg[1][0][p1], Jg[1][1][p1], Jg[1][2][p1]};
    const double c2[3] = {Jg[2][0][p2], Jg[2][1][p2], Jg[2][2][p2]};
    double r[3][3];
    const double det = adjugate(c0, c1, c2, r);
    const double g0 = G[0][p0], g1 = G[1][p1], g2 = G[2][p2];
    double q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) q[d] = c[d] * (g0 * r[0][d] + g1 * r[1][d] + g2 * r[2][d]);
    const double idet = 1.0 / det;
    Acc[0][p0] += dot3(r[0], q) * idet;
    Acc[1][p1] += dot3(r[1], q) * idet;
    Acc[2][p2] += dot3(r[2], q) * idet;
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double B[4];
    bil4(Acc[m], B);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const double t = 0.5 * B[p];
      const int b = p & 1, cc = p >> 1;
      if (m == 0) { y[1 + 2 * b + 4 * cc] += t; y[0 + 2 * b + 4 * cc] -= t; }
      if (m == 1) { y[b + 2 + 4 * cc] += t; y[b + 4 * cc] -= t; }
      if (m == 2) { y[b + 2 * cc + 4] += t; y[b + 2 * cc] -= t; }
    }
  }
}

// 1/x from the hardware reciprocal estimate refined by two Newton steps
// (e = 1 - x r, r += r e), within an ulp or two of the rounded quotient; for
// the moderate, positive det J of valid elements.
__device__ __forceinline__ double inv_newton(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Jacobian columns at the Gauss points times 2 (the 1/2 of gauss_jacobian left
// out): J2[m][d][pair] = 2 dx_d/dxi_m.
__device__ __forceinline__ void gauss_jacobian2(const double xe[3][8], double J2[3][3][4]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double e[3][4];
    edge_diffs(xe[d], e);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      double o[4];
      bil4(e[m], o);
#pragma unroll
      for (int p = 0; p < 4; ++p) J2[m][d][p] = o[p];
    }
  }
}

// element_apply with J2 = 2J and the reference gradients at the Gauss points
// also left doubled: the adjugate rows of J2 are 4r, det J2 = 8 det J, so each
// Gauss point adds 2 * 4 * 4 / 8 = 4 times its term to the accumulators, and the
// spread back to the nodes takes 1/8 instead of 1/2.  The 1/det comes from
// inv_newton.  Used by the per-solve kernels (apply, residual, divergence).
__device__ __forceinline__ void element_apply2(const double J2[3][3][4], const double v[8],
                                               const double c[3], double y[8]) {
  double ev[3][4], G[3][4];
  edge_diffs(v, ev);
#pragma unroll
  for (int m = 0; m < 3; ++m) bil4(ev[m], G[m]);
  double Acc[3][4] = {};
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    const int sx = g & 1, sy = (g >> 1) & 1, sz = g >> 2;
    GP_PAIRS(sx, sy, sz);
    const double c0[3] = {J2[0][0][p0], J2[0][1][p0], J2[0][2][p0]};
    const double c1[3] = {J2[1][0][p1], J2[1][1][p1], J2[1][2][p1]};
    const double c2[3] = {J2[2][0][p2], J2[2][1][p2], J2[2][2][p2]};
    double r[3][3];
    const double idet = inv_newton(adjugate(c0, c1, c2, r));
    const double g0 = G[0][p0], g1 = G[1][p1], g2 = G[2][p2];
    double q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) q[d] = c[d] * idet * (g0 * r[0][d] + g1 * r[1][d] + g2 * r[2][d]);
    Acc[0][p0] += dot3(r[0], q);
    Acc[1][p1] += dot3(r[1], q);
    Acc[2][p2] += dot3(r[2], q);
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double B[4];
    bil4(Acc[m], B);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const double t = 0.125 * B[p];
      const int b = p & 1, cc = p >> 1;
      if (m == 0) { y[1 + 2 * b + 4 * cc] += t; y[0 + 2 * b + 4 * cc] -= t; }
      if (m == 1) { y[b + 2 + 4 * cc] += t; y[b + 4 * cc] -= t; }
      if (m == 2) { y[b + 2 * cc + 4] += t; y[b + 2 * cc] -= t; }
    }
  }
}

// K_e v on a terrain-following element: the x of a node depends on i only and
// its y on j only (columns of a structured horizontal grid), so over the
// element dx/dxi = hx/2, dy/deta = hy/2 and only z varies.  With the Jacobian
// columns (hx/2, 0, zx), (0, hy/2, zy), (0, 0, zz) at a Gauss point, det J =
// hx hy zz / 4; the physical gradient w from the reference gradient g is
// w2 = g2/zz, w0 = (g0 - zx w2)/(hx/2), w1 = (g1 - zy w2)/(hy/2); the flux is
// q = c w; and det J times J^-1 q, which the Gauss point adds to the three
// reference directions, is (hy zz q0, hx zz q1, hx hy q2 - hy zx q0 - hx zy q1)/4.
// Zg and G hold the z derivatives and the reference gradients doubled (bil4 of
// the edge differences without the 1/2), whose ratios are the same; the
// accumulators therefore hold 4 times the terms, like element_apply2's, and
// the spread to the nodes takes 1/8.
__device__ __forceinline__ void element_apply_tf(const double Zg[3][4], double hx, double hy,
                                                 double ihx2, double ihy2, const double v[8],
                                                 const double c[3], double y[8]) {
  double ev[3][4], G[3][4];
  edge_diffs(v, ev);
#pragma unroll
  for (int m = 0; m < 3; ++m) bil4(ev[m], G[m]);
  const double hxy = hx * hy;
  double Acc[3][4] = {};
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    const int sx = g & 1, sy = (g >> 1) & 1, sz = g >> 2;
    GP_PAIRS(sx, sy, sz);
    const double zx = Zg[0][p0], zy = Zg[1][p1], zz = Zg[2][p2];
    const double w2 = G[2][p2] * inv_newton(zz);
    const double q0 = c[0] * (G[0][p0] - zx * w2) * ihx2;  // ihx2 = 1/hx, G and zx doubled
    const double q1 = c[1] * (G[1][p1] - zy * w2) * ihy2;
    const double q2 = c[2] * w2;
    const double t0 = hy * q0, t1 = hx * q1;
    Acc[0][p0] += t0 * zz;
    Acc[1][p1] += t1 * zz;
    Acc[2][p2] += hxy * q2 - zx * t0 - zy * t1;
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double B[4];
    bil4(Acc[m], B);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const double t = 0.125 * B[p];
      const int b = p & 1, cc = p >> 1;
      if (m == 0) { y[1 + 2 * b + 4 * cc] += t; y[0 + 2 * b + 4 * cc] -= t; }
      if (m == 1) { y[b + 2 + 4 * cc] += t; y[b + 4 * cc] -= t; }
      if (m == 2) { y[b + 2 * cc + 4] += t; y[b + 2 * cc] -= t; }
    }
  }
}

// Spread a reference-space vector w (one value per direction, at the centre)
// to the nodes: y_a += s * sum_m sign_m(a) w_m.
__device__ __forceinline__ void spread_centre(const double w[3], double s, double y[8]) {
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const double sx = (a & 1) ? 1.0 : -1.0, sy = (a & 2) ? 1.0 : -1.0, sz = (a & 4) ? 1.0 : -1.0;
    y[a] += s * (sx * w[0] + sy * w[1] + sz * w[2]);
  }
}

// f_e: -8 detJ(0) B(0)^T u0 = -sum_m sign_m(a) (r_m . u0).
__device__ __forceinline__ void element_rhs(const double xe[3][8], const double u0[3], double y[8]) {
  double cj[3][3], r[3][3];
  centre_jacobian(xe, cj);
  (void)adjugate(cj[0], cj[1], cj[2], r);
  const double w[3] = {dot3(r[0], u0), dot3(r[1], u0), dot3(r[2], u0)};
  spread_centre(w, -1.0, y);
}

// g_lambda contribution G_1^T diag(c) g: sum_m sign_m(a)/8 (r_m . diag(c) g) / det.
__device__ __forceinline__ void element_recover_adjoint(const double xe[3][8], const double g[3],
                                                        const double c[3], double y[8]) {
  double cj[3][3], r[3][3];
  centre_jacobian(xe, cj);
  const double det = adjugate(cj[0], cj[1], cj[2], r);
  const double cg[3] = {c[0] * g[0], c[1] * g[1], c[2] * g[2]};
  const double w[3] = {dot3(r[0], cg), dot3(r[1], cg), dot3(r[2], cg)};
  spread_centre(w, 0.125 / det, y);
}

__device__ __forceinline__ size_t node_id(int i, int j, int k, int NX, int NY) {
  return (size_t)i + (size_t)NX * ((size_t)j + (size_t)NY * (size_t)k);
}

// ---------------------------------------------------------------- geometry check

__global__ __launch_bounds__(256) void geometry_check_kernel(const double* __restrict__ X,
                                                             const double* __restrict__ Y,
                                                             const double* __restrict__ Z, int nx,
                                                             int ny, int nz,
                                                             unsigned long long* first_bad) {
  const long long E = (long long)nx * ny * nz;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((long long)nx * ny));
  const int NX = nx + 1, NY = ny + 1;
  double xe[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const size_t n = node_id(i + (a & 1), j + ((a >> 1) & 1), k + (a >> 2), NX, NY);
    xe[0][a] = X[n];
    xe[1][a] = Y[n];
    xe[2][a] = Z[n];
  }
  double Jg[3][3][4];
  gauss_jacobian(xe, Jg);
  bool ok = true;
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    GP_PAIRS(g & 1, (g >> 1) & 1, g >> 2);
    const double c0[3] = {Jg[0][0][p0], Jg[0][1][p0], Jg[0][2][p0]};
    const double c1[3] = {Jg[1][0][p1], Jg[1][1][p1], Jg[1][2][p1]};
    const double c2[3] = {Jg[2][0][p2], Jg[2][1][p2], Jg[2][2][p2]};
    double r[3][3];
    const double det = adjugate(c0, c1, c2, r);
    ok = ok && (det > 0.0);
  }
  double cj[3][3], r[3][3];
  centre_jacobian(xe, cj);
  const double det0 = adjugate(cj[0], cj[1], cj[2], r);
  ok = ok && (det0 > 0.0);
  if (!ok) atomicMin(first_bad, (unsigned long long)e);
}

// ---------------------------------------------------------------- stencil assembly

// One colour class of elements (parity of i, j, k): elements of a class share
// no node, so each adds its 8x8 matrix into the node stencils without races.
__global__ __launch_bounds__(256) void assemble_kernel(const double* __restrict__ X,
                                                       const double* __restrict__ Y,
                                                       const double* __restrict__ Z, int nx, int ny,
                                                       int nz, double c0, double c1, double c2,
                                                       int pi, int pj, int pk,
                                                       double* __restrict__ st) {
  const int mx = (nx - pi + 1) / 2, my = (ny - pj + 1) / 2, mz = (nz - pk + 1) / 2;
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long long)mx * my * mz) return;
  const int i = 2 * (int)(tid % mx) + pi;
  const int j = 2 * (int)((tid / mx) % my) + pj;
  const int k = 2 * (int)(tid / ((long long)mx * my)) + pk;
  const int NX = nx + 1, NY = ny + 1;
  const StLayout L = Dims{nx, ny, nz}.layout();
  double xe[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const size_t n = node_id(i + (a & 1), j + ((a >> 1) & 1), k + (a >> 2), NX, NY);
    xe[0][a] = X[n];
    xe[1][a] = Y[n];
    xe[2][a] = Z[n];
  }
  double Jg[3][3][4];
  gauss_jacobian(xe, Jg);
  const double c[3] = {c0, c1, c2};
  // column b of K_e is K_e applied to the b-th unit vector
#pragma unroll 1
  for (int b = 0; b < 8; ++b) {
    double v[8], y[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      v[a] = (a == b) ? 1.0 : 0.0;
      y[a] = 0.0;
    }
    element_apply(Jg, v, c, y);
    const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
      const int o = (bx - ax + 1) + 3 * (by - ay + 1) + 9 * (bz - az + 1);
      const size_t idx = st_entry<double>(L.node(i + ax, j + ay, k + az), o);
      st[idx] += y[a];
    }
  }
}

// ---------------------------------------------------------------- element tiles

constexpr int TE = 16;       // element columns per tile side
constexpr int TN = TE - 1;   // owned node columns per tile side
constexpr int PN = TE + 1;   // node columns per tile side that the elements touch
constexpr int PP = PN * PN;  // nodes of one tile plane

// Element loop with deterministic per-node accumulation.  A block owns a
// TN x TN patch of node columns and evaluates the TE x TE element columns
// touching it (one element column per thread), marching up the layers.
//
// The PN x PN node values of a tile plane (coordinates, and the nodal field
// where the mode has one) are staged in LDS, so each node is read from memory
// once per block instead of by every element around it; the loads of plane
// k + 2 are issued before the elements of layer k are evaluated and stored
// after them, so their latency hides behind that work.  Each element leaves
// its 4 lower and 4 upper corner contributions in LDS; the owner of a node sums,
// in a fixed order, the lower contributions of the current layer, and keeps the
// sum of the upper ones for the next plane.
//
// TF (terrain-following grid: x of a node depends on i only, y on j only):
// only z and the nodal field are staged per plane, each element column takes
// its x, y extent once, and the Gauss-point work is element_apply_tf's.
// LDS of one block, in doubles: two staged planes, the lower and upper corner
// contributions per channel, and the reduction slots.
constexpr int tile_lds_doubles(int mode, bool tf) {
  const bool nodev = mode == M_APPLY || mode == M_RESID || mode == M_DIV;
  const int na = (tf ? 1 : 3) + (nodev ? 1 : 0), ch = mode == M_DIV ? 2 : 1;
  return 2 * na * PP + 2 * ch * 4 * 256 + 256;
}
constexpr int tile_lds_max(int mode) {
  return tile_lds_doubles(mode, false) > tile_lds_doubles(mode, true) ? tile_lds_doubles(mode, false)
                                                                      : tile_lds_doubles(mode, true);
}

template <int MODE, bool TF>
__device__ __forceinline__ void elem_tile_body(const TileJob& A, int bx, int by, double* smem) {
  constexpr int CH = (MODE == M_DIV) ? 2 : 1;
  constexpr bool NODEV = (MODE == M_APPLY || MODE == M_RESID || MODE == M_DIV);
  constexpr bool ELEMV = (MODE == M_RHS || MODE == M_DIV || MODE == M_ADJ);
  constexpr bool GAUSS = NODEV;
  constexpr int NC = TF ? 1 : 3;         // staged coordinate arrays: z, or x, y, z
  constexpr int NA = NC + (NODEV ? 1 : 0);  // and the nodal field
  double (*s_pl)[NA][PP] = reinterpret_cast<double (*)[NA][PP]>(smem);
  double (*s_lo)[4][256] = reinterpret_cast<double (*)[4][256]>(smem + 2 * NA * PP);
  double (*s_up)[4][256] = reinterpret_cast<double (*)[4][256]>(smem + 2 * NA * PP + CH * 4 * 256);
  double* s_red = smem + 2 * NA * PP + 2 * CH * 4 * 256;

  const int t = threadIdx.x, ex = t % TE, ey = t / TE;
  const int i0 = bx * TN, j0 = by * TN;
  const int ie = i0 - 1 + ex, je = j0 - 1 + ey;
  const int nx = A.nx, ny = A.ny, nz = A.nz, NX = nx + 1, NY = ny + 1;
  const bool ev = ie >= 0 && ie < nx && je >= 0 && je < ny;
  const bool own = ex >= 1 && ey >= 1 && ie <= nx && je <= ny;
  const bool colfree = own && !A.faces.x_fixed(ie, NX) && !A.faces.y_fixed(je, NY);
  const int kf = A.faces.k_first(), kl = A.faces.k_last(nz + 1);
  const size_t plane = (size_t)NX * NY;
  const size_t E = (size_t)nx * ny * nz;

  // TF: the element column's x and y extent (the same on every layer)
  double x0 = 0.0, x1 = 1.0, y0 = 0.0, y1 = 1.0, hx = 1.0, hy = 1.0, ihx = 1.0, ihy = 1.0;
  if (TF && ev) {
    const size_t n = (size_t)je * NX + ie;
    x0 = A.X[n];
    x1 = A.X[n + 1];
    y0 = A.Y[n];
    y1 = A.Y[n + NX];
    hx = x1 - x0;
    hy = y1 - y0;
    ihx = 1.0 / hx;
    ihy = 1.0 / hy;
  }

  // staging: thread t loads tile node t, and t + 256 where that exists;
  // nodes outside the grid repeat the nearest grid node (no element uses them)
  constexpr int NH = (PP + 255) / 256;
  size_t src[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    const int q = min(t + 256 * h, PP - 1);
    const int gi = min(max(i0 - 1 + q % PN, 0), nx), gj = min(max(j0 - 1 + q / PN, 0), ny);
    src[h] = (size_t)gj * NX + gi;
  }
  double pre[NH][NA];
  auto load_plane = [&](int k) {
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const size_t n = (size_t)k * plane + src[h];
      if (!TF) {
        pre[h][0] = A.X[n];
        pre[h][1] = A.Y[n];
      }
      pre[h][NC - 1] = A.Z[n];
      if (NODEV) pre[h][NA - 1] = A.v[n];
    }
  };
  auto store_plane = [&](int b) {
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int q = t + 256 * h;
      if (q < PP) {
#pragma unroll
        for (int a = 0; a < NA; ++a) s_pl[b][a][q] = pre[h][a];
      }
    }
  };

  double acc[CH], carry[CH];
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) acc[ch] = carry[ch] = 0.0;

  auto node_out = [&](int k, const double s[CH]) {
    const size_t n = (size_t)k * plane + (size_t)je * NX + ie;
    const bool fr = colfree && k >= kf && k <= kl;
    if (MODE == M_APPLY) {
      A.out[n] = s[0];
    } else if (MODE == M_RESID) {
      const double r = fr ? A.f[n] - s[0] : 0.0;
      A.out[n] = r;
      acc[0] += r * r;
    } else {
      const double o = fr ? s[0] : 0.0;
      A.out[n] = o;
      acc[0] += o * o;
      if (CH == 2) {
        const double o1 = fr ? s[CH - 1] : 0.0;
        acc[CH - 1] += o1 * o1;
      }
    }
  };

  load_plane(0);
  store_plane(0);
  load_plane(1);
  store_plane(1);
  __syncthreads();
  for (int k = 0; k < nz; ++k) {
    const bool more = k + 2 <= nz;
    if (more) load_plane(k + 2);  // in flight while the elements of layer k are evaluated
    double y[CH][8];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
      for (int a = 0; a < 8; ++a) y[ch][a] = 0.0;
    if (ev) {
      double xe[3][8], ve[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int b = (k + (a >> 2)) & 1;
        const int q = ex + (a & 1) + PN * (ey + ((a >> 1) & 1));
        if (TF) {
          xe[0][a] = (a & 1) ? x1 : x0;
          xe[1][a] = (a & 2) ? y1 : y0;
        } else {
          xe[0][a] = s_pl[b][0][q];
          xe[1][a] = s_pl[b][1][q];
        }
        xe[2][a] = s_pl[b][NC - 1][q];
        ve[a] = NODEV ? s_pl[b][NA - 1][q] : 0.0;
      }
      if (GAUSS && TF) {
        double e[3][4], Zg[3][4];
        edge_diffs(xe[2], e);
#pragma unroll
        for (int m = 0; m < 3; ++m) bil4(e[m], Zg[m]);
        element_apply_tf(Zg, hx, hy, ihx, ihy, ve, A.c, y[0]);
      } else if (GAUSS) {
        double J2[3][3][4];
        gauss_jacobian2(xe, J2);
        element_apply2(J2, ve, A.c, y[0]);
      }
      if (ELEMV) {
        const size_t e = (size_t)k * nx * ny + (size_t)je * nx + ie;
        const double u[3] = {A.ue[e], A.ue[E + e], A.ue[2 * E + e]};
        if (MODE == M_RHS) element_rhs(xe, u, y[0]);
        if (MODE == M_ADJ) element_recover_adjoint(xe, u, A.c, y[0]);
        if (MODE == M_DIV) {
          // D0 = 8 detJ(0) B(0)^T u0, the negative of the right-hand side
          double tmp[8] = {};
          element_rhs(xe, u, tmp);
#pragma unroll
          for (int a = 0; a < 8; ++a) {
            y[0][a] -= tmp[a];
            y[CH - 1][a] = -tmp[a];
          }
          // the recovered wind u0 + diag(c) grad lambda(centre), as recover_body
          // computes it, written by the tile that owns the element's lower
          // corner node (each element exactly once)
          if (A.uout && ex >= 1 && ey >= 1) {
            double cj[3][3], r[3][3], g[3];
            centre_jacobian(xe, cj);
            const double det = adjugate(cj[0], cj[1], cj[2], r);
            centre_ref_grad(ve, g);
            const double idet = 1.0 / det;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const double gx = (g[0] * r[0][d] + g[1] * r[1][d] + g[2] * r[2][d]) * idet;
              A.uout[d * E + e] = u[d] + A.c[d] * gx;
            }
          }
        }
      }
    }
    __syncthreads();  // the last layer's contributions are summed and plane k is no longer read
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        s_lo[ch][q][t] = y[ch][q];
        s_up[ch][q][t] = y[ch][q + 4];
      }
    if (more) store_plane(k & 1);
    __syncthreads();
    if (own) {
      double sum[CH];
#pragma unroll
      for (int ch = 0; ch < CH; ++ch) {
        const double v = s_lo[ch][3][t - TE - 1] + s_lo[ch][2][t - TE] + s_lo[ch][1][t - 1] +
                         s_lo[ch][0][t];
        sum[ch] = k > 0 ? v + carry[ch] : v;
        carry[ch] = s_up[ch][3][t - TE - 1] + s_up[ch][2][t - TE] + s_up[ch][1][t - 1] +
                    s_up[ch][0][t];
      }
      node_out(k, sum);
    }
  }
  if (own) node_out(nz, carry);
  if (A.partials) {
    const int nb = A.gx * A.gy, bid = by * A.gx + bx;
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) block_sum_to(acc[ch], s_red, &A.partials[(size_t)ch * nb + bid]);
  }
  __syncthreads();  // the LDS slots are reused by the next work item of a batched launch
}

// TFM: 0 general grid, 1 terrain-following grid, 2 read from *A.tf_flag (0 =
// terrain-following), for a caller that only knows it on the device.
// Tiles are taken in x-fastest order, each XCD a contiguous range of them:
// a tile's node rows share their first and last cache lines with the tiles
// beside it in x, which then run on the same XCD and find them in its L2.
template <int MODE, int TFM>
__global__ __launch_bounds__(256) void elem_tile_kernel(TileJob A) {
  __shared__ double smem[TFM == 2 ? tile_lds_max(MODE) : tile_lds_doubles(MODE, TFM == 1)];
  const int b = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int bx = b % gridDim.x, by = b / gridDim.x;
  if (TFM == 1 || (TFM == 2 && *A.tf_flag == 0))
    elem_tile_body<MODE, true>(A, bx, by, smem);
  else
    elem_tile_body<MODE, false>(A, bx, by, smem);
}

template <int MODE>
__global__ __launch_bounds__(256) void elem_tile_batched(WorkList W) {
  __shared__ double smem[tile_lds_max(MODE)];
  for (int g = blockIdx.x; g < W.total; g += gridDim.x) {
    int lo = 0, hi = W.njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (W.prefix[mid] <= g) lo = mid;
      else hi = mid - 1;
    }
    if (!W.active[W.member[lo]]) continue;
    const TileJob& A = static_cast<const TileJob*>(W.jobs)[lo];
    const int b = g - W.prefix[lo];
    if (A.tf)
      elem_tile_body<MODE, true>(A, b % A.gx, b / A.gx, smem);
    else
      elem_tile_body<MODE, false>(A, b % A.gx, b / A.gx, smem);
  }
}

// Sets *flag when some node's x differs from that of node (i, 0, 0) or its y
// from that of node (0, j, 0): then the grid is not terrain-following.
__global__ __launch_bounds__(256) void structure_check_kernel(const double* __restrict__ X,
                                                              const double* __restrict__ Y, int NX,
                                                              int NY, size_t N, int* flag) {
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % NX), j = (int)((n / NX) % NY);
    if (X[n] != X[i] || Y[n] != Y[(size_t)j * NX]) atomicOr(flag, 1);
  }
}

// ---------------------------------------------------------------- element-wise kernels

// One thread per element column, marching up: recovery u = u0 + diag(c) grad lambda(0).
__device__ __forceinline__ void recover_body(const RecoverJob& R, int bx, int by) {
  const int ie = bx * 64 + (threadIdx.x & 63);
  const int je = by * 4 + (threadIdx.x >> 6);
  const int nx = R.nx, ny = R.ny, nz = R.nz;
  if (ie >= nx || je >= ny) return;
  const int NX = nx + 1, NY = ny + 1;
  const size_t plane = (size_t)NX * NY, E = (size_t)nx * ny * nz;
  double xe[3][8], v[8];
  auto load = [&](int k, int h) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const size_t n = (size_t)k * plane + (size_t)(je + (q >> 1)) * NX + ie + (q & 1);
      xe[0][q + h] = R.X[n];
      xe[1][q + h] = R.Y[n];
      xe[2][q + h] = R.Z[n];
      v[q + h] = R.lam[n];
    }
  };
  load(0, 0);
  for (int k = 0; k < nz; ++k) {
    load(k + 1, 4);
    double cj[3][3], r[3][3], g[3];
    centre_jacobian(xe, cj);
    const double det = adjugate(cj[0], cj[1], cj[2], r);
    centre_ref_grad(v, g);
    const double idet = 1.0 / det;
    const size_t e = (size_t)k * nx * ny + (size_t)je * nx + ie;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double gx = (g[0] * r[0][d] + g[1] * r[1][d] + g[2] * r[2][d]) * idet;
      R.u[d * E + e] = R.u0[d * E + e] + R.c[d] * gx;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int d = 0; d < 3; ++d) xe[d][q] = xe[d][q + 4];
      v[q] = v[q + 4];
    }
  }
}

__global__ __launch_bounds__(256) void recover_kernel(RecoverJob R) {
  recover_body(R, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void recover_batched(WorkList W) {
  for (int g = blockIdx.x; g < W.total; g += gridDim.x) {
    int lo = 0, hi = W.njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (W.prefix[mid] <= g) lo = mid;
      else hi = mid - 1;
    }
    if (!W.active[W.member[lo]]) continue;
    const RecoverJob& R = static_cast<const RecoverJob*>(W.jobs)[lo];
    const int b = g - W.prefix[lo];
    recover_body(R, b % R.gx, b / R.gx);
  }
}

// Adjoint element terms: dL/du0 = g_u - 8 detJ(0) B(0) mu (FP32 out) and the
// per-block sums of dL/dc_d = sum_e g_u,d (B(0) lambda)_d
//                             - sum_e sum_g detJ_g (B_g mu)_d (B_g lambda)_d.
__global__ __launch_bounds__(256) void adjoint_elem_kernel(
    const double* __restrict__ X, const double* __restrict__ Y, const double* __restrict__ Z,
    const double* __restrict__ lam, const double* __restrict__ mu, const double* __restrict__ gu,
    float* __restrict__ dL_du0, double* __restrict__ partials, int nx, int ny, int nz) {
  __shared__ double s_red[256];
  const int ie = blockIdx.x * 64 + (threadIdx.x & 63);
  const int je = blockIdx.y * 4 + (threadIdx.x >> 6);
  const bool act = ie < nx && je < ny;
  const int NX = nx + 1, NY = ny + 1;
  const size_t plane = (size_t)NX * NY, E = (size_t)nx * ny * nz;
  double acc[3] = {0.0, 0.0, 0.0};
  if (act) {
    double xe[3][8], vl[8], vm[8];
    auto load = [&](int k, int h) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const size_t n = (size_t)k * plane + (size_t)(je + (q >> 1)) * NX + ie + (q & 1);
        xe[0][q + h] = X[n];
        xe[1][q + h] = Y[n];
        xe[2][q + h] = Z[n];
        vl[q + h] = lam[n];
        vm[q + h] = mu[n];
      }
    };
    load(0, 0);
    for (int k = 0; k < nz; ++k) {
      load(k + 1, 4);
      const size_t e = (size_t)k * nx * ny + (size_t)je * nx + ie;
      const double g[3] = {gu[e], gu[E + e], gu[2 * E + e]};
      // centre terms
      double cj[3][3], r[3][3], gl[3], gm[3];
      centre_jacobian(xe, cj);
      const double det0 = adjugate(cj[0], cj[1], cj[2], r);
      centre_ref_grad(vl, gl);
      centre_ref_grad(vm, gm);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double tl = gl[0] * r[0][d] + gl[1] * r[1][d] + gl[2] * r[2][d];  // det * grad lambda
        const double tm = gm[0] * r[0][d] + gm[1] * r[1][d] + gm[2] * r[2][d];  // det * grad mu
        dL_du0[d * E + e] = (float)(g[d] - 8.0 * tm);
        acc[d] += g[d] * tl / det0;
      }
      // Gauss-point terms
      double Jg[3][3][4], el[3][4], em[3][4], Gl[3][4], Gm[3][4];
      gauss_jacobian(xe, Jg);
      edge_diffs(vl, el);
      edge_diffs(vm, em);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        bil4(el[m], Gl[m]);
        bil4(em[m], Gm[m]);
      }
#pragma unroll
      for (int gp = 0; gp < 8; ++gp) {
        GP_PAIRS(gp & 1, (gp >> 1) & 1, gp >> 2);
        const double c0[3] = {Jg[0][0][p0], Jg[0][1][p0], Jg[0][2][p0]};
        const double c1[3] = {Jg[1][0][p1], Jg[1][1][p1], Jg[1][2][p1]};
        const double c2[3] = {Jg[2][0][p2], Jg[2][1][p2], Jg[2][2][p2]};
        double rr[3][3];
        const double det = adjugate(c0, c1, c2, rr);
        const double idet = 1.0 / det;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double tl = 0.5 * (Gl[0][p0] * rr[0][d] + Gl[1][p1] * rr[1][d] + Gl[2][p2] * rr[2][d]);
          const double tm = 0.5 * (Gm[0][p0] * rr[0][d] + Gm[1][p1] * rr[1][d] + Gm[2][p2] * rr[2][d]);
          acc[d] -= tl * tm * idet;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int d = 0; d < 3; ++d) xe[d][q] = xe[d][q + 4];
        vl[q] = vl[q + 4];
        vm[q] = vm[q + 4];
      }
    }
  }
  const int nb = gridDim.x * gridDim.y, bid = blockIdx.y * gridDim.x + blockIdx.x;
  for (int d = 0; d < 3; ++d) block_sum_to(acc[d], s_red, &partials[(size_t)d * nb + bid]);
}

__global__ __launch_bounds__(256) void sumsq_kernel(const double* __restrict__ v, size_t n,
                                                    double* __restrict__ partials) {
  __shared__ double s_red[256];
  double a = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    a += v[i] * v[i];
  block_sum_to(a, s_red, &partials[blockIdx.x]);
}

dim3 tile_grid(const mcw_handle& h) {
  return dim3((h.d.NX() + TN - 1) / TN, (h.d.NY() + TN - 1) / TN);
}

}  // namespace

// ---------------------------------------------------------------- launchers

TileJob tile_job(const mcw_handle& h) {
  TileJob A{};
  A.tf = h.terrain ? 1 : 0;
  A.X = h.X.as<double>();
  A.Y = h.Y.as<double>();
  A.Z = h.Z.as<double>();
  A.nx = h.d.nx;
  A.ny = h.d.ny;
  A.nz = h.d.nz;
  A.c[0] = h.c[0];
  A.c[1] = h.c[1];
  A.c[2] = h.c[2];
  A.faces = h.faces;
  const dim3 g = tile_grid(h);
  A.gx = (int)g.x;
  A.gy = (int)g.y;
  return A;
}

RecoverJob recover_job(const mcw_handle& h, const double* u0, const double* lam, double* u) {
  RecoverJob R{};
  R.X = h.X.as<double>();
  R.Y = h.Y.as<double>();
  R.Z = h.Z.as<double>();
  R.lam = lam;
  R.u0 = u0;
  R.u = u;
  R.nx = h.d.nx;
  R.ny = h.d.ny;
  R.nz = h.d.nz;
  R.c[0] = h.c[0];
  R.c[1] = h.c[1];
  R.c[2] = h.c[2];
  R.gx = (h.d.nx + 63) / 64;
  R.gy = (h.d.ny + 3) / 4;
  return R;
}

void launch_tile_batched(int mode, const WorkList& W, hipStream_t s) {
  if (W.total <= 0) return;
  const unsigned g = (unsigned)std::max(1, std::min(W.total, 4096));
  switch (mode) {
    case M_RESID: elem_tile_batched<M_RESID><<<g, 256, 0, s>>>(W); break;
    case M_RHS: elem_tile_batched<M_RHS><<<g, 256, 0, s>>>(W); break;
    case M_DIV: elem_tile_batched<M_DIV><<<g, 256, 0, s>>>(W); break;
    default: throw Error{MCW_INVALID_ARG, "unsupported batched element mode"};
  }
  MCW_CHECK_LAUNCH();
}

void launch_recover_batched(const WorkList& W, hipStream_t s) {
  if (W.total <= 0) return;
  const unsigned g = (unsigned)std::max(1, std::min(W.total, 8192));
  recover_batched<<<g, 256, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

void launch_geometry_check(const mcw_handle& h, long long* first_bad) {
  const long long E = (long long)h.d.nx * h.d.ny * h.d.nz;
  const unsigned blocks = (unsigned)((E + 255) / 256);
  geometry_check_kernel<<<blocks, 256, 0, h.stream>>>(h.X.as<double>(), h.Y.as<double>(),
                                                      h.Z.as<double>(), h.d.nx, h.d.ny, h.d.nz,
                                                      reinterpret_cast<unsigned long long*>(first_bad));
  MCW_CHECK_LAUNCH();
}

void launch_assemble_stencil(const mcw_handle& h, double* st64) {
  const int nx = h.d.nx, ny = h.d.ny, nz = h.d.nz;
  for (int pk = 0; pk < 2; ++pk)
    for (int pj = 0; pj < 2; ++pj)
      for (int pi = 0; pi < 2; ++pi) {
        const long long m = (long long)((nx - pi + 1) / 2) * ((ny - pj + 1) / 2) * ((nz - pk + 1) / 2);
        if (m == 0) continue;
        assemble_kernel<<<(unsigned)((m + 255) / 256), 256, 0, h.stream>>>(
            h.X.as<double>(), h.Y.as<double>(), h.Z.as<double>(), nx, ny, nz, h.c[0], h.c[1],
            h.c[2], pi, pj, pk, st64);
        MCW_CHECK_LAUNCH();
      }
}

// mode 0: out = K x (no boundary conditions); mode 1: out = f - K x at free nodes, 0 elsewhere.
void launch_apply(const mcw_handle& h, const double* x, const double* f, double* out, int mode,
                  double* partials, size_t* n_part) {
  TileJob A = tile_job(h);
  A.v = x;
  A.f = f;
  A.out = out;
  A.partials = partials;
  const dim3 g = tile_grid(h);
  if (partials) need_partials((size_t)g.x * g.y, h.n_partials);
  if (mode == 0 && A.tf)
    elem_tile_kernel<M_APPLY, 1><<<g, 256, 0, h.stream>>>(A);
  else if (mode == 0)
    elem_tile_kernel<M_APPLY, 0><<<g, 256, 0, h.stream>>>(A);
  else if (A.tf)
    elem_tile_kernel<M_RESID, 1><<<g, 256, 0, h.stream>>>(A);
  else
    elem_tile_kernel<M_RESID, 0><<<g, 256, 0, h.stream>>>(A);
  MCW_CHECK_LAUNCH();
  if (n_part) *n_part = (size_t)g.x * g.y;
}

void launch_rhs(const mcw_handle& h, const double* u0, double* f, double* partials, size_t* n_part) {
  TileJob A = tile_job(h);
  A.ue = u0;
  A.out = f;
  A.partials = partials;
  const dim3 g = tile_grid(h);
  if (partials) need_partials((size_t)g.x * g.y, h.n_partials);
  if (A.tf)
    elem_tile_kernel<M_RHS, 1><<<g, 256, 0, h.stream>>>(A);
  else
    elem_tile_kernel<M_RHS, 0><<<g, 256, 0, h.stream>>>(A);
  MCW_CHECK_LAUNCH();
  if (n_part) *n_part = (size_t)g.x * g.y;
}

size_t tile_count(const Dims& d) {
  return (size_t)((d.NX() + TN - 1) / TN) * (size_t)((d.NY() + TN - 1) / TN);
}

void launch_divergence_ref(const GridRef& G, const double* u0, const double* lam, double* D,
                           double* partials, hipStream_t s, double* u) {
  TileJob A{};
  A.uout = u;
  A.X = G.X;
  A.Y = G.Y;
  A.Z = G.Z;
  A.nx = G.d.nx;
  A.ny = G.d.ny;
  A.nz = G.d.nz;
  for (int d = 0; d < 3; ++d) A.c[d] = G.c[d];
  A.faces = G.faces;
  const dim3 g((G.d.NX() + TN - 1) / TN, (G.d.NY() + TN - 1) / TN);
  A.gx = (int)g.x;
  A.gy = (int)g.y;
  A.ue = u0;
  A.v = lam;
  A.out = D;
  A.partials = partials;
  A.tf = G.tf;
  A.tf_flag = G.tf_flag;
  if (G.tf_flag)
    elem_tile_kernel<M_DIV, 2><<<g, 256, 0, s>>>(A);
  else if (G.tf)
    elem_tile_kernel<M_DIV, 1><<<g, 256, 0, s>>>(A);
  else
    elem_tile_kernel<M_DIV, 0><<<g, 256, 0, s>>>(A);
  MCW_CHECK_LAUNCH();
}

void launch_structure_check(const double* X, const double* Y, const Dims& d, int* flag,
                            hipStream_t s) {
  const size_t N = d.N();
  const unsigned blocks = (unsigned)std::min<size_t>((N + 255) / 256, 8192);
  structure_check_kernel<<<blocks, 256, 0, s>>>(X, Y, d.NX(), d.NY(), N, flag);
  MCW_CHECK_LAUNCH();
}

void launch_divergence(const mcw_handle& h, const double* u0, const double* lam, double* D,
                       double* partials, size_t* n_part, double* u) {
  const size_t tiles = tile_count(h.d);
  if (partials) need_partials(2 * tiles, h.n_partials);
  GridRef G{h.X.as<double>(), h.Y.as<double>(), h.Z.as<double>(), h.d, {h.c[0], h.c[1], h.c[2]},
            h.faces, h.terrain ? 1 : 0, nullptr};
  launch_divergence_ref(G, u0, lam, D, partials, h.stream, u);
  if (n_part) *n_part = tiles;
}

void launch_adjoint_scatter(const mcw_handle& h, const double* g_u, double* g_lam, double* partials,
                            size_t* n_part) {
  TileJob A = tile_job(h);
  A.ue = g_u;
  A.out = g_lam;
  A.partials = partials;
  const dim3 g = tile_grid(h);
  if (partials) need_partials((size_t)g.x * g.y, h.n_partials);
  if (A.tf)
    elem_tile_kernel<M_ADJ, 1><<<g, 256, 0, h.stream>>>(A);
  else
    elem_tile_kernel<M_ADJ, 0><<<g, 256, 0, h.stream>>>(A);
  MCW_CHECK_LAUNCH();
  if (n_part) *n_part = (size_t)g.x * g.y;
}

void launch_recover(const mcw_handle& h, const double* u0, const double* lam, double* u) {
  const RecoverJob R = recover_job(h, u0, lam, u);
  recover_kernel<<<dim3(R.gx, R.gy), 256, 0, h.stream>>>(R);
  MCW_CHECK_LAUNCH();
}

void launch_adjoint_elements(const mcw_handle& h, const double* g_u, const double* lam,
                             const double* mu, float* dL_du0, double* partials, size_t* n_part) {
  const dim3 g((h.d.nx + 63) / 64, (h.d.ny + 3) / 4);
  need_partials(3 * (size_t)g.x * g.y, h.n_partials);
  adjoint_elem_kernel<<<g, 256, 0, h.stream>>>(h.X.as<double>(), h.Y.as<double>(),
                                               h.Z.as<double>(), lam, mu, g_u, dL_du0, partials,
                                               h.d.nx, h.d.ny, h.d.nz);
  MCW_CHECK_LAUNCH();
  if (n_part) *n_part = (size_t)g.x * g.y;
}

void launch_check_finite(const mcw_handle& h, const double* v, size_t n, double* partials,
                         size_t* n_part) {
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  need_partials(blocks, h.n_partials);
  sumsq_kernel<<<blocks, 256, 0, h.stream>>>(v, n, partials);
  MCW_CHECK_LAUNCH();
  if (n_part) *n_part = blocks;
}

}  // namespace mcw
