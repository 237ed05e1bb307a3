// Steps on either side of the solve in a coupled fire-atmosphere model: the
// coarse atmospheric wind interpolated to the element centres (the solve's u0)
// and the horizontal wind at a fixed height above the terrain taken from the
// solved wind (what the fire model reads).  The paper places the solve in the
// spot of the plain interpolation (Sec. 1); the vertical rule is linear in
// height above ground between levels, constant above the top level and the
// neutral log law below the lowest one.
//
// One thread per element column, lanes along x; each thread marches up its
// column keeping the corner nodes of the current plane in registers, so node
// coordinates are read once per plane and the (small, cached) coarse columns
// are searched with a hint that only moves up.
#include "mcw_internal.hpp"

namespace mcw {
namespace {

constexpr int CT = 256;

struct InterpJob {
  const double *X, *Y, *Z;
  int nx, ny, nz;
  // coarse wind
  int ncx, ncy, nl;
  double x0, y0, dx, dy, z0;
  const double* hagl;  // (nl, ncy, ncx)
  const double* wind;  // (3, nl, ncy, ncx)
  double* u0;          // (3, nz, ny, nx)
};

// Lower index and weight along one axis; the position is clamped to the grid.
__device__ __forceinline__ void axis_cell(double pos, double origin, double spacing, int n, int& i0,
                                          double& w) {
  double s = (pos - origin) / spacing;
  s = fmin(fmax(s, 0.0), (double)(n - 1));
  int i = (int)floor(s);
  i = i < n - 2 ? i : n - 2;
  i0 = i;
  w = s - (double)i;
}

// Wind of one coarse column at height zeta; `l` is the search hint (the last
// level at or below the previous height of this column).
__device__ __forceinline__ void column_wind(const InterpJob& J, size_t plane, size_t c, double zeta,
                                            int& l, double v[3]) {
  const double* h = J.hagl + c;
  while (l + 1 < J.nl && h[(size_t)(l + 1) * plane] <= zeta) ++l;
  while (l > 0 && h[(size_t)l * plane] > zeta) --l;
  const size_t dstride = (size_t)J.nl * plane;
  const double* w = J.wind + c;
  const double h0 = h[0];
  if (zeta >= h[(size_t)(J.nl - 1) * plane]) {
    for (int d = 0; d < 3; ++d) v[d] = w[d * dstride + (size_t)(J.nl - 1) * plane];
  } else if (zeta >= h0) {
    const double ha = h[(size_t)l * plane], hb = h[(size_t)(l + 1) * plane];
    const double t = (zeta - ha) / (hb - ha);
    for (int d = 0; d < 3; ++d)
      v[d] = (1.0 - t) * w[d * dstride + (size_t)l * plane] + t * w[d * dstride + (size_t)(l + 1) * plane];
  } else if (zeta <= J.z0) {
    v[0] = v[1] = v[2] = 0.0;
  } else {
    const double f = log(zeta / J.z0) / log(h0 / J.z0);
    for (int d = 0; d < 3; ++d) v[d] = w[d * dstride] * f;
  }
}

__global__ __launch_bounds__(CT) void interp_wind_kernel(InterpJob J) {
  const size_t col = (size_t)blockIdx.x * CT + threadIdx.x;
  if (col >= (size_t)J.nx * J.ny) return;
  const int i = (int)(col % J.nx), j = (int)(col / J.nx);
  const int NX = J.nx + 1;
  const size_t nplane = (size_t)NX * (J.ny + 1);
  const size_t n00 = (size_t)j * NX + i, n10 = n00 + 1, n01 = n00 + NX, n11 = n01 + 1;
  double xl[4], yl[4], zl[4];
  const size_t nodes[4] = {n00, n10, n01, n11};
  for (int q = 0; q < 4; ++q) {
    xl[q] = J.X[nodes[q]];
    yl[q] = J.Y[nodes[q]];
    zl[q] = J.Z[nodes[q]];
  }
  const double zs = 0.25 * (zl[0] + zl[1] + zl[2] + zl[3]);
  const size_t cplane = (size_t)J.ncx * J.ncy;
  int cell_i = -1, cell_j = -1;
  int hint[4] = {0, 0, 0, 0};
  const size_t eplane = (size_t)J.nx * J.ny, estride = eplane * J.nz;
  for (int k = 0; k < J.nz; ++k) {
    double xu[4], yu[4], zu[4];
    const size_t p = (size_t)(k + 1) * nplane;
    for (int q = 0; q < 4; ++q) {
      xu[q] = J.X[p + nodes[q]];
      yu[q] = J.Y[p + nodes[q]];
      zu[q] = J.Z[p + nodes[q]];
    }
    double xc = 0.0, yc = 0.0, zc = 0.0;
    for (int q = 0; q < 4; ++q) {
      xc += xl[q] + xu[q];
      yc += yl[q] + yu[q];
      zc += zl[q] + zu[q];
    }
    xc *= 0.125;
    yc *= 0.125;
    zc *= 0.125;
    const double zeta = zc - zs;
    int I, Jc;
    double a, b;
    axis_cell(xc, J.x0, J.dx, J.ncx, I, a);
    axis_cell(yc, J.y0, J.dy, J.ncy, Jc, b);
    if (I != cell_i || Jc != cell_j) {
      cell_i = I;
      cell_j = Jc;
      hint[0] = hint[1] = hint[2] = hint[3] = 0;
    }
    const double wq[4] = {(1.0 - a) * (1.0 - b), a * (1.0 - b), (1.0 - a) * b, a * b};
    double u[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 4; ++q) {
      const size_t c = (size_t)(Jc + (q >> 1)) * J.ncx + (I + (q & 1));
      double v[3];
      column_wind(J, cplane, c, zeta, hint[q], v);
      for (int d = 0; d < 3; ++d) u[d] += wq[q] * v[d];
    }
    const size_t e = (size_t)k * eplane + col;
    for (int d = 0; d < 3; ++d) J.u0[d * estride + e] = u[d];
    for (int q = 0; q < 4; ++q) {
      xl[q] = xu[q];
      yl[q] = yu[q];
      zl[q] = zu[q];
    }
  }
}

// hagl must start above z0 and increase up every column; bad[0] = 1 otherwise
__global__ __launch_bounds__(CT) void coarse_check_kernel(const double* __restrict__ hagl, int nl,
                                                          size_t plane, double z0, int* bad) {
  const size_t c = (size_t)blockIdx.x * CT + threadIdx.x;
  if (c >= plane) return;
  double prev = z0;
  bool ok = true;
  for (int l = 0; l < nl; ++l) {
    const double h = hagl[(size_t)l * plane + c];
    ok = ok && isfinite(h) && h > prev;
    prev = h;
  }
  if (!ok) bad[0] = 1;
}

__global__ void clear_flag_kernel(int* bad) {
  if (threadIdx.x == 0) bad[0] = 0;
}

struct SurfaceJob {
  const double* Z;
  const double* u;  // (3, nz, ny, nx)
  int nx, ny, nz;
  double height, z0;
  double* uv;  // (2, ny, nx)
};

__global__ __launch_bounds__(CT) void surface_wind_kernel(SurfaceJob S) {
  const size_t col = (size_t)blockIdx.x * CT + threadIdx.x;
  if (col >= (size_t)S.nx * S.ny) return;
  const int i = (int)(col % S.nx), j = (int)(col / S.nx);
  const int NX = S.nx + 1;
  const size_t nplane = (size_t)NX * (S.ny + 1);
  const size_t n00 = (size_t)j * NX + i;
  const size_t nodes[4] = {n00, n00 + 1, n00 + NX, n00 + NX + 1};
  double zl = 0.0, zu = 0.0;
  for (int q = 0; q < 4; ++q) zl += S.Z[nodes[q]];
  for (int q = 0; q < 4; ++q) zu += S.Z[nplane + nodes[q]];
  const double zs = 0.25 * zl;
  double zeta = 0.125 * (zl + zu) - zs;  // centre of layer 0
  const size_t eplane = (size_t)S.nx * S.ny, estride = eplane * S.nz;
  const double H = S.height;
  double out[2];
  if (H < zeta) {
    // below the lowest centre: log law from it
    const double f = H <= S.z0 ? 0.0 : log(H / S.z0) / log(zeta / S.z0);
    for (int d = 0; d < 2; ++d) out[d] = S.u[d * estride + col] * f;
  } else {
    int k = 0;
    double zeta_k = zeta, zeta_n = zeta;
    while (k + 1 < S.nz) {
      // centre of layer k+1: planes k+1 and k+2
      const double za = zu;
      double zb = 0.0;
      for (int q = 0; q < 4; ++q) zb += S.Z[(size_t)(k + 2) * nplane + nodes[q]];
      zeta_n = 0.125 * (za + zb) - zs;
      if (zeta_n > H) break;
      zu = zb;
      zeta_k = zeta_n;
      ++k;
    }
    if (k == S.nz - 1) {
      for (int d = 0; d < 2; ++d) out[d] = S.u[d * estride + (size_t)k * eplane + col];
    } else {
      const double t = (H - zeta_k) / (zeta_n - zeta_k);
      for (int d = 0; d < 2; ++d)
        out[d] = (1.0 - t) * S.u[d * estride + (size_t)k * eplane + col] +
                 t * S.u[d * estride + (size_t)(k + 1) * eplane + col];
    }
  }
  S.uv[col] = out[0];
  S.uv[eplane + col] = out[1];
}

unsigned blocks_for(size_t n) { return (unsigned)((n + CT - 1) / CT); }

}  // namespace

bool launch_coarse_check(const mcw_handle& h, const mcw_coarse_wind& cw) {
  int* bad = h.flag.as<int>();
  clear_flag_kernel<<<1, 64, 0, h.stream>>>(bad);
  MCW_CHECK_LAUNCH();
  const size_t plane = (size_t)cw.ncx * cw.ncy;
  coarse_check_kernel<<<blocks_for(plane), CT, 0, h.stream>>>(cw.hagl, cw.nl, plane, cw.z0, bad);
  MCW_CHECK_LAUNCH();
  int flag = 0;
  MCW_HIP(hipMemcpyAsync(&flag, bad, sizeof(int), hipMemcpyDeviceToHost, h.stream));
  MCW_HIP(hipStreamSynchronize(h.stream));
  return flag == 0;
}

void launch_interp_wind(const mcw_handle& h, const mcw_coarse_wind& cw, double* u0) {
  InterpJob J{};
  J.X = h.X.as<double>();
  J.Y = h.Y.as<double>();
  J.Z = h.Z.as<double>();
  J.nx = h.d.nx;
  J.ny = h.d.ny;
  J.nz = h.d.nz;
  J.ncx = cw.ncx;
  J.ncy = cw.ncy;
  J.nl = cw.nl;
  J.x0 = cw.x0;
  J.y0 = cw.y0;
  J.dx = cw.dx;
  J.dy = cw.dy;
  J.z0 = cw.z0;
  J.hagl = cw.hagl;
  J.wind = cw.wind;
  J.u0 = u0;
  interp_wind_kernel<<<blocks_for((size_t)h.d.nx * h.d.ny), CT, 0, h.stream>>>(J);
  MCW_CHECK_LAUNCH();
}

void launch_surface_wind(const mcw_handle& h, const double* u, double height, double z0, double* uv) {
  const SurfaceJob S{h.Z.as<double>(), u, h.d.nx, h.d.ny, h.d.nz, height, z0, uv};
  surface_wind_kernel<<<blocks_for((size_t)h.d.nx * h.d.ny), CT, 0, h.stream>>>(S);
  MCW_CHECK_LAUNCH();
}

}  // namespace mcw
