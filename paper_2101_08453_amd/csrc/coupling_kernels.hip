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
// coordinates are read once per plane, and searches the coarse columns with a
// hint that only moves up.  A block covers a 64 x 4 tile of element columns and
// first copies the coarse columns around its tile to LDS, so that the searches
// and the interpolation read LDS instead of chains of dependent global loads.
#include "mcw_internal.hpp"

namespace mcw {
namespace {

constexpr int CT = 256;

// element columns per block of the interpolation, and the LDS it may use for
// staged coarse columns (each takes 4 nl doubles: height, then 3 components)
constexpr int IT_X = 64, IT_Y = 4;
constexpr int STAGE_BYTES = 32 * 1024;

struct InterpJob {
  const double *X, *Y, *Z;
  int nx, ny, nz, tiles_x;
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
// level at or below the previous height of this column).  h[l * hs] is the
// height of level l and w[d * wd + l * ws] its component d, in global memory
// (strides of the coarse grid) or in LDS (a staged column).
__device__ __forceinline__ void column_wind(const InterpJob& J, const double* h, size_t hs,
                                            const double* w, size_t ws, size_t wd, double zeta,
                                            int& l, double v[3]) {
  while (l + 1 < J.nl && h[(size_t)(l + 1) * hs] <= zeta) ++l;
  while (l > 0 && h[(size_t)l * hs] > zeta) --l;
  const double h0 = h[0];
  if (zeta >= h[(size_t)(J.nl - 1) * hs]) {
    for (int d = 0; d < 3; ++d) v[d] = w[d * wd + (size_t)(J.nl - 1) * ws];
  } else if (zeta >= h0) {
    const double ha = h[(size_t)l * hs], hb = h[(size_t)(l + 1) * hs];
    const double t = (zeta - ha) / (hb - ha);
    for (int d = 0; d < 3; ++d)
      v[d] = (1.0 - t) * w[d * wd + (size_t)l * ws] + t * w[d * wd + (size_t)(l + 1) * ws];
  } else if (zeta <= J.z0) {
    v[0] = v[1] = v[2] = 0.0;
  } else {
    const double f = log(zeta / J.z0) / log(h0 / J.z0);
    for (int d = 0; d < 3; ++d) v[d] = w[d * wd] * f;
  }
}

// Element centre (mean of the 8 corners) from the corner nodes of two planes.
__device__ __forceinline__ void centre_of(const double xl[4], const double yl[4], const double zl[4],
                                          const double xu[4], const double yu[4], const double zu[4],
                                          double& xc, double& yc, double& zc) {
  xc = yc = zc = 0.0;
  for (int q = 0; q < 4; ++q) {
    xc += xl[q] + xu[q];
    yc += yl[q] + yu[q];
    zc += zl[q] + zu[q];
  }
  xc *= 0.125;
  yc *= 0.125;
  zc *= 0.125;
}

__global__ __launch_bounds__(IT_X * IT_Y) void interp_wind_kernel(InterpJob J) {
  extern __shared__ double stage[];
  __shared__ int win[4];  // staged coarse columns: I in [win[0], win[1]], J in [win[2], win[3]]
  const int i = (blockIdx.x % J.tiles_x) * IT_X + (threadIdx.x % IT_X);
  const int j = (blockIdx.x / J.tiles_x) * IT_Y + (threadIdx.x / IT_X);
  const bool in = i < J.nx && j < J.ny;
  const size_t col = in ? (size_t)j * J.nx + i : 0;
  const int NX = J.nx + 1;
  const size_t nplane = (size_t)NX * (J.ny + 1);
  const size_t n00 = in ? (size_t)j * NX + i : 0, n10 = n00 + 1, n01 = n00 + NX, n11 = n01 + 1;
  const size_t nodes[4] = {n00, n10, n01, n11};
  double xl[4], yl[4], zl[4], xu[4], yu[4], zu[4];
  for (int q = 0; q < 4; ++q) {
    xl[q] = J.X[nodes[q]];
    yl[q] = J.Y[nodes[q]];
    zl[q] = J.Z[nodes[q]];
    xu[q] = J.X[nplane + nodes[q]];
    yu[q] = J.Y[nplane + nodes[q]];
    zu[q] = J.Z[nplane + nodes[q]];
  }
  const double zs = 0.25 * (zl[0] + zl[1] + zl[2] + zl[3]);
  const size_t cplane = (size_t)J.ncx * J.ncy;
  // the coarse cells under the tile's bottom-layer centres, and their corners
  double xc, yc, zc;
  centre_of(xl, yl, zl, xu, yu, zu, xc, yc, zc);
  int I, Jc;
  double a, b;
  axis_cell(xc, J.x0, J.dx, J.ncx, I, a);
  axis_cell(yc, J.y0, J.dy, J.ncy, Jc, b);
  if (threadIdx.x == 0) {
    win[0] = win[2] = 1 << 30;
    win[1] = win[3] = -1;
  }
  __syncthreads();
  if (in) {
    atomicMin(&win[0], I);
    atomicMax(&win[1], I + 1);
    atomicMin(&win[2], Jc);
    atomicMax(&win[3], Jc + 1);
  }
  __syncthreads();
  const int wi0 = win[0], wi1 = win[1], wj0 = win[2], wj1 = win[3];
  const int wx = wi1 - wi0 + 1, ncols = wx * (wj1 - wj0 + 1);
  const int cw = 4 * J.nl;  // doubles per staged column
  const bool staged = wi1 >= wi0 && (size_t)ncols * cw * sizeof(double) <= (size_t)STAGE_BYTES;
  if (staged) {
    for (int t = threadIdx.x; t < ncols * cw; t += blockDim.x) {
      const int slot = t / cw, r = t % cw, part = r / J.nl, l = r % J.nl;
      const size_t c = (size_t)(wj0 + slot / wx) * J.ncx + (wi0 + slot % wx);
      stage[t] = part == 0 ? J.hagl[(size_t)l * cplane + c]
                           : J.wind[((size_t)(part - 1) * J.nl + l) * cplane + c];
    }
  }
  __syncthreads();
  if (!in) return;
  int cell_i = -1, cell_j = -1;
  int hint[4] = {0, 0, 0, 0};
  const size_t eplane = (size_t)J.nx * J.ny, estride = eplane * J.nz;
  for (int k = 0; k < J.nz; ++k) {
    if (k > 0) {
      const size_t p = (size_t)(k + 1) * nplane;
      for (int q = 0; q < 4; ++q) {
        xl[q] = xu[q];
        yl[q] = yu[q];
        zl[q] = zu[q];
        xu[q] = J.X[p + nodes[q]];
        yu[q] = J.Y[p + nodes[q]];
        zu[q] = J.Z[p + nodes[q]];
      }
      centre_of(xl, yl, zl, xu, yu, zu, xc, yc, zc);
      axis_cell(xc, J.x0, J.dx, J.ncx, I, a);
      axis_cell(yc, J.y0, J.dy, J.ncy, Jc, b);
    }
    const double zeta = zc - zs;
    if (I != cell_i || Jc != cell_j) {
      cell_i = I;
      cell_j = Jc;
      hint[0] = hint[1] = hint[2] = hint[3] = 0;
    }
    const bool lds = staged && I >= wi0 && I + 1 <= wi1 && Jc >= wj0 && Jc + 1 <= wj1;
    const double wq[4] = {(1.0 - a) * (1.0 - b), a * (1.0 - b), (1.0 - a) * b, a * b};
    double u[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 4; ++q) {
      const int ci = I + (q & 1), cj = Jc + (q >> 1);
      double v[3];
      if (lds) {
        const double* sc = stage + (size_t)((cj - wj0) * wx + (ci - wi0)) * cw;
        column_wind(J, sc, 1, sc + J.nl, 1, J.nl, zeta, hint[q], v);
      } else {
        const size_t c = (size_t)cj * J.ncx + ci;
        column_wind(J, J.hagl + c, cplane, J.wind + c, cplane, (size_t)J.nl * cplane, zeta, hint[q], v);
      }
      for (int d = 0; d < 3; ++d) u[d] += wq[q] * v[d];
    }
    const size_t e = (size_t)k * eplane + col;
    for (int d = 0; d < 3; ++d) J.u0[d * estride + e] = u[d];
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
  J.tiles_x = (h.d.nx + IT_X - 1) / IT_X;
  const unsigned tiles = (unsigned)J.tiles_x * (unsigned)((h.d.ny + IT_Y - 1) / IT_Y);
  interp_wind_kernel<<<tiles, IT_X * IT_Y, STAGE_BYTES, h.stream>>>(J);
  MCW_CHECK_LAUNCH();
}

void launch_surface_wind(const mcw_handle& h, const double* u, double height, double z0, double* uv) {
  const SurfaceJob S{h.Z.as<double>(), u, h.d.nx, h.d.ny, h.d.nz, height, z0, uv};
  surface_wind_kernel<<<blocks_for((size_t)h.d.nx * h.d.ny), CT, 0, h.stream>>>(S);
  MCW_CHECK_LAUNCH();
}

}  // namespace mcw
