// Multigrid kernels on 27-point node stencils (Sec. 3 of Mandel et al.):
// Gauss-Seidel in vertical sweeps with the columns in four red-black groups,
// residual, restriction f_c = P^T r, prolongation u += P u_c, the Galerkin
// coarse operator K_c = P^T K P (eq. (7)), the coarsest direct solve, and the
// precision casts of the FP32-inside-FP64 refinement.
//
// Stencil layout: 27 coefficient planes of N entries; coefficient o =
// (di+1) + 3(dj+1) + 9(dk+1) of node (i,j,k) couples it to (i+di, j+dj, k+dk).
// Within each grid row the entries are stored even-i first, then odd-i, so a
// colour pass (every other i) reads contiguous memory.  Entries towards
// nodes off the grid are exactly zero, so neighbour indices are clamped.
// Node vectors are in natural x-fastest order.
#include "mcw_internal.hpp"

namespace mcw {
namespace {

constexpr int BX = 64;  // columns per block along x (one wave)
constexpr int BY = 4;   // rows of columns per block

__device__ __forceinline__ int rowpos(int i, int NXe) { return (i & 1) ? NXe + (i >> 1) : (i >> 1); }

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so that neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, rem = n & 7, x = b & 7, s = b >> 3;
  return x * q + min(x, rem) + s;
}

// ---------------------------------------------------------------- smoother

// One colour pass: every column (i, j) with i = ci mod 2, j = cj mod 2 runs
// pointwise Gauss-Seidel from the bottom to the top.  Neighbour columns belong
// to other colours and are not changed during the pass; the value below is
// this thread's own freshly updated one.
template <class T>
__global__ __launch_bounds__(256) void gs_pass_kernel(const T* __restrict__ st,
                                                      const T* __restrict__ f, T* __restrict__ x,
                                                      int NX, int NY, int NZ, Faces fc, int ci,
                                                      int cj, int ncx, int ncy, int tiles_x,
                                                      int nblocks) {
  const int b = xcd_remap(blockIdx.x, nblocks);
  const int ii = (b % tiles_x) * BX + (threadIdx.x % BX);
  const int jj = (b / tiles_x) * BY + (threadIdx.x / BX);
  if (ii >= ncx || jj >= ncy) return;
  const int i = 2 * ii + ci, j = 2 * jj + cj;
  if (fc.x_fixed(i, NX) || fc.y_fixed(j, NY)) return;
  const int im = i > 0 ? i - 1 : i, ip = i < NX - 1 ? i + 1 : i;
  const int jm = j > 0 ? j - 1 : j, jp = j < NY - 1 ? j + 1 : j;
  const int NXe = (NX + 1) >> 1;
  const int cols[9] = {jm * NX + im, jm * NX + i, jm * NX + ip, j * NX + im, j * NX + i,
                       j * NX + ip, jp * NX + im, jp * NX + i, jp * NX + ip};
  const size_t plane = (size_t)NX * NY;
  const size_t N = plane * NZ;
  const int cpos = j * NX + rowpos(i, NXe);
  const int kf = fc.k_first(), kl = fc.k_last(NZ);
  T xm[9], x0[9], xp[9];
  {
    const size_t pm = (size_t)(kf > 0 ? kf - 1 : 0) * plane, p0 = (size_t)kf * plane;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      xm[q] = x[pm + cols[q]];
      x0[q] = x[p0 + cols[q]];
    }
  }
  for (int k = kf; k <= kl; ++k) {
    const size_t pp = (size_t)(k + 1 < NZ ? k + 1 : NZ - 1) * plane;
#pragma unroll
    for (int q = 0; q < 9; ++q) xp[q] = x[pp + cols[q]];
    const size_t cb = (size_t)k * plane + cpos;
    T s = f[(size_t)k * plane + cols[4]];
#pragma unroll
    for (int o = 0; o < 27; ++o) {
      if (o == 13) continue;
      const int dk = o / 9, q = o % 9;
      const T xv = dk == 0 ? xm[q] : (dk == 1 ? x0[q] : xp[q]);
      s -= st[(size_t)o * N + cb] * xv;
    }
    const T xn = s / st[(size_t)13 * N + cb];
    x[(size_t)k * plane + cols[4]] = xn;
    x0[4] = xn;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      xm[q] = x0[q];
      x0[q] = xp[q];
    }
  }
}

// ---------------------------------------------------------------- residual

template <class T, bool NORM>
__global__ __launch_bounds__(256) void residual_kernel(const T* __restrict__ st,
                                                       const T* __restrict__ x,
                                                       const T* __restrict__ f, T* __restrict__ r,
                                                       int NX, int NY, int NZ, Faces fc,
                                                       int tiles_x, int nblocks,
                                                       double* __restrict__ partials) {
  __shared__ double s_red[256];
  const int b = xcd_remap(blockIdx.x, nblocks);
  const int i = (b % tiles_x) * BX + (threadIdx.x % BX);
  const int j = (b / tiles_x) * BY + (threadIdx.x / BX);
  double acc = 0.0;
  if (i < NX && j < NY) {
    const size_t plane = (size_t)NX * NY, N = plane * NZ;
    const bool colfree = !fc.x_fixed(i, NX) && !fc.y_fixed(j, NY);
    const int kf = fc.k_first(), kl = fc.k_last(NZ);
    const int im = i > 0 ? i - 1 : i, ip = i < NX - 1 ? i + 1 : i;
    const int jm = j > 0 ? j - 1 : j, jp = j < NY - 1 ? j + 1 : j;
    const int NXe = (NX + 1) >> 1;
    const int cols[9] = {jm * NX + im, jm * NX + i, jm * NX + ip, j * NX + im, j * NX + i,
                         j * NX + ip, jp * NX + im, jp * NX + i, jp * NX + ip};
    const int cpos = j * NX + rowpos(i, NXe);
    T xm[9], x0[9], xp[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      xm[q] = x[cols[q]];
      x0[q] = xm[q];
    }
    for (int k = 0; k < NZ; ++k) {
      const size_t pp = (size_t)(k + 1 < NZ ? k + 1 : NZ - 1) * plane;
#pragma unroll
      for (int q = 0; q < 9; ++q) xp[q] = x[pp + cols[q]];
      T res = T(0);
      if (colfree && k >= kf && k <= kl) {
        const size_t cb = (size_t)k * plane + cpos;
        T s = f[(size_t)k * plane + cols[4]];
#pragma unroll
        for (int o = 0; o < 27; ++o) {
          const int dk = o / 9, q = o % 9;
          const T xv = dk == 0 ? xm[q] : (dk == 1 ? x0[q] : xp[q]);
          s -= st[(size_t)o * N + cb] * xv;
        }
        res = s;
      }
      r[(size_t)k * plane + cols[4]] = res;
      if (NORM) acc += (double)res * (double)res;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        xm[q] = x0[q];
        x0[q] = xp[q];
      }
    }
  }
  if (NORM) {
    s_red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) s_red[threadIdx.x] += s_red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = s_red[0];
  }
}

// ---------------------------------------------------------------- transfers

// rc = P^T r: coarse node (I,J,K) gathers the fine nodes of its support with
// weight 1 (the kept node) or 1/2 (a dropped neighbour), per direction.
template <class T>
__global__ __launch_bounds__(256) void restrict_kernel(const T* __restrict__ r, T* __restrict__ rc,
                                                       int NXf, int NYf, int NXc, int NYc, int NZc,
                                                       Faces fc, DirMapDev mx, DirMapDev my,
                                                       DirMapDev mz) {
  const int I = blockIdx.x * BX + (threadIdx.x % BX);
  const int J = blockIdx.y * BY + (threadIdx.x / BX);
  if (I >= NXc || J >= NYc) return;
  const size_t pf = (size_t)NXf * NYf, pc = (size_t)NXc * NYc;
  const bool colfree = !fc.x_fixed(I, NXc) && !fc.y_fixed(J, NYc);
  const int kf = fc.k_first(), kl = fc.k_last(NZc);
  const int xlo = mx.slo[I], xhi = mx.shi[I], xc = mx.ctr[I];
  const int ylo = my.slo[J], yhi = my.shi[J], yc = my.ctr[J];
  for (int K = 0; K < NZc; ++K) {
    T v = T(0);
    if (colfree && K >= kf && K <= kl) {
      const int zlo = mz.slo[K], zhi = mz.shi[K], zc = mz.ctr[K];
      for (int pz = zlo; pz <= zhi; ++pz) {
        const T wz = pz == zc ? T(1) : T(0.5);
        for (int py = ylo; py <= yhi; ++py) {
          const T wy = py == yc ? wz : T(0.5) * wz;
          const T* row = r + (size_t)pz * pf + (size_t)py * NXf;
          for (int px = xlo; px <= xhi; ++px) v += (px == xc ? wy : T(0.5) * wy) * row[px];
        }
      }
    }
    rc[(size_t)K * pc + (size_t)J * NXc + I] = v;
  }
}

// x += P e: fine node p interpolates from coarse lo[p] and hi[p] per direction.
template <class T>
__global__ __launch_bounds__(256) void prolong_kernel(const T* __restrict__ e, T* __restrict__ x,
                                                      int NXf, int NYf, int NZf, int NXc, int NYc,
                                                      Faces fc, DirMapDev mx, DirMapDev my,
                                                      DirMapDev mz, int tiles_x, int nblocks) {
  const int b = xcd_remap(blockIdx.x, nblocks);
  const int i = (b % tiles_x) * BX + (threadIdx.x % BX);
  const int j = (b / tiles_x) * BY + (threadIdx.x / BX);
  if (i >= NXf || j >= NYf) return;
  if (fc.x_fixed(i, NXf) || fc.y_fixed(j, NYf)) return;
  const size_t pf = (size_t)NXf * NYf, pc = (size_t)NXc * NYc;
  const int kf = fc.k_first(), kl = fc.k_last(NZf);
  const int xa = mx.lo[i], xb = mx.hi[i];
  const int ya = my.lo[j], yb = my.hi[j];
  const T wx = xa == xb ? T(1) : T(0.5), wxb = xa == xb ? T(0) : T(0.5);
  const T wy = ya == yb ? T(1) : T(0.5), wyb = ya == yb ? T(0) : T(0.5);
  for (int k = kf; k <= kl; ++k) {
    const int za = mz.lo[k], zb = mz.hi[k];
    const T wz = za == zb ? T(1) : T(0.5), wzb = za == zb ? T(0) : T(0.5);
    const T* pa = e + (size_t)za * pc;
    const T* pb = e + (size_t)zb * pc;
    auto plane_val = [&](const T* p) {
      return wy * (wx * p[(size_t)ya * NXc + xa] + wxb * p[(size_t)ya * NXc + xb]) +
             wyb * (wx * p[(size_t)yb * NXc + xa] + wxb * p[(size_t)yb * NXc + xb]);
    };
    x[(size_t)k * pf + (size_t)j * NXf + i] += wz * plane_val(pa) + wzb * plane_val(pb);
  }
}

// ---------------------------------------------------------------- Galerkin operator

// K_c(A, A+d) = sum_p sum_q P(p,A) K(p,q) P(q,A+d) over the supports of the
// two coarse nodes, restricted to |q - p| <= 1 per direction.
__global__ __launch_bounds__(256) void rap_kernel(const double* __restrict__ stf,
                                                  double* __restrict__ stc, int NXf, int NYf,
                                                  int NZf, int NXc, int NYc, int NZc, DirMapDev mx,
                                                  DirMapDev my, DirMapDev mz) {
  const size_t pc = (size_t)NXc * NYc, Nc = pc * NZc;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= Nc) return;
  const int I = (int)(gid % NXc), J = (int)((gid / NXc) % NYc), K = (int)(gid / pc);
  const size_t pf = (size_t)NXf * NYf, Nf = pf * NZf;
  const int NXef = (NXf + 1) >> 1, NXec = (NXc + 1) >> 1;
  const size_t outpos = (size_t)K * pc + (size_t)J * NXc + rowpos(I, NXec);
  for (int o = 0; o < 27; ++o) {
    const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
    const int Bx = I + dx, By = J + dy, Bz = K + dz;
    double acc = 0.0;
    if (Bx >= 0 && Bx < NXc && By >= 0 && By < NYc && Bz >= 0 && Bz < NZc) {
      for (int pz = mz.slo[K]; pz <= mz.shi[K]; ++pz) {
        const double wpz = pz == mz.ctr[K] ? 1.0 : 0.5;
        const int qz0 = max(mz.slo[Bz], pz - 1), qz1 = min(mz.shi[Bz], pz + 1);
        for (int qz = qz0; qz <= qz1; ++qz) {
          const double wz = wpz * (qz == mz.ctr[Bz] ? 1.0 : 0.5);
          for (int py = my.slo[J]; py <= my.shi[J]; ++py) {
            const double wpy = wz * (py == my.ctr[J] ? 1.0 : 0.5);
            const int qy0 = max(my.slo[By], py - 1), qy1 = min(my.shi[By], py + 1);
            for (int qy = qy0; qy <= qy1; ++qy) {
              const double wy = wpy * (qy == my.ctr[By] ? 1.0 : 0.5);
              for (int px = mx.slo[I]; px <= mx.shi[I]; ++px) {
                const double wpx = wy * (px == mx.ctr[I] ? 1.0 : 0.5);
                const size_t prow = (size_t)pz * pf + (size_t)py * NXf + rowpos(px, NXef);
                const int qx0 = max(mx.slo[Bx], px - 1), qx1 = min(mx.shi[Bx], px + 1);
                for (int qx = qx0; qx <= qx1; ++qx) {
                  const double w = wpx * (qx == mx.ctr[Bx] ? 1.0 : 0.5);
                  const int of = (qx - px + 1) + 3 * (qy - py + 1) + 9 * (qz - pz + 1);
                  acc += w * stf[(size_t)of * Nf + prow];
                }
              }
            }
          }
        }
      }
    }
    stc[(size_t)o * Nc + outpos] = acc;
  }
}

// FP32 copy of an FP64 stencil.  The off-diagonal entries are rounded, and
// the diagonal is set to minus their (rounded) sum, so that constants stay in
// the null space of the unconstrained FP32 operator as they are for K.
__global__ __launch_bounds__(256) void round_stencil_kernel(const double* __restrict__ s64,
                                                            float* __restrict__ s32, size_t N) {
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double sum = 0.0;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    if (o == 13) continue;
    const float v = (float)s64[(size_t)o * N + n];
    s32[(size_t)o * N + n] = v;
    sum += (double)v;
  }
  s32[(size_t)13 * N + n] = (float)(-sum);
}

template <class T>
__global__ __launch_bounds__(256) void unsplit_kernel(const T* __restrict__ s, T* __restrict__ out,
                                                      int NX, size_t rows) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t N = rows * NX;
  if (gid >= N * 27) return;
  const size_t o = gid / N, n = gid % N, row = n / NX;
  const int i = (int)(n % NX);
  out[gid] = s[o * N + row * NX + rowpos(i, (NX + 1) >> 1)];
}

// ---------------------------------------------------------------- coarsest level

// e[idx] = Kinv r[idx] for the free coarsest nodes (Kinv symmetric, so column
// `row` is read with consecutive threads on consecutive addresses).
template <class T>
__global__ __launch_bounds__(256) void coarse_solve_kernel(int n, const double* __restrict__ inv,
                                                           const int* __restrict__ idx,
                                                           const T* __restrict__ r,
                                                           T* __restrict__ e) {
  extern __shared__ double rs[];
  for (int t = threadIdx.x; t < n; t += blockDim.x) rs[t] = (double)r[idx[t]];
  __syncthreads();
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += inv[(size_t)j * n + row] * rs[j];
  e[idx[row]] = (T)s;
}

// ---------------------------------------------------------------- vectors

template <class T>
__global__ __launch_bounds__(256) void fill_kernel(T* __restrict__ p, size_t n, T v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(256) void scale_to_f32_kernel(const double* __restrict__ r,
                                                           double scale, float* __restrict__ r32,
                                                           size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    r32[i] = (float)(r[i] * scale);
}

__global__ __launch_bounds__(256) void update_lambda_kernel(const float* __restrict__ e,
                                                            double inv_scale,
                                                            double* __restrict__ lam, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    lam[i] += (double)e[i] * inv_scale;
}

__global__ __launch_bounds__(256) void axpy64_kernel(double alpha, const double* __restrict__ x,
                                                     double* __restrict__ y, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    y[i] += alpha * x[i];
}

__global__ __launch_bounds__(256) void zero_fixed_kernel(double* __restrict__ v, int NX, int NY,
                                                         int NZ, Faces fc) {
  const size_t plane = (size_t)NX * NY, N = plane * NZ;
  const int kf = fc.k_first(), kl = fc.k_last(NZ);
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / plane);
    if (fc.x_fixed(i, NX) || fc.y_fixed(j, NY) || k < kf || k > kl) v[n] = 0.0;
  }
}

// Deterministic final sum of per-block partials: thread t adds entries
// t, t+256, ... in order, then a fixed tree.
__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ partials,
                                                           size_t n_part, int width,
                                                           double* __restrict__ out) {
  __shared__ double s[256];
  for (int w = 0; w < width; ++w) {
    double a = 0.0;
    for (size_t i = threadIdx.x; i < n_part; i += 256) a += partials[(size_t)w * n_part + i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[w] = s[0];
    __syncthreads();
  }
}

unsigned grid_stride_blocks(size_t n) {
  const size_t b = (n + 255) / 256;
  return (unsigned)(b < 16384 ? (b == 0 ? 1 : b) : 16384);
}

struct ColGrid {
  int tiles_x, nblocks;
};

ColGrid col_grid(int ncx, int ncy) {
  ColGrid g;
  g.tiles_x = (ncx + BX - 1) / BX;
  g.nblocks = g.tiles_x * ((ncy + BY - 1) / BY);
  return g;
}

}  // namespace

// ---------------------------------------------------------------- launchers

template <class T>
void launch_smooth_sweep(const Dims& d, const Faces& fc, const T* st, const T* f, T* x,
                         hipStream_t s) {
  static const int order[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
  for (int c = 0; c < 4; ++c) {
    const int ci = order[c][0], cj = order[c][1];
    const int ncx = (d.NX() - ci + 1) / 2, ncy = (d.NY() - cj + 1) / 2;
    if (ncx <= 0 || ncy <= 0) continue;
    const ColGrid g = col_grid(ncx, ncy);
    gs_pass_kernel<T><<<g.nblocks, 256, 0, s>>>(st, f, x, d.NX(), d.NY(), d.NZ(), fc, ci, cj, ncx,
                                                ncy, g.tiles_x, g.nblocks);
    MCW_CHECK_LAUNCH();
  }
}

template <class T>
void launch_residual(const Dims& d, const Faces& fc, const T* st, const T* x, const T* f, T* r,
                     double* partials, size_t* n_part, hipStream_t s) {
  const ColGrid g = col_grid(d.NX(), d.NY());
  if (partials)
    residual_kernel<T, true><<<g.nblocks, 256, 0, s>>>(st, x, f, r, d.NX(), d.NY(), d.NZ(), fc,
                                                       g.tiles_x, g.nblocks, partials);
  else
    residual_kernel<T, false><<<g.nblocks, 256, 0, s>>>(st, x, f, r, d.NX(), d.NY(), d.NZ(), fc,
                                                        g.tiles_x, g.nblocks, nullptr);
  MCW_CHECK_LAUNCH();
  if (n_part) *n_part = g.nblocks;
}

template <class T>
void launch_restrict(const Dims& df, const Dims& dc, const Faces& fc, const DirMapDev& mx,
                     const DirMapDev& my, const DirMapDev& mz, const T* r, T* rc, hipStream_t s) {
  const dim3 g((dc.NX() + BX - 1) / BX, (dc.NY() + BY - 1) / BY);
  restrict_kernel<T><<<g, 256, 0, s>>>(r, rc, df.NX(), df.NY(), dc.NX(), dc.NY(), dc.NZ(), fc, mx,
                                       my, mz);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_prolong_dims(const Dims& df, const Dims& dc, const Faces& fc, const DirMapDev& mx,
                         const DirMapDev& my, const DirMapDev& mz, const T* e, T* x,
                         hipStream_t s) {
  const ColGrid g = col_grid(df.NX(), df.NY());
  prolong_kernel<T><<<g.nblocks, 256, 0, s>>>(e, x, df.NX(), df.NY(), df.NZ(), dc.NX(), dc.NY(),
                                              fc, mx, my, mz, g.tiles_x, g.nblocks);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_coarse_solve(int n, const double* inv, const int* idx, const T* r, T* e,
                         hipStream_t s) {
  const unsigned blocks = (unsigned)((n + 255) / 256);
  coarse_solve_kernel<T><<<blocks, 256, (size_t)n * sizeof(double), s>>>(n, inv, idx, r, e);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_fill(T* p, size_t n, T v, hipStream_t s) {
  if (n == 0) return;
  fill_kernel<T><<<grid_stride_blocks(n), 256, 0, s>>>(p, n, v);
  MCW_CHECK_LAUNCH();
}

void launch_rap(const Dims& df, const Dims& dc, const DirMapDev& mx, const DirMapDev& my,
                const DirMapDev& mz, const double* stf, double* stc, hipStream_t s) {
  const size_t Nc = dc.N();
  rap_kernel<<<(unsigned)((Nc + 255) / 256), 256, 0, s>>>(stf, stc, df.NX(), df.NY(), df.NZ(),
                                                          dc.NX(), dc.NY(), dc.NZ(), mx, my, mz);
  MCW_CHECK_LAUNCH();
}

void launch_round_stencil(const Dims& d, const double* st64, float* st32, hipStream_t s) {
  const size_t N = d.N();
  round_stencil_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(st64, st32, N);
  MCW_CHECK_LAUNCH();
}

void launch_unsplit_stencil(const Dims& d, const void* st, void* out, int is_double,
                            hipStream_t s) {
  const size_t rows = (size_t)d.NY() * d.NZ();
  const size_t tot = rows * d.NX() * 27;
  const unsigned blocks = (unsigned)((tot + 255) / 256);
  if (is_double)
    unsplit_kernel<double><<<blocks, 256, 0, s>>>(static_cast<const double*>(st),
                                                  static_cast<double*>(out), d.NX(), rows);
  else
    unsplit_kernel<float><<<blocks, 256, 0, s>>>(static_cast<const float*>(st),
                                                 static_cast<float*>(out), d.NX(), rows);
  MCW_CHECK_LAUNCH();
}

void launch_scale_to_f32(const Dims& d, const Faces& fc, const double* r, double scale, float* r32,
                         hipStream_t s) {
  (void)fc;
  const size_t N = d.N();
  scale_to_f32_kernel<<<grid_stride_blocks(N), 256, 0, s>>>(r, scale, r32, N);
  MCW_CHECK_LAUNCH();
}

void launch_update_lambda(size_t n, const float* e, double inv_scale, double* lam, hipStream_t s) {
  update_lambda_kernel<<<grid_stride_blocks(n), 256, 0, s>>>(e, inv_scale, lam, n);
  MCW_CHECK_LAUNCH();
}

void launch_axpy64(size_t n, double alpha, const double* x, double* y, hipStream_t s) {
  axpy64_kernel<<<grid_stride_blocks(n), 256, 0, s>>>(alpha, x, y, n);
  MCW_CHECK_LAUNCH();
}

void launch_zero_fixed(const Dims& d, const Faces& fc, double* v, hipStream_t s) {
  zero_fixed_kernel<<<grid_stride_blocks(d.N()), 256, 0, s>>>(v, d.NX(), d.NY(), d.NZ(), fc);
  MCW_CHECK_LAUNCH();
}

void launch_sum_partials(const double* partials, size_t n_part, int width, double* out,
                         hipStream_t s) {
  sum_partials_kernel<<<1, 256, 0, s>>>(partials, n_part, width, out);
  MCW_CHECK_LAUNCH();
}

#define MCW_INST(T)                                                                             \
  template void launch_smooth_sweep<T>(const Dims&, const Faces&, const T*, const T*, T*,       \
                                       hipStream_t);                                            \
  template void launch_residual<T>(const Dims&, const Faces&, const T*, const T*, const T*, T*, \
                                   double*, size_t*, hipStream_t);                              \
  template void launch_restrict<T>(const Dims&, const Dims&, const Faces&, const DirMapDev&,    \
                                   const DirMapDev&, const DirMapDev&, const T*, T*,            \
                                   hipStream_t);                                                \
  template void launch_prolong_dims<T>(const Dims&, const Dims&, const Faces&,                  \
                                       const DirMapDev&, const DirMapDev&, const DirMapDev&,    \
                                       const T*, T*, hipStream_t);                              \
  template void launch_coarse_solve<T>(int, const double*, const int*, const T*, T*,            \
                                       hipStream_t);                                            \
  template void launch_fill<T>(T*, size_t, T, hipStream_t);
MCW_INST(float)
MCW_INST(double)
#undef MCW_INST

}  // namespace mcw
