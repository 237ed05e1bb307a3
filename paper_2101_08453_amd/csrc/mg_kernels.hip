// Multigrid kernels on 27-point node stencils (Sec. 3 of Mandel et al.):
// Gauss-Seidel in vertical sweeps with the columns in four red-black groups,
// residual, restriction f_c = P^T r, prolongation u += P u_c, the Galerkin
// coarse operator K_c = P^T K P (eq. (7)), the coarsest direct solve, and the
// precision casts of the FP32-inside-FP64 refinement.
//
// Stencils use the grouped layout of StLayout / st_entry (mcw_internal.hpp);
// coefficient o = (di+1) + 3(dj+1) + 9(dk+1) of node (i,j,k) couples it to
// (i+di, j+dj, k+dk).  Entries towards nodes off the grid are exactly zero,
// so neighbour indices are clamped.  Caller-facing node vectors are in natural
// x-fastest order in memory; the V-cycle's level vectors (x, f, r) use the same
// row-split order as the stencils (even x indices of a row first, then the
// odd ones, no padding), so a colour pass reads and writes them contiguously.
//
// Every kernel is a device body run on one job's local block; the single
// launches run it on blockIdx, the batched launches (several independent
// problems in one persistent launch) walk a flattened (job, block) list.
#include <algorithm>

#include "mcw_internal.hpp"

namespace mcw {
namespace {

constexpr int BX = 64;  // columns per block along x (one wave)
constexpr int BY = 4;   // rows of columns per block

// Position of x index i inside its row in the row-split order of level vectors.
__device__ __forceinline__ int sx(int i, int NXe) { return (i & 1) ? NXe + (i >> 1) : (i >> 1); }

__device__ __forceinline__ StLayout dev_layout(int NX, int NY) {
  StLayout L;
  L.NY = NY;
  const int NXe = (NX + 1) >> 1;
  L.NXeP = (NXe + 63) & ~63;
  L.rowlen = L.NXeP + ((NX - NXe + 63) & ~63);
  return L;
}

// The SW stencil values of node p, read as 16-byte groups that lie 1 KB apart,
// with non-temporal loads: a pass streams each stencil value once, so it
// should not displace the x values that neighbouring columns reuse.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
// FP32: the 25 stored coefficients into a[o], the column coupling below a[4]
// from `below` (the o = 22 coefficient of the node below, 0 on the bottom
// plane), and the diagonal a[13] formed from them (the same values that
// mcw_get_stencil reports).
__device__ __forceinline__ void load_stencil_nt(const float* __restrict__ st, size_t p, float a[SW],
                                                float below) {
  const float* base = st + (p >> 6) * (size_t)(64 * SW32);
  const f32x4* v = reinterpret_cast<const f32x4*>(base) + (p & 63);
  float b[SW32];
#pragma unroll
  for (int g = 0; g < 6; ++g) {
    const f32x4 t = __builtin_nontemporal_load(v + g * 64);
    b[4 * g] = t.x; b[4 * g + 1] = t.y; b[4 * g + 2] = t.z; b[4 * g + 3] = t.w;
  }
  b[24] = __builtin_nontemporal_load(base + 1536 + (p & 63));
#pragma unroll
  for (int o = 0; o < 27; ++o)
    if (stored32(o)) a[o] = b[slot32(o)];
  a[4] = below;
  a[13] = stencil_diag(a);
}
// FP64: all 27 coefficients are stored; `below` is not used.
__device__ __forceinline__ void load_stencil_nt(const double* __restrict__ st, size_t p, double a[SW],
                                                double /*below*/) {
  const f64x2* v = reinterpret_cast<const f64x2*>(st) + (p >> 6) * (SW / 2) * 64 + (p & 63);
#pragma unroll
  for (int g = 0; g < SW / 2; ++g) {
    const f64x2 t = __builtin_nontemporal_load(v + g * 64);
    a[2 * g] = t.x; a[2 * g + 1] = t.y;
  }
}
template <class T>
__device__ __forceinline__ T load_nt(const T* p) { return __builtin_nontemporal_load(p); }

// FP16 stencils: the 25 stored scaled coefficients as FP32 into a[o], a[4]
// from `below` (scaled as well) and the diagonal formed from them, as for FP32
// stencils.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ void load_stencil_h16(const _Float16* __restrict__ st, size_t p, float a[SW],
                                                 float below) {
  const _Float16* base = st + (p >> 6) * (size_t)(64 * SW16);
  const f16x8* v = reinterpret_cast<const f16x8*>(base) + (p & 63);
  float b[SW16];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const f16x8 t = __builtin_nontemporal_load(v + g * 64);
#pragma unroll
    for (int e = 0; e < 8; ++e) b[8 * g + e] = (float)t[e];
  }
  b[24] = (float)__builtin_nontemporal_load(base + 1536 + (p & 63));
#pragma unroll
  for (int o = 0; o < 27; ++o)
    if (stored32(o)) a[o] = b[slot32(o)];
  a[4] = below;
  a[13] = stencil_diag(a);
}

// Stencil formats of a kernel instance: SF 0 holds T values (no scaling), SF 1
// FP16 values scaled by 1/sc.  Each launch, single or batched, runs the
// instance of its stencils' format, so an FP32 or FP64 kernel carries no FP16
// code (a format chosen per job at run time cost the batched FP32 kernels up
// to 40 registers per lane).  `below` is the o = 22 coefficient of the node
// under p, in the units of a (FP32 and FP16 formats; FP64 stores it).
template <class T, int SF>
__device__ __forceinline__ void load_stencil(const ColJob& J, size_t p, T a[SW], T below) {
  if constexpr (sizeof(T) == 4 && SF == 1)
    load_stencil_h16(static_cast<const _Float16*>(J.st), p, a, below);
  else
    load_stencil_nt(static_cast<const T*>(J.st), p, a, below);
}

// The o = 22 coefficient (the coupling to the node above) of node p, in the
// units load_stencil gives: what a column march that starts above p, or runs
// downwards, needs for the a[4] of the node above p.  Zero for FP64 stencils,
// which store a[4] themselves.
template <class T, int SF>
__device__ __forceinline__ T up_coupling(const ColJob& J, size_t p) {
  if constexpr (sizeof(T) == 8) {
    return T(0);
  } else if constexpr (SF == 1) {
    return (float)static_cast<const _Float16*>(J.st)[st_entry16(p, 22)];
  } else {
    return static_cast<const float*>(J.st)[st_entry<float>(p, 22)];
  }
}

// v times the job's scale factor s, except for format 0 (T stencils, s = 1).
// s is a power of two, so the product is exact; it must not be contracted into
// the FMA of the first stencil term, which would round that term's product on
// its own and make a batched FP32 member (s = 1) differ from a single launch.
template <int SF, class T>
__device__ __forceinline__ T scaled(T v, float s) {
#pragma clang fp contract(off)
  if constexpr (SF == 0) return v;
  else return v * (T)s;
}

// Job owning global work item g of a batched launch (prefix has njobs+1 entries).
__device__ __forceinline__ int find_job(const int* __restrict__ prefix, int njobs, int g) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}


// Run BODY(job, local block) over the work list W of a batched launch.
#define MCW_BATCHED_LOOP(JOBT, BODY)                                            \
  for (int g = blockIdx.x; g < W.total; g += gridDim.x) {                       \
    const int j = find_job(W.prefix, W.njobs, g);                               \
    if (!W.active[W.member[j]]) continue;                                       \
    const JOBT& J_ = static_cast<const JOBT*>(W.jobs)[j];                       \
    BODY(J_, g - W.prefix[j]);                                                  \
  }

// ---------------------------------------------------------------- smoother

// Pointwise Gauss-Seidel down one column (i, j) of the colour in J: bottom to
// top, or top to bottom for the reverse (adjoint) sweep.  Neighbour columns
// belong to other colours and are not changed meanwhile; the value below (or
// above) is this thread's own freshly updated one.
// r = f - K x of a whole column, zero: a fixed column, or one that a line
// solve has just made exact.
template <class T>
__device__ __forceinline__ void zero_column_r(const ColJob& J, int i, int j) {
  T* __restrict__ rl = static_cast<T*>(J.rlast);
  const size_t plane = (size_t)J.NX * J.NY;
  const int own = j * J.NX + sx(i, (J.NX + 1) >> 1);
  for (int k = 0; k < J.NZ; ++k) rl[(size_t)k * plane + own] = T(0);
}

// With J.rlast (forward passes of the last colour only) the column's residual
// is written as well.  Right after node k is solved its residual is zero up to
// rounding; of the later updates in the sweep only that of node k + 1 above it
// couples to it (neighbour columns are other colours, all done before), so its
// final residual is -a_k(above) (x_{k+1,new} - x_{k+1,old}), and the top free
// node's is zero.  The residual kernel then skips these columns.
//
// SIDE (the forward (1,1) pass that ends a sweep, run in the same launch as
// the (0,1) pass of its row): the only later changes to the residual of the
// (0,1) columns (i - 1, j) and (i + 1, j) beside this one are this column's
// own updates, on the planes k - 1, k, k + 1 around each of their nodes k.
// Their sums of a (x_new - x_old), with a this node's coupling to that
// neighbour (K is symmetric, so it is the neighbour's coupling to this node),
// in the stencil's units, go to row j - 1 of J.rside, which the launch does
// not otherwise use: the left neighbour's at column i - 1, the right one's at
// column i.  side_residual then finishes those columns' residual.
template <class T, bool REV, int SF = 0, bool SIDE = false>
__device__ __forceinline__ void gs_column(const ColJob& J, int i, int j) {
  const T* __restrict__ f = static_cast<const T*>(J.f);
  T* __restrict__ x = static_cast<T*>(J.x);
  const int NX = J.NX, NY = J.NY, NZ = J.NZ;
  T* __restrict__ rl = REV ? nullptr : static_cast<T*>(J.rlast);
  T* __restrict__ rs = (SIDE && !REV) ? static_cast<T*>(J.rside) : nullptr;
  if (J.fc.x_fixed(i, NX) || J.fc.y_fixed(j, NY)) {
    if (rl) zero_column_r<T>(J, i, j);
    return;
  }
  const int im = i > 0 ? i - 1 : i, ip = i < NX - 1 ? i + 1 : i;
  const int jm = j > 0 ? j - 1 : j, jp = j < NY - 1 ? j + 1 : j;
  const StLayout L = dev_layout(NX, NY);
  const int NXe = (NX + 1) >> 1;
  const int sm = sx(im, NXe), s0 = sx(i, NXe), sp = sx(ip, NXe);
  const int cols[9] = {jm * NX + sm, jm * NX + s0, jm * NX + sp, j * NX + sm, j * NX + s0,
                       j * NX + sp, jp * NX + sm, jp * NX + s0, jp * NX + sp};
  const size_t plane = (size_t)NX * NY;
  const int kf = J.fc.k_first(), kl = J.fc.k_last(NZ);
  if (rl) {
    for (int k = 0; k < kf; ++k) rl[(size_t)k * plane + cols[4]] = T(0);
    for (int k = kl; k < NZ; ++k) rl[(size_t)k * plane + cols[4]] = T(0);
  }
  T a_up = T(0);  // the coupling of the node below to this one
  // SIDE: row j - 1 slots of the side sums, and the sums still open for the
  // planes k - 1 and k (left, right)
  const int sl_at = (j - 1) * NX + sx(i - 1, NXe), sr_at = (j - 1) * NX + s0;
  T pl0 = T(0), pl1 = T(0), pr0 = T(0), pr1 = T(0);
  // the forward march carries the node below's upward coupling, the a[4] of
  // the next node (the bottom free node's comes from the plane under it)
  T below = (!REV && kf > 0) ? up_coupling<T, SF>(J, L.node(i, j, kf - 1)) : T(0);
  // rolling window of the 3 x 9 neighbour values: xl the plane already passed,
  // x0 the current plane, xn the plane ahead
  T xl[9], x0[9], xn[9];
  {
    const int k0 = REV ? kl : kf;
    const int kb = REV ? (kl + 1 < NZ ? kl + 1 : NZ - 1) : (kf > 0 ? kf - 1 : 0);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      xl[q] = x[(size_t)kb * plane + cols[q]];
      x0[q] = x[(size_t)k0 * plane + cols[q]];
    }
  }
  for (int t = 0; t <= kl - kf; ++t) {
    const int k = REV ? kl - t : kf + t;
    const int ka = REV ? (k > 0 ? k - 1 : 0) : (k + 1 < NZ ? k + 1 : NZ - 1);
#pragma unroll
    for (int q = 0; q < 9; ++q) xn[q] = x[(size_t)ka * plane + cols[q]];
    if (REV) below = k > 0 ? up_coupling<T, SF>(J, L.node(i, j, k - 1)) : T(0);
    T a[SW];
    load_stencil<T, SF>(J, L.node(i, j, k), a, below);
    below = a[22];
    T s = scaled<SF>(load_nt(f + (size_t)k * plane + cols[4]), J.isc);
#pragma unroll
    for (int o = 0; o < 27; ++o) {
      if (o == 13) continue;
      const int dk = o / 9, q = o % 9;
      // dk = 0 is the plane below, 2 the plane above
      const T* lo = REV ? xn : xl;
      const T* hi = REV ? xl : xn;
      const T xv = dk == 0 ? lo[q] : (dk == 1 ? x0[q] : hi[q]);
      s -= a[o] * xv;
    }
    const T xnew = s / a[13];
    if (!REV && rl) {
      if (t > 0) rl[(size_t)(k - 1) * plane + cols[4]] = scaled<SF>(-a_up * (xnew - x0[4]), J.sc);
      a_up = a[22];
    }
    if (SIDE && !REV) {
      // plane k - 1 is complete with this node's term (its couplings o = 3
      // and 5 reach the plane below); plane k + 1 opens with o = 21 and 23
      const T d = xnew - x0[4];
      pl0 += a[3] * d;
      pr0 += a[5] * d;
      if (t > 0) {
        rs[(size_t)(k - 1) * plane + sl_at] = pl0;
        rs[(size_t)(k - 1) * plane + sr_at] = pr0;
      }
      pl0 = pl1 + a[12] * d;
      pr0 = pr1 + a[14] * d;
      pl1 = a[21] * d;
      pr1 = a[23] * d;
    }
    x[(size_t)k * plane + cols[4]] = xnew;
    x0[4] = xnew;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      xl[q] = x0[q];
      x0[q] = xn[q];
    }
  }
  if (SIDE && !REV && kl >= kf) {
    // the top free plane's sums (the plane above it is fixed)
    rs[(size_t)kl * plane + sl_at] = pl0;
    rs[(size_t)kl * plane + sr_at] = pr0;
  }
}

// The residual of the (0,1) column (i, j) once the (1,1) pass of its row has
// run with SIDE: the term its own pass left in r (the update above each node,
// as for the last colour) minus the side sums the (1,1) columns beside it left
// in row j - 1, scaled to r's units.  A fixed column's r is zero already; a
// fixed or absent neighbour column changed nothing.
template <class T, int SF>
__device__ __forceinline__ void side_residual(const ColJob& J0, int i, int j) {
  const int NX = J0.NX, NY = J0.NY;
  if (J0.fc.x_fixed(i, NX) || J0.fc.y_fixed(j, NY)) return;
  T* __restrict__ r = static_cast<T*>(J0.rlast);
  const int NXe = (NX + 1) >> 1;
  const size_t plane = (size_t)NX * NY;
  const int own = j * NX + sx(i, NXe);
  const bool hl = i > 0 && !J0.fc.x_fixed(i - 1, NX);
  const bool hr = i + 1 < NX && !J0.fc.x_fixed(i + 1, NX);
  const int al = (j - 1) * NX + sx(i > 0 ? i - 1 : i, NXe), ar = (j - 1) * NX + sx(i, NXe);
  const int kf = J0.fc.k_first(), kl = J0.fc.k_last(J0.NZ);
  // eight planes at a time, their loads issued together (clamped to the top
  // free plane, so every load is in range and unconditional); an absent
  // neighbour's sum is taken as zero, which adds exactly nothing
  constexpr int CH = 8;
  for (int k0 = kf; k0 <= kl; k0 += CH) {
    T v[CH], sl[CH], sr[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const size_t o = (size_t)min(k0 + c, kl) * plane;
      v[c] = r[o + own];
      sl[c] = r[o + al];
      sr[c] = r[o + ar];
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (k0 + c > kl) break;
      const T side = (hl ? sl[c] : T(0)) + (hr ? sr[c] : T(0));
      r[(size_t)(k0 + c) * plane + own] = v[c] - scaled<SF>(side, J0.sc);
    }
  }
}

// Vertical line Gauss-Seidel on one column (i, j) of the colour in J: the
// column's free nodes are solved together with the neighbour columns (and the
// column's fixed end nodes) held at their current values.  The column block is
// tridiagonal in the couplings o = 4 (below), 13 (self), 22 (above); forward
// elimination from the bottom leaves the modified upper coefficients and the
// modified right-hand sides, back substitution from the top finishes x.  The
// solve is exact in the column, so a reverse sweep differs from a forward one
// only in the order of the colours.
// With LDS the thread keeps both sequences in its own LDS slots (ls, stride
// ls_stride; the c of free plane t at ls[t * stride], the right-hand side at
// ls[(np + t) * stride]) and writes x once; otherwise they go to J.r and x.
// The arithmetic is the same either way.
template <class T, int SF = 0, bool LDS = false>
__device__ __forceinline__ void line_column(const ColJob& J, int i, int j, T* ls = nullptr,
                                            int ls_stride = 0) {
  const T* __restrict__ f = static_cast<const T*>(J.f);
  T* __restrict__ x = static_cast<T*>(J.x);
  T* __restrict__ cb = static_cast<T*>(J.r);
  const int NX = J.NX, NY = J.NY, NZ = J.NZ;
  if (J.fc.x_fixed(i, NX) || J.fc.y_fixed(j, NY)) return;
  const int im = i > 0 ? i - 1 : i, ip = i < NX - 1 ? i + 1 : i;
  const int jm = j > 0 ? j - 1 : j, jp = j < NY - 1 ? j + 1 : j;
  const StLayout L = dev_layout(NX, NY);
  const int NXe = (NX + 1) >> 1;
  const int sm = sx(im, NXe), s0 = sx(i, NXe), sp = sx(ip, NXe);
  const int cols[9] = {jm * NX + sm, jm * NX + s0, jm * NX + sp, j * NX + sm, j * NX + s0,
                       j * NX + sp, jp * NX + sm, jp * NX + s0, jp * NX + sp};
  const size_t plane = (size_t)NX * NY;
  const int kf = J.fc.k_first(), kl = J.fc.k_last(NZ);
  if (kf > kl) return;
  T xb[9], x0[9], xa[9];  // planes k-1, k, k+1
  {
    const int kb = kf > 0 ? kf - 1 : 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      xb[q] = x[(size_t)kb * plane + cols[q]];
      x0[q] = x[(size_t)kf * plane + cols[q]];
    }
  }
  T cprev = T(0), dprev = T(0);
  T below = kf > 0 ? up_coupling<T, SF>(J, L.node(i, j, kf - 1)) : T(0);
  for (int k = kf; k <= kl; ++k) {
    const int ka = k + 1 < NZ ? k + 1 : NZ - 1;
#pragma unroll
    for (int q = 0; q < 9; ++q) xa[q] = x[(size_t)ka * plane + cols[q]];
    T a[SW];
    load_stencil<T, SF>(J, L.node(i, j, k), a, below);
    below = a[22];
    T s = scaled<SF>(load_nt(f + (size_t)k * plane + cols[4]), J.isc);
    const bool first = k == kf, last = k == kl;
#pragma unroll
    for (int o = 0; o < 27; ++o) {
      if (o == 13) continue;
      // the couplings to the column's own free nodes stay on the left-hand side
      if (o == 4 && !first) continue;
      if (o == 22 && !last) continue;
      const int dk = o / 9, q = o % 9;
      const T xv = dk == 0 ? xb[q] : (dk == 1 ? x0[q] : xa[q]);
      s -= a[o] * xv;
    }
    const T sub = first ? T(0) : a[4];
    const T sup = last ? T(0) : a[22];
    const T den = a[13] - sub * cprev;
    const T c = sup / den;
    const T d = (s - sub * dprev) / den;
    if constexpr (LDS) {
      ls[(k - kf) * ls_stride] = c;
      ls[(kl - kf + 1 + k - kf) * ls_stride] = d;
    } else {
      cb[(size_t)k * plane + cols[4]] = c;
      x[(size_t)k * plane + cols[4]] = d;
    }
    cprev = c;
    dprev = d;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      xb[q] = x0[q];
      x0[q] = xa[q];
    }
  }
  T xnext = dprev;  // x at kl is its modified right-hand side
  if constexpr (LDS) {
    const int np = kl - kf + 1;
    x[(size_t)kl * plane + cols[4]] = xnext;
    for (int k = kl - 1; k >= kf; --k) {
      xnext = ls[(np + k - kf) * ls_stride] - ls[(k - kf) * ls_stride] * xnext;
      x[(size_t)k * plane + cols[4]] = xnext;
    }
  } else {
    for (int k = kl - 1; k >= kf; --k) {
      const size_t p = (size_t)k * plane + cols[4];
      xnext = x[p] - cb[p] * xnext;
      x[p] = xnext;
    }
  }
}

template <class T, bool REV, bool LINE, int SF = 0, bool LDS = false>
__device__ __forceinline__ void smooth_column(const ColJob& J, int i, int j, T* ls = nullptr) {
  if constexpr (LINE) {
    line_column<T, SF, LDS>(J, i, j, ls, (int)blockDim.x);
    if (J.rlast) zero_column_r<T>(J, i, j);
  } else {
    gs_column<T, REV, SF>(J, i, j);
  }
}

// One colour pass: a thread per column (i, j) with i = ci mod 2, j = cj mod 2,
// tiles of 64 x J.by columns per block.
template <class T, bool REV, bool LINE, int SF, bool LDS = false, bool SIDE = false>
__device__ __forceinline__ void gs_pass_body(const ColJob& J, int b, T* ls = nullptr) {
  const int ii = (b % J.tiles_x) * BX + (threadIdx.x % BX);
  const int jj = (b / J.tiles_x) * J.by + (threadIdx.x / BX);
  if (ii >= J.ncx || jj >= J.ncy) return;
  if constexpr (SIDE && !LINE && !REV)
    gs_column<T, false, SF, true>(J, 2 * ii + J.ci, 2 * jj + J.cj);
  else
    smooth_column<T, REV, LINE, SF, LDS>(J, 2 * ii + J.ci, 2 * jj + J.cj, ls);
}

// side_residual over the (0,1) columns of a one-colour job's tiles, after the
// (1,1) pass with SIDE (the one-colour form of the SIDE fused pass)
template <class T, int SF>
__device__ __forceinline__ void side_pass_body(const ColJob& J, int b) {
  const int ii = (b % J.tiles_x) * BX + (threadIdx.x % BX);
  const int jj = (b / J.tiles_x) * J.by + (threadIdx.x / BX);
  if (ii >= J.ncx || jj >= J.ncy) return;
  side_residual<T, SF>(J, 2 * ii + J.ci, 2 * jj + J.cj);
}

// Dynamic LDS of the line smoother: 2 values per free plane for each thread.
extern __shared__ __align__(16) unsigned char mcw_dyn_lds[];
template <class T, bool LDS>
__device__ __forceinline__ T* line_slots() {
  if constexpr (LDS) return reinterpret_cast<T*>(mcw_dyn_lds) + threadIdx.x;
  else return nullptr;
}

// Two colour passes of the same rows in one launch: colour J0 then colour J1
// on every row j = cj mod 2, one block per row.  The J1 columns of a row couple
// only to the J0 columns of the same row (and to untouched rows j +- 1), so a
// block barrier between the two halves keeps the order of the separate passes
// and gives the same result bit for bit, with one launch instead of two.
// Each XCD takes a contiguous range of rows, so that the blocks of rows j and
// j + 2 running there at the same time share row j + 1 in its L2.
// Threads per block: 1024 for the pointwise smoother, 512 for the line
// smoother, whose column solve keeps 2 values per free plane and thread in
// LDS (60 KB for 15 planes in FP32; the FP64 Thomas sweep also needs more
// than the 128 registers a 1024-thread block leaves per lane).
// The FP64 pass that also leaves the side sums (SIDE) takes 512 as well: with
// 1024 threads it would spill more of its 128 registers per lane.
template <class T, bool LINE, bool SIDE = false>
constexpr int fused_threads() { return LINE || (SIDE && sizeof(T) == 8) ? 512 : 1024; }

// SIDE (forward point smoother, odd rows, the last pre-smoothing sweep): J0,
// colour (0,1), and J1, colour (1,1), both write r; after a second barrier
// the (0,1) columns' residual is finished from J1's side sums.
template <class T, bool REV, bool LINE, int SF, bool LDS = false, bool SIDE = false>
__global__ __launch_bounds__((fused_threads<T, LINE, SIDE>())) void gs_fused_kernel(ColJob J0, ColJob J1) {
  const int j = 2 * xcd_remap(blockIdx.x, gridDim.x) + J0.cj;
  T* ls = line_slots<T, LDS>();
  for (int ii = threadIdx.x; ii < J0.ncx; ii += blockDim.x)
    smooth_column<T, REV, LINE, SF, LDS>(J0, 2 * ii + J0.ci, j, ls);
  __syncthreads();
  if constexpr (SIDE) {
    for (int ii = threadIdx.x; ii < J1.ncx; ii += blockDim.x)
      gs_column<T, false, SF, true>(J1, 2 * ii + J1.ci, j);
    __syncthreads();
    for (int ii = threadIdx.x; ii < J0.ncx; ii += blockDim.x)
      side_residual<T, SF>(J0, 2 * ii + J0.ci, j);
  } else {
    for (int ii = threadIdx.x; ii < J1.ncx; ii += blockDim.x)
      smooth_column<T, REV, LINE, SF, LDS>(J1, 2 * ii + J1.ci, j, ls);
  }
}

template <class T, bool REV, bool LINE, int SF, bool LDS = false, bool SIDE = false>
__global__ __launch_bounds__(256) void gs_pass_kernel(ColJob J) {
  gs_pass_body<T, REV, LINE, SF, LDS, SIDE>(J, xcd_remap(blockIdx.x, J.nblocks), line_slots<T, LDS>());
}

template <class T, int SF>
__global__ __launch_bounds__(256) void side_residual_kernel(ColJob J) {
  side_pass_body<T, SF>(J, xcd_remap(blockIdx.x, J.nblocks));
}

template <class T, int SF, bool SIDE = false>
__device__ __forceinline__ void gs_pass_fwd(const ColJob& J, int b) {
  gs_pass_body<T, false, false, SF, false, SIDE>(J, b);
}
template <class T, int SF>
__device__ __forceinline__ void gs_pass_rev(const ColJob& J, int b) { gs_pass_body<T, true, false, SF>(J, b); }

template <class T, int SF, bool SIDE = false>
__global__ __launch_bounds__(256) void gs_pass_batched(WorkList W) {
  MCW_BATCHED_LOOP(ColJob, (gs_pass_fwd<T, SF, SIDE>))
}

template <class T, int SF>
__global__ __launch_bounds__(256) void side_residual_batched(WorkList W) {
  MCW_BATCHED_LOOP(ColJob, (side_pass_body<T, SF>))
}

template <class T, int SF>
__global__ __launch_bounds__(256) void gs_pass_batched_rev(WorkList W) {
  MCW_BATCHED_LOOP(ColJob, (gs_pass_rev<T, SF>))
}

// Batched two-colour pass: work item b of a job is row 2b + cj, run as
// gs_fused_kernel runs a row (colour J0, block barrier, colour J1), with
// blocks of 256 threads looping over the row's columns.  Every thread of a
// block walks the same work items, so the barrier is reached uniformly.
// With SIDE, as gs_fused_kernel with SIDE (a second barrier per work item).
template <class T, bool REV, int SF, bool SIDE = false>
__device__ __forceinline__ void gs_fused_item(const FusedJob& F, int b) {
  const int j = 2 * b + F.J0.cj;
  for (int ii = threadIdx.x; ii < F.J0.ncx; ii += blockDim.x)
    gs_column<T, REV, SF>(F.J0, 2 * ii + F.J0.ci, j);
  __syncthreads();
  for (int ii = threadIdx.x; ii < F.J1.ncx; ii += blockDim.x)
    gs_column<T, REV, SF, SIDE>(F.J1, 2 * ii + F.J1.ci, j);
  if constexpr (SIDE) {
    __syncthreads();
    for (int ii = threadIdx.x; ii < F.J0.ncx; ii += blockDim.x)
      side_residual<T, SF>(F.J0, 2 * ii + F.J0.ci, j);
  }
}

template <class T, bool REV, int SF, bool SIDE = false>
__global__ __launch_bounds__(256) void gs_fused_batched(WorkList W) {
  MCW_BATCHED_LOOP(FusedJob, (gs_fused_item<T, REV, SF, SIDE>))
}

// ---------------------------------------------------------------- residual

// r = f - K x at free nodes (f null: r = -K x), 0 at fixed nodes; returns this
// thread's sum of r^2, or of x r with DOTX.
template <class T, bool DOTX = false, int SF = 0>
__device__ __forceinline__ double residual_body(const ColJob& J, int b) {
  const T* __restrict__ x = static_cast<const T*>(J.x);
  const T* __restrict__ f = static_cast<const T*>(J.f);
  T* __restrict__ r = static_cast<T*>(J.r);
  const int NX = J.NX, NY = J.NY, NZ = J.NZ;
  // lanes follow the row-split order, so f, r and the stencil are read contiguously
  const int qx = (b % J.tiles_x) * BX + (threadIdx.x % BX);
  const int jr = (b / J.tiles_x) * J.by + (threadIdx.x / BX);
  const int j = J.skip11 == 2 ? 2 * jr : jr;  // 2: the even rows only
  double acc = 0.0;
  if (qx >= NX || j >= NY) return acc;
  const size_t plane = (size_t)NX * NY;
  const int NXe = (NX + 1) >> 1;
  const int i = qx < NXe ? 2 * qx : 2 * (qx - NXe) + 1;
  const int own = j * NX + qx;
  if (J.skip11 == 1 && (i & j & 1)) return acc;  // written by the sweep's last colour pass
  if (J.fc.x_fixed(i, NX) || J.fc.y_fixed(j, NY)) {
    for (int k = 0; k < NZ; ++k) r[(size_t)k * plane + own] = T(0);
    return acc;
  }
  const int kf = J.fc.k_first(), kl = J.fc.k_last(NZ);
  const int im = i > 0 ? i - 1 : i, ip = i < NX - 1 ? i + 1 : i;
  const int jm = j > 0 ? j - 1 : j, jp = j < NY - 1 ? j + 1 : j;
  const StLayout L = dev_layout(NX, NY);
  const int sm = sx(im, NXe), sp = sx(ip, NXe);
  const int cols[9] = {jm * NX + sm, jm * NX + sx(i, NXe), jm * NX + sp, j * NX + sm, own,
                       j * NX + sp, jp * NX + sm, jp * NX + sx(i, NXe), jp * NX + sp};
  T xm[9], x0[9], xp[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    xm[q] = x[cols[q]];
    x0[q] = xm[q];
  }
  // every k is computed (all loads are in range) so that the loads of a plane
  // are issued together; rows of fixed planes are then set to zero
  T below = T(0);  // the node below's upward coupling: a[4] of plane k
  for (int k = 0; k < NZ; ++k) {
    const size_t pp = (size_t)(k + 1 < NZ ? k + 1 : NZ - 1) * plane;
#pragma unroll
    for (int q = 0; q < 9; ++q) xp[q] = x[pp + cols[q]];
    T a[SW];
    load_stencil<T, SF>(J, L.node(i, j, k), a, below);
    below = a[22];
    T s = f ? scaled<SF>(load_nt(f + (size_t)k * plane + own), J.isc) : T(0);
#pragma unroll
    for (int o = 0; o < 27; ++o) {
      const int dk = o / 9, q = o % 9;
      const T xv = dk == 0 ? xm[q] : (dk == 1 ? x0[q] : xp[q]);
      s -= a[o] * xv;
    }
    const T res = (k >= kf && k <= kl) ? scaled<SF>(s, J.sc) : T(0);
    r[(size_t)k * plane + own] = res;
    acc += (double)(DOTX ? x0[4] : res) * (double)res;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      xm[q] = x0[q];
      x0[q] = xp[q];
    }
  }
  return acc;
}

template <class T, bool NORM, bool DOTX, int SF>
__global__ __launch_bounds__(256) void residual_kernel(ColJob J, double* __restrict__ partials) {
  __shared__ double s_red[256];
  const double acc = residual_body<T, DOTX, SF>(J, xcd_remap(blockIdx.x, J.nblocks));
  if (NORM) {
    block_sum_to(acc, s_red, &partials[blockIdx.x]);
  }
}

template <class T, int SF>
__device__ __forceinline__ void residual_nonorm(const ColJob& J, int b) { (void)residual_body<T, false, SF>(J, b); }

// q = -K p with p.q per block, as residual_kernel<T, true, true, SF> does for block b
template <class T, int SF>
__device__ __forceinline__ void residual_dot_item(const ColJob& J, int b) {
  __shared__ double s_red[256];
  const double acc = residual_body<T, true, SF>(J, xcd_remap(b, J.nblocks));
  block_sum_to(acc, s_red, &J.part[b]);
}

template <class T, int SF>
__global__ __launch_bounds__(256) void residual_dot_batched(WorkList W) {
  MCW_BATCHED_LOOP(ColJob, (residual_dot_item<T, SF>))
}

template <class T, int SF>
__global__ __launch_bounds__(256) void residual_batched(WorkList W) {
  MCW_BATCHED_LOOP(ColJob, (residual_nonorm<T, SF>))
}

// ---------------------------------------------------------------- transfers

// rc = P^T r: coarse node (I,J,K) gathers the fine nodes of its support with
// weight 1 (the kept node) or 1/2 (a dropped neighbour), per direction.  A
// thread marches up the fine planes under one coarse column, loading two
// planes ahead: each fine plane's horizontal sum is formed once and added to
// the (at most two) coarse planes whose support holds it, in the order of the
// fine planes, so every coarse value is the same sum as a direct gather.
template <class T, bool HC>
__device__ __forceinline__ void restrict_column(const XferJob& X, int b) {
  const T* __restrict__ r = static_cast<const T*>(X.src);
  T* __restrict__ rc = static_cast<T*>(X.dst);
  const int I = (b % X.tiles_x) * BX + (threadIdx.x % BX);
  const int J = (b / X.tiles_x) * BY + (threadIdx.x / BX);
  if (I >= X.NXc || J >= X.NYc) return;
  const size_t pf = (size_t)X.NXf * X.NYf, pc = (size_t)X.NXc * X.NYc;
  const int NXef = (X.NXf + 1) >> 1, NXec = (X.NXc + 1) >> 1;
  T* __restrict__ out = rc + (size_t)J * X.NXc + sx(I, NXec);
  const int kf = X.fc.k_first(), kl = X.fc.k_last(X.NZc);
  const bool colfree = !X.fc.x_fixed(I, X.NXc) && !X.fc.y_fixed(J, X.NYc);
  if (!colfree || kf > kl) {
    for (int K = 0; K < X.NZc; ++K) out[(size_t)K * pc] = T(0);
    return;
  }
  for (int K = 0; K < kf; ++K) out[(size_t)K * pc] = T(0);
  for (int K = kl + 1; K < X.NZc; ++K) out[(size_t)K * pc] = T(0);
  // the horizontal support (HC: the directions are coarsened): the kept index
  // and its dropped neighbours, an absent neighbour repeating the kept index
  // with weight 0; without horizontal coarsening, the node itself
  constexpr int S = HC ? 9 : 1;
  const int xc = X.mx.ctr[I], xlo = X.mx.slo[I], xhi = X.mx.shi[I];
  const int yc = X.my.ctr[J], ylo = X.my.slo[J], yhi = X.my.shi[J];
  const T wx[3] = {xlo < xc ? T(0.5) : T(0), T(1), xhi > xc ? T(0.5) : T(0)};
  const T wy[3] = {ylo < yc ? T(0.5) : T(0), T(1), yhi > yc ? T(0.5) : T(0)};
  size_t off[S];
  if (HC) {
    const int ox[3] = {sx(xlo, NXef), sx(xc, NXef), sx(xhi, NXef)};
    const int oy[3] = {ylo, yc, yhi};
#pragma unroll
    for (int a = 0; a < S / 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) off[3 * a + c] = (size_t)oy[a] * X.NXf + ox[c];
  } else {
    off[0] = (size_t)J * X.NXf + sx(I, NXef);
  }
  auto load_plane = [&](int pz, T (&v)[S]) {
    const T* __restrict__ pl = r + (size_t)pz * pf;
#pragma unroll
    for (int q = 0; q < S; ++q) v[q] = pl[off[q]];
  };
  auto plane_sum = [&](const T (&v)[S]) {
    if (!HC) return v[0];
    T h = T(0);
#pragma unroll
    for (int a = 0; a < S / 3; ++a) {
      T row = T(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) row += wx[c] * v[3 * a + c];
      h += wy[a] * row;
    }
    return h;
  };
  // fine planes of the free coarse planes' supports.  Plane pz + 2 is loaded
  // while plane pz is summed (clamped to the last plane, so that every load is
  // issued unconditionally and stays in flight); the three buffers rotate by
  // unrolling, not by copies, which would wait for the loads.
  const int p0 = X.mz.slo[kf], p1 = X.mz.shi[kl];
  T acc = T(0);
  auto step = [&](int pz, const T (&cur)[S], T (&ahead)[S]) {
    load_plane(min(pz + 2, p1), ahead);
    const T h = plane_sum(cur);
    const int Klo = X.mz.lo[pz], Khi = X.mz.hi[pz];
    if (Klo == Khi) {
      // kept plane of Klo, weight 1; Klo is complete unless a dropped plane follows
      acc += T(1) * h;
      if (X.mz.shi[Klo] == pz) {
        out[(size_t)Klo * pc] = acc;
        acc = T(0);
      }
    } else {
      // dropped plane between Klo and Khi = Klo + 1, weight 1/2 to each: it
      // ends the support of Klo and starts that of Khi
      acc += T(0.5) * h;
      out[(size_t)Klo * pc] = Klo >= kf ? acc : T(0);
      acc = T(0);
      acc += T(0.5) * h;
    }
  };
  T b0[S], b1[S], b2[S];
  load_plane(p0, b0);
  load_plane(min(p0 + 1, p1), b1);
  for (int pz = p0;; pz += 3) {
    step(pz, b0, b2);
    if (pz + 1 > p1) break;
    step(pz + 1, b1, b0);
    if (pz + 2 > p1) break;
    step(pz + 2, b2, b1);
    if (pz + 3 > p1) break;
  }
}

template <class T>
__device__ __forceinline__ void restrict_body(const XferJob& X, int b) {
  if (X.NXc != X.NXf) restrict_column<T, true>(X, b);
  else restrict_column<T, false>(X, b);
}

template <class T>
__global__ __launch_bounds__(256) void restrict_kernel(XferJob X) {
  restrict_body<T>(X, xcd_remap(blockIdx.x, X.nblocks));
}

template <class T>
__global__ __launch_bounds__(256) void restrict_batched(WorkList W) {
  MCW_BATCHED_LOOP(XferJob, restrict_body<T>)
}

// x += P e: fine node p interpolates from coarse lo[p] and hi[p] per direction.
//
// Column version (every level in the batched launch; levels that keep every
// horizontal node in the single-grid launch): a thread updates one fine column;
// the last two coarse values are kept, as consecutive fine planes share them.
template <class T>
__device__ __forceinline__ void prolong_body(const XferJob& X, int b) {
  const T* __restrict__ e = static_cast<const T*>(X.src);
  T* __restrict__ x = static_cast<T*>(X.dst);
  // lanes follow the row-split order of x, so the updates of a wave are contiguous
  const int q = (b % X.tiles_x) * BX + (threadIdx.x % BX);
  const int j = (b / X.tiles_x) * BY + (threadIdx.x / BX);
  if (q >= X.NXf || j >= X.NYf) return;
  const int NXef = (X.NXf + 1) >> 1, NXec = (X.NXc + 1) >> 1;
  const int i = q < NXef ? 2 * q : 2 * (q - NXef) + 1;
  if (X.fc.x_fixed(i, X.NXf) || X.fc.y_fixed(j, X.NYf)) return;
  const size_t pf = (size_t)X.NXf * X.NYf, pc = (size_t)X.NXc * X.NYc;
  const int kf = X.fc.k_first(), kl = X.fc.k_last(X.NZf);
  const int xa = sx(X.mx.lo[i], NXec), xb = sx(X.mx.hi[i], NXec);
  const int ya = X.my.lo[j], yb = X.my.hi[j];
  const int NXc = X.NXc;
  // a kept index reads one coarse value, a dropped one the mean of two; the
  // conditions are uniform over a wave (one half-row) or the whole launch
  // (planes), so each node loads only the coarse values it weighs
  auto row_val = [&](const T* row) { return xa == xb ? row[xa] : T(0.5) * (row[xa] + row[xb]); };
  auto plane_val = [&](const T* p) {
    const T va = row_val(p + (size_t)ya * NXc);
    return ya == yb ? va : T(0.5) * (va + row_val(p + (size_t)yb * NXc));
  };
  // consecutive fine planes share coarse planes: keep the last two values
  int c0 = -1, c1 = -1;
  T v0 = T(0), v1 = T(0);
  auto coarse_plane = [&](int z) {
    if (z == c1) return v1;
    if (z == c0) return v0;
    const T v = plane_val(e + (size_t)z * pc);
    c0 = c1;
    v0 = v1;
    c1 = z;
    v1 = v;
    return v;
  };
  for (int k = kf; k <= kl; ++k) {
    const int za = X.mz.lo[k], zb = X.mz.hi[k];
    const T va = coarse_plane(za);
    const T v = za == zb ? va : T(0.5) * (va + coarse_plane(zb));
    x[(size_t)k * pf + (size_t)j * X.NXf + q] += v;
  }
}

template <class T>
__global__ __launch_bounds__(256) void prolong_kernel(XferJob X) {
  prolong_body<T>(X, xcd_remap(blockIdx.x, X.nblocks));
}

// Single-grid prolongation on horizontally coarsened levels (every other node
// kept in x and y).  A thread owns the fine columns (2q, 2q+1) x (2J, 2J+1)
// around coarse column (q, J); they interpolate from the coarse columns
// (q, q+1) x (J, J+1) only, each loaded once per coarse plane instead of once
// per fine column.  The column is updated D fine planes at a time: the chunk's
// coarse planes (a uniform count, at most D+1) and the x of its planes are all
// loaded before the first is used.  A kept index takes the same coarse value
// twice and 0.5 (v + v) = v exactly, so every mean is formed as in the column
// version (x, then y, then z, low index first) and the result is the same to
// the bit.  The job's tiles cover the coarse columns.  (The body is written in
// the kernel itself: through a device function taking the job by reference the
// compiler lowers the choice of coarse planes with per-lane index chains and
// needs half again as many registers.)
template <class T, int D>
__global__ __launch_bounds__(256) void prolong_pairs_kernel(XferJob X) {
  const int b = xcd_remap(blockIdx.x, X.nblocks);
  const T* __restrict__ e = static_cast<const T*>(X.src);
  T* __restrict__ x = static_cast<T*>(X.dst);
  const int qc = (b % X.tiles_x) * BX + (threadIdx.x % BX);
  const int Jc = (b / X.tiles_x) * BY + (threadIdx.x / BX);
  if (qc >= X.NXc || Jc >= X.NYc) return;
  const int kf = X.fc.k_first(), kl = X.fc.k_last(X.NZf);
  if (kf > kl) return;
  const size_t pf = (size_t)X.NXf * X.NYf, pc = (size_t)X.NXc * X.NYc;
  const int NXef = (X.NXf + 1) >> 1, NXec = (X.NXc + 1) >> 1;
  // fine column c = 2w + u is (2q+u, 2J+w): whether it exists and is free, and
  // its row-split offset in a plane
  bool act[4];
  size_t fo[4];
  // per fine x index 2q+u (y index 2J+w): 2 for the mean of coarse q and q+1,
  // else which of the two it is (the last fine node is kept even when odd)
  int cx[2], cy[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = 2 * qc + u;
    const bool in = i < X.NXf;
    const int lo = in ? X.mx.lo[i] : qc, hi = in ? X.mx.hi[i] : qc;
    cx[u] = lo != hi ? 2 : (lo == qc ? 0 : 1);
  }
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const int j = 2 * Jc + w;
    const bool in = j < X.NYf;
    const int lo = in ? X.my.lo[j] : Jc, hi = in ? X.my.hi[j] : Jc;
    cy[w] = lo != hi ? 2 : (lo == Jc ? 0 : 1);
  }
#pragma unroll
  for (int w = 0; w < 2; ++w)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = 2 * qc + u, j = 2 * Jc + w;
      act[2 * w + u] = i < X.NXf && j < X.NYf && !X.fc.x_fixed(i, X.NXf) && !X.fc.y_fixed(j, X.NYf);
      fo[2 * w + u] = act[2 * w + u] ? (size_t)j * X.NXf + sx(i, NXef) : 0;
    }
  // coarse columns (q, J), (q+1, J), (q, J+1), (q+1, J+1), clamped to the grid
  const int q1 = min(qc + 1, X.NXc - 1), J1 = min(Jc + 1, X.NYc - 1);
  const size_t co[4] = {(size_t)Jc * X.NXc + sx(qc, NXec), (size_t)Jc * X.NXc + sx(q1, NXec),
                        (size_t)J1 * X.NXc + sx(qc, NXec), (size_t)J1 * X.NXc + sx(q1, NXec)};
  // the four fine columns' values v on one coarse plane from its 2 x 2 values c
  auto horizontal = [&](const T (&c)[4], T (&v)[4]) {
    T row[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        row[r][u] = cx[u] == 2 ? T(0.5) * (c[2 * r] + c[2 * r + 1]) : c[2 * r + cx[u]];
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        v[2 * w + u] = cy[w] == 2 ? T(0.5) * (row[0][u] + row[1][u]) : row[cy[w]][u];
  };
  constexpr int M = D + 1;
  for (int k0 = kf; k0 <= kl; k0 += D) {
    const int z0 = X.mz.lo[k0], z1 = X.mz.hi[min(k0 + D - 1, kl)];
    T cv[M][4], xv[D][4];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (z0 + m <= z1) {
        const T* __restrict__ p = e + (size_t)(z0 + m) * pc;
#pragma unroll
        for (int c = 0; c < 4; ++c) cv[m][c] = p[co[c]];
      }
    }
#pragma unroll
    for (int t = 0; t < D; ++t) {
      if (k0 + t <= kl) {
        const T* __restrict__ p = x + (size_t)(k0 + t) * pf;
#pragma unroll
        for (int c = 0; c < 4; ++c) xv[t][c] = p[fo[c]];
      }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (z0 + m <= z1) {
        T v[4];
        horizontal(cv[m], v);
#pragma unroll
        for (int c = 0; c < 4; ++c) cv[m][c] = v[c];
      }
    }
#pragma unroll
    for (int t = 0; t < D; ++t) {
      const int k = k0 + t;
      if (k <= kl) {
        // fine plane k between coarse planes lo[k] and hi[k] (equal when kept)
        const int da = X.mz.lo[k] - z0, db = X.mz.hi[k] - z0;
        T* __restrict__ p = x + (size_t)k * pf;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          T va = cv[0][c], vb = cv[0][c];
#pragma unroll
          for (int m = 1; m < M; ++m) {
            va = da == m ? cv[m][c] : va;
            vb = db == m ? cv[m][c] : vb;
          }
          if (act[c]) p[fo[c]] = xv[t][c] + (da == db ? va : T(0.5) * (va + vb));
        }
      }
    }
  }
}

template <class T>
__global__ __launch_bounds__(256) void prolong_batched(WorkList W) {
  MCW_BATCHED_LOOP(XferJob, prolong_body<T>)
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
  const StLayout Lf = dev_layout(NXf, NYf), Lc = dev_layout(NXc, NYc);
  const size_t outpos = Lc.node(I, J, K);
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
                const size_t prow = Lf.node(px, py, pz);
                const int qx0 = max(mx.slo[Bx], px - 1), qx1 = min(mx.shi[Bx], px + 1);
                for (int qx = qx0; qx <= qx1; ++qx) {
                  const double w = wpx * (qx == mx.ctr[Bx] ? 1.0 : 0.5);
                  const int of = (qx - px + 1) + 3 * (qy - py + 1) + 9 * (qz - pz + 1);
                  acc += w * stf[st_entry<double>(prow, of)];
                }
              }
            }
          }
        }
      }
    }
    stc[st_entry<double>(outpos, o)] = acc;
  }
  stc[st_entry<double>(outpos, 27)] = 0.0;
}

// FP32 copy of an FP64 stencil: the stored off-diagonal entries (all but the
// coupling to the node below, which is the node below's upward one) rounded
// once.  The kernels form the diagonal as minus the sum of the off-diagonals,
// so that constants stay in the null space of the unconstrained FP32 operator
// as they are for K.
__global__ __launch_bounds__(256) void round_stencil_kernel(const double* __restrict__ s64,
                                                            float* __restrict__ s32, int NX, int NY,
                                                            size_t N) {
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const StLayout L = dev_layout(NX, NY);
  const size_t p = L.node((int)(n % NX), (int)((n / NX) % NY), (int)(n / ((size_t)NX * NY)));
#pragma unroll
  for (int o = 0; o < 27; ++o)
    if (stored32(o)) s32[st_entry<float>(p, o)] = (float)s64[st_entry<double>(p, o)];
}

// FP16 copy: each stored off-diagonal (as for FP32) divided by the level scale
// (exact) and rounded once, from FP64, to the nearest FP16 value; values below
// the smallest normal FP16 number (2^-14, i.e. below 2^-14 of the level's
// scale) are stored as zero.
// This is the definition the tests check; it does not depend on how the
// hardware treats FP16 subnormals.
__global__ __launch_bounds__(256) void round_stencil16_kernel(const double* __restrict__ s64,
                                                              _Float16* __restrict__ s16, int NX,
                                                              int NY, size_t N, double inv_scale) {
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const StLayout L = dev_layout(NX, NY);
  const size_t p = L.node((int)(n % NX), (int)((n / NX) % NY), (int)(n / ((size_t)NX * NY)));
#pragma unroll
  for (int o = 0; o < 27; ++o)
    if (stored32(o)) {
      const double v = s64[st_entry<double>(p, o)] * inv_scale;
      s16[st_entry16(p, o)] = fabs(v) < 0x1p-14 ? (_Float16)0.0 : (_Float16)v;
    }
}

// Largest |off-diagonal| of an FP64 stencil: a per-block maximum (fixed tree),
// then one block over the block maxima.
__global__ __launch_bounds__(256) void absmax_kernel(const double* __restrict__ s64, int NX, int NY,
                                                     size_t N, double* __restrict__ out) {
  __shared__ double sm[256];
  const StLayout L = dev_layout(NX, NY);
  double m = 0.0;
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    const size_t p = L.node((int)(n % NX), (int)((n / NX) % NY), (int)(n / ((size_t)NX * NY)));
    for (int o = 0; o < 27; ++o)
      if (o != 13) m = fmax(m, fabs(s64[st_entry<double>(p, o)]));
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void max_of_kernel(const double* __restrict__ v, int n,
                                                     double* __restrict__ out) {
  __shared__ double sm[256];
  double m = 0.0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) m = fmax(m, v[t]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0];
}

// FP16 stencil in natural order, as the FP32 values the kernels use times the scale
__global__ __launch_bounds__(256) void unsplit16_kernel(const _Float16* __restrict__ s,
                                                        float* __restrict__ out, int NX, int NY,
                                                        size_t N, float scale) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= N * 27) return;
  const size_t o = gid / N, n = gid % N;
  const StLayout L = dev_layout(NX, NY);
  const int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((size_t)NX * NY));
  const size_t p = L.node(i, j, k);
  // the coupling to the node below is that node's upward one (0 on the bottom plane)
  const float below = k > 0 ? (float)s[st_entry16(L.node(i, j, k - 1), 22)] : 0.f;
  if (o == 13) {
    float a[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) a[q] = stored32(q) ? (float)s[st_entry16(p, q)] : 0.f;
    a[4] = below;
    out[gid] = stencil_diag(a) * scale;
  } else if (o == 4) {
    out[gid] = below * scale;
  } else {
    out[gid] = (float)s[st_entry16(p, (int)o)] * scale;
  }
}

template <class T>
__global__ __launch_bounds__(256) void unsplit_kernel(const T* __restrict__ s, T* __restrict__ out,
                                                      int NX, int NY, size_t N) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= N * 27) return;
  const size_t o = gid / N, n = gid % N;
  const StLayout L = dev_layout(NX, NY);
  const int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((size_t)NX * NY));
  const size_t p = L.node(i, j, k);
  if constexpr (sizeof(T) == 4) {
    // the coupling to the node below is that node's upward one (0 on the bottom plane)
    const float below = k > 0 ? s[st_entry<float>(L.node(i, j, k - 1), 22)] : 0.f;
    if (o == 13) {
      float a[27];
#pragma unroll
      for (int q = 0; q < 27; ++q) a[q] = stored32(q) ? s[st_entry<float>(p, q)] : 0.f;
      a[4] = below;
      out[gid] = stencil_diag(a);
      return;
    }
    if (o == 4) {
      out[gid] = below;
      return;
    }
  }
  out[gid] = s[st_entry<T>(p, (int)o)];
}

// ---------------------------------------------------------------- coarsest level

// e[idx] = Kinv r[idx] for the free coarsest nodes (Kinv symmetric, so column
// `row` is read with consecutive lanes on consecutive addresses).  A block of
// four waves computes 64 rows: wave w sums the w-th quarter of the columns, and
// the four partial sums are added in wave order.  LDS: r (n doubles), then the
// 4 x 64 partial sums.
constexpr int COARSE_ROWS = 64;
template <class T>
__device__ __forceinline__ void coarse_body(const CoarseJob& C, int b, double* rs) {
  const T* __restrict__ r = static_cast<const T*>(C.r);
  T* __restrict__ e = static_cast<T*>(C.e);
  const int n = C.n;
  double* part = rs + n;
  __syncthreads();  // rs and part may still be read by the previous work item
  for (int t = threadIdx.x; t < n; t += blockDim.x) rs[t] = (double)r[C.idx[t]];
  __syncthreads();
  const int lane = threadIdx.x % COARSE_ROWS, w = threadIdx.x / COARSE_ROWS;
  const int row = b * COARSE_ROWS + lane;
  const int q = (n + 3) / 4, j0 = min(n, w * q), j1 = min(n, j0 + q);
  double s = 0.0;
  if (row < n) {
    // unrolled so that several columns' loads are in flight; one sum, in order
#pragma unroll 8
    for (int jj = j0; jj < j1; ++jj) s += C.inv[(size_t)jj * n + row] * rs[jj];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (w == 0 && row < n)
    e[C.idx[row]] = (T)(((part[lane] + part[COARSE_ROWS + lane]) + part[2 * COARSE_ROWS + lane]) +
                        part[3 * COARSE_ROWS + lane]);
}

template <class T>
__global__ __launch_bounds__(256) void coarse_solve_kernel(CoarseJob C) {
  extern __shared__ double rs[];
  coarse_body<T>(C, blockIdx.x, rs);
}

template <class T>
__global__ __launch_bounds__(256) void coarse_solve_batched(WorkList W) {
  extern __shared__ double rs[];
  for (int g = blockIdx.x; g < W.total; g += gridDim.x) {
    const int j = find_job(W.prefix, W.njobs, g);
    if (!W.active[W.member[j]]) continue;
    coarse_body<T>(static_cast<const CoarseJob*>(W.jobs)[j], g - W.prefix[j], rs);
  }
}

// ---------------------------------------------------------------- vectors

// p = *q (a device scalar of type T), or 0 when q is null
template <class T>
__device__ __forceinline__ void fill_body(const VecJob& V, int b) {
  T* __restrict__ p = static_cast<T*>(V.p);
  const T v = V.q ? *static_cast<const T*>(V.q) : T(0);
  for (size_t i = (size_t)b * 256 + threadIdx.x; i < V.n; i += (size_t)V.nblocks * 256) p[i] = v;
}

// Row-split position of natural node n of an NX-wide grid.
__device__ __forceinline__ size_t split_pos(size_t n, int NX) {
  const size_t row = n / NX;
  return row * NX + sx((int)(n - row * NX), (NX + 1) >> 1);
}

// r32 (row-split) = (float)(r (natural) * scale)
__device__ __forceinline__ void scale_body(const VecJob& V, int b) {
  const double* __restrict__ r = static_cast<const double*>(V.q);
  float* __restrict__ r32 = static_cast<float*>(V.p);
  const double s = *V.scale;
  for (size_t i = (size_t)b * 256 + threadIdx.x; i < V.n; i += (size_t)V.nblocks * 256)
    r32[split_pos(i, V.NX)] = (float)(r[i] * s);
}

// lam (natural) += (double)e (row-split) / scale
__device__ __forceinline__ void update_body(const VecJob& V, int b) {
  const float* __restrict__ e = static_cast<const float*>(V.q);
  double* __restrict__ lam = static_cast<double*>(V.p);
  const double inv = 1.0 / *V.scale;
  for (size_t i = (size_t)b * 256 + threadIdx.x; i < V.n; i += (size_t)V.nblocks * 256)
    lam[i] += (double)e[split_pos(i, V.NX)] * inv;
}

// natural <-> row-split copies of a level vector
template <class T>
__global__ __launch_bounds__(256) void relayout_kernel(const T* __restrict__ src, T* __restrict__ dst,
                                                       size_t n, int NX, int to_split) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t q = split_pos(i, NX);
    if (to_split) dst[q] = src[i];
    else dst[i] = src[q];
  }
}

// Only the fixed nodes are visited: the whole planes below kf and above kl,
// then on each free plane the x = 0, x = NX-1, y = 0 and y = NY-1 lines that are
// fixed (a corner may be written twice, with the same zero).
__device__ __forceinline__ void zero_fixed_body(const VecJob& V, int b) {
  double* __restrict__ v = static_cast<double*>(V.p);
  const int NX = V.NX, NY = V.NY, NZ = V.NZ;
  const size_t plane = (size_t)NX * NY;
  const int kf = V.fc.k_first(), kl = V.fc.k_last(NZ);
  const size_t below = (size_t)kf * plane;                                  // planes 0..kf-1
  const size_t above = (size_t)(NZ - 1 - (kl >= kf - 1 ? kl : kf - 1)) * plane;  // planes kl+1..NZ-1
  const size_t line = 2 * (size_t)NY + 2 * (size_t)NX;                      // face nodes of a plane
  const size_t nfree = kl >= kf ? (size_t)(kl - kf + 1) : 0;
  const size_t total = below + above + nfree * line;
  const bool fx0 = V.fc.x_fixed(0, NX), fx1 = V.fc.x_fixed(NX - 1, NX);
  const bool fy0 = V.fc.y_fixed(0, NY), fy1 = V.fc.y_fixed(NY - 1, NY);
  for (size_t t = (size_t)b * 256 + threadIdx.x; t < total; t += (size_t)V.nblocks * 256) {
    if (t < below) {
      v[t] = 0.0;
    } else if (t < below + above) {
      v[(size_t)NZ * plane - above + (t - below)] = 0.0;
    } else {
      const size_t u = t - below - above;
      const size_t k = (size_t)kf + u / line;
      const size_t r = u % line;
      double* pl = v + k * plane;
      if (r < (size_t)NY) {
        if (fx0) pl[r * NX] = 0.0;
      } else if (r < 2 * (size_t)NY) {
        if (fx1) pl[(r - NY) * NX + NX - 1] = 0.0;
      } else if (r < 2 * (size_t)NY + NX) {
        if (fy0) pl[r - 2 * (size_t)NY] = 0.0;
      } else {
        if (fy1) pl[(size_t)(NY - 1) * NX + (r - 2 * (size_t)NY - NX)] = 0.0;
      }
    }
  }
}

template <class T>
__global__ __launch_bounds__(256) void fill_kernel(T* __restrict__ p, size_t n, T v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// p[i] = a pseudo-random value in [-1, 1): the splitmix64 finaliser of i + seed
// (Steele, Lea and Flood, "Fast splittable pseudorandom number generators").
__global__ __launch_bounds__(256) void hash_fill_kernel(double* __restrict__ p, size_t n,
                                                        unsigned long long seed) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    unsigned long long z = (unsigned long long)i + seed * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    p[i] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
  }
}

template <class T>
__global__ __launch_bounds__(256) void fill_batched(WorkList W) {
  MCW_BATCHED_LOOP(VecJob, fill_body<T>)
}
__global__ __launch_bounds__(256) void scale_kernel(VecJob V) { scale_body(V, blockIdx.x); }
__global__ __launch_bounds__(256) void scale_batched(WorkList W) { MCW_BATCHED_LOOP(VecJob, scale_body) }
__global__ __launch_bounds__(256) void update_kernel(VecJob V) { update_body(V, blockIdx.x); }
__global__ __launch_bounds__(256) void update_batched(WorkList W) { MCW_BATCHED_LOOP(VecJob, update_body) }
__global__ __launch_bounds__(256) void zero_fixed_kernel(VecJob V) { zero_fixed_body(V, blockIdx.x); }
__global__ __launch_bounds__(256) void zero_fixed_batched(WorkList W) {
  MCW_BATCHED_LOOP(VecJob, zero_fixed_body)
}

__global__ __launch_bounds__(256) void axpy64_kernel(double alpha, const double* __restrict__ x,
                                                     double* __restrict__ y, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    y[i] += alpha * x[i];
}

// Deterministic final sum of per-block partials: thread t adds entries
// t, t+256, ... in order, then a fixed tree.
// Each thread adds partials i, i + 256, i + 512, ... in that order; eight are
// loaded before the first of them is added, so the loads overlap instead of
// each waiting for the add before it (same order of additions, same result).
__device__ __forceinline__ void sum_body(const SumJob& S, double* s) {
  for (int w = 0; w < S.width; ++w) {
    const double* __restrict__ p = S.partials + (size_t)w * S.n_part;
    double a = 0.0;
    size_t i = threadIdx.x;
    for (; i + 7 * 256 < S.n_part; i += 8 * 256) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p[i + (size_t)u * 256];
#pragma unroll
      for (int u = 0; u < 8; ++u) a += v[u];
    }
    for (; i < S.n_part; i += 256) a += p[i];
    block_sum_to(a, s, &S.out[w]);
  }
}

__global__ __launch_bounds__(256) void sum_partials_kernel(SumJob S) {
  __shared__ double s[256];
  sum_body(S, s);
}

// one block per job
__global__ __launch_bounds__(256) void sum_partials_batched(const SumJob* __restrict__ jobs, int n) {
  __shared__ double s[256];
  for (int j = blockIdx.x; j < n; j += gridDim.x) sum_body(jobs[j], s);
}

unsigned grid_stride_blocks(size_t n) {
  const size_t b = (n + 255) / 256;
  return (unsigned)(b < 16384 ? (b == 0 ? 1 : b) : 16384);
}

unsigned batched_grid(int total) { return (unsigned)std::max(1, std::min(total, 8192)); }

}  // namespace

// ---------------------------------------------------------------- job builders

ColJob col_job(const Dims& d, const Faces& fc, StRef st, const void* f, void* x, void* r,
               int colour, int by) {
  ColJob J{};
  J.by = by;
  J.st = st.p;
  J.h16 = st.h16;
  J.sc = st.sc;
  J.isc = st.isc;
  J.f = f;
  J.x = x;
  J.r = r;
  J.NX = d.NX();
  J.NY = d.NY();
  J.NZ = d.NZ();
  J.fc = fc;
  if (colour >= 0) {
    static const int order[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
    J.ci = order[colour][0];
    J.cj = order[colour][1];
    J.ncx = (d.NX() - J.ci + 1) / 2;
    J.ncy = (d.NY() - J.cj + 1) / 2;
  } else {
    J.ncx = d.NX();
    J.ncy = d.NY();
  }
  J.tiles_x = (J.ncx + BX - 1) / BX;
  J.nblocks = std::max(0, J.tiles_x * ((J.ncy + by - 1) / by));
  return J;
}

void residual_skip(ColJob& J, int mode) {
  if (mode < 0 || mode > 2) throw Error{MCW_HIP_ERROR, "internal error: residual skip mode"};
  J.skip11 = mode;
  if (mode == 2) {
    J.ncy = (J.NY + 1) / 2;
    J.nblocks = std::max(0, J.tiles_x * ((J.ncy + J.by - 1) / J.by));
  }
}

XferJob xfer_job(const Dims& df, const Dims& dc, const Faces& fc, const DirMapDev& mx,
                 const DirMapDev& my, const DirMapDev& mz, const void* src, void* dst,
                 bool restriction) {
  XferJob X{};
  X.src = src;
  X.dst = dst;
  X.NXf = df.NX();
  X.NYf = df.NY();
  X.NZf = df.NZ();
  X.NXc = dc.NX();
  X.NYc = dc.NY();
  X.NZc = dc.NZ();
  X.fc = fc;
  X.mx = mx;
  X.my = my;
  X.mz = mz;
  const int nxc = restriction ? X.NXc : X.NXf, nyc = restriction ? X.NYc : X.NYf;
  X.tiles_x = (nxc + BX - 1) / BX;
  X.nblocks = X.tiles_x * ((nyc + BY - 1) / BY);
  return X;
}

CoarseJob coarse_job(int n, const double* inv, const int* idx, const void* r, void* e) {
  CoarseJob C{n, inv, idx, r, e, (n + COARSE_ROWS - 1) / COARSE_ROWS};
  return C;
}

VecJob vec_job(void* p, const void* q, size_t n, const double* scale) {
  VecJob V{};
  V.p = p;
  V.q = q;
  V.n = n;
  V.scale = scale;
  V.nblocks = (int)std::min<size_t>((n + 255) / 256, 2048);
  if (V.nblocks < 1) V.nblocks = 1;
  return V;
}

// ---------------------------------------------------------------- single launches

// LDS bytes of a line-smoother launch with `threads` threads per block when
// the column solve can keep its two sequences there (at most 64 KB), else 0
// (the sequences then go through the level's line buffer and x).
template <class T>
size_t line_lds_bytes(const Dims& d, const Faces& fc, int threads) {
  const int np = fc.k_last(d.NZ()) - fc.k_first() + 1;
  const size_t bytes = 2 * (size_t)std::max(np, 0) * (size_t)threads * sizeof(T);
  return np > 0 && bytes <= 65536 ? bytes : 0;
}

template <class T, bool LINE, int SF>
int smooth_sweep_f(const Dims& d, const Faces& fc, StRef st, const T* f, T* x, T* cbuf,
                   hipStream_t s, int by, bool reverse, T* r_last) {
  if (reverse) r_last = nullptr;
  if (by == 0) {
    // colours (0,0),(1,0) then (0,1),(1,1); reversed: (1,1),(0,1) then (1,0),(0,0)
    for (int pr = 0; pr < 2; ++pr) {
      const int c0 = reverse ? 3 - 2 * pr : 2 * pr, c1 = reverse ? c0 - 1 : c0 + 1;
      ColJob J0 = col_job(d, fc, st, f, x, cbuf, c0, 1);
      ColJob J1 = col_job(d, fc, st, f, x, cbuf, c1, 1);
      if (c1 == 3) J1.rlast = r_last;
      if (J0.ncy <= 0) continue;
      const int cols = std::max(J0.ncx, J1.ncx);
      const int threads = std::min(fused_threads<T, LINE>(), std::max(64, (cols + 63) / 64 * 64));
      if constexpr (!LINE) {
        if (c1 == 3 && r_last) {
          // the odd rows of the sweep that ends the pre-smoothing: both colours
          // leave their residual
          J0.rlast = r_last;
          J1.rside = r_last;
          const int ts = std::min(threads, fused_threads<T, false, true>());
          gs_fused_kernel<T, false, false, SF, false, true><<<J0.ncy, ts, 0, s>>>(J0, J1);
          MCW_CHECK_LAUNCH();
          continue;
        }
      }
      if constexpr (LINE) {
        const size_t lds = line_lds_bytes<T>(d, fc, threads);
        if (lds) {
          if (reverse)
            gs_fused_kernel<T, true, LINE, SF, true><<<J0.ncy, threads, lds, s>>>(J0, J1);
          else
            gs_fused_kernel<T, false, LINE, SF, true><<<J0.ncy, threads, lds, s>>>(J0, J1);
          MCW_CHECK_LAUNCH();
          continue;
        }
      }
      if (reverse)
        gs_fused_kernel<T, true, LINE, SF><<<J0.ncy, threads, 0, s>>>(J0, J1);
      else
        gs_fused_kernel<T, false, LINE, SF><<<J0.ncy, threads, 0, s>>>(J0, J1);
      MCW_CHECK_LAUNCH();
    }
    // every odd row's residual is in place when the point smoother's odd rows
    // ran with r_last (a level with no odd row has none to compute)
    return r_last ? (LINE ? 1 : 2) : 0;
  }
  const size_t lds = LINE ? line_lds_bytes<T>(d, fc, BX * by) : 0;
  ColJob J01{};  // colour (0,1) of the sweep that ends the pre-smoothing
  for (int cc = 0; cc < 4; ++cc) {
    const int c = reverse ? 3 - cc : cc;
    ColJob J = col_job(d, fc, st, f, x, cbuf, c, by);
    if (c == 3) J.rlast = r_last;
    if constexpr (!LINE) {
      if (r_last && c == 2) {
        J.rlast = r_last;
        J01 = J;
      }
      if (r_last && c == 3) {
        // as the fused pass with SIDE: the (1,1) pass leaves the side sums,
        // then the (0,1) columns' residual is finished
        J.rside = r_last;
        if (J.nblocks > 0) {
          gs_pass_kernel<T, false, false, SF, false, true><<<J.nblocks, BX * by, 0, s>>>(J);
          MCW_CHECK_LAUNCH();
        }
        if (J01.nblocks > 0) {
          side_residual_kernel<T, SF><<<J01.nblocks, BX * by, 0, s>>>(J01);
          MCW_CHECK_LAUNCH();
        }
        continue;
      }
    }
    if (J.nblocks <= 0) continue;
    if constexpr (LINE) {
      if (lds) {
        if (reverse)
          gs_pass_kernel<T, true, LINE, SF, true><<<J.nblocks, BX * by, lds, s>>>(J);
        else
          gs_pass_kernel<T, false, LINE, SF, true><<<J.nblocks, BX * by, lds, s>>>(J);
        MCW_CHECK_LAUNCH();
        continue;
      }
    }
    if (reverse)
      gs_pass_kernel<T, true, LINE, SF><<<J.nblocks, BX * by, 0, s>>>(J);
    else
      gs_pass_kernel<T, false, LINE, SF><<<J.nblocks, BX * by, 0, s>>>(J);
    MCW_CHECK_LAUNCH();
  }
  return r_last ? (LINE ? 1 : 2) : 0;
}

// format 1 (FP16 stencil) exists for FP32 V-cycles only
template <class T, bool LINE>
int smooth_sweep_t(const Dims& d, const Faces& fc, StRef st, const T* f, T* x, T* cbuf,
                   hipStream_t s, int by, bool reverse, T* r_last) {
  if constexpr (sizeof(T) == 4) {
    if (st.h16) return smooth_sweep_f<T, LINE, 1>(d, fc, st, f, x, cbuf, s, by, reverse, r_last);
  }
  return smooth_sweep_f<T, LINE, 0>(d, fc, st, f, x, cbuf, s, by, reverse, r_last);
}

template <class T>
int launch_smooth_sweep(const Dims& d, const Faces& fc, StRef st, const T* f, T* x,
                        hipStream_t s, int by, bool reverse, T* line_buf, T* r_last) {
  if (line_buf) return smooth_sweep_t<T, true>(d, fc, st, f, x, line_buf, s, by, reverse, r_last);
  return smooth_sweep_t<T, false>(d, fc, st, f, x, nullptr, s, by, reverse, r_last);
}

// ---- conjugate gradients on level-0 vectors, coefficients kept on the device
// sc[0] = r.z of the current step, sc[1] = alpha, sc[2] = beta, sc[3] = r.r.
// Each kernel is a body run by block `blk` of `nblk` (grid-stride within the
// vector), so a batched launch over several members does the same arithmetic,
// in the same order, as the single launch of each.

namespace {

// per-block FP64 partial sums of a.b and, when c is given, a.c (channel-major)
template <class T>
__device__ __forceinline__ void dot2_body(const T* __restrict__ a, const T* __restrict__ b,
                                          const T* __restrict__ c, size_t n,
                                          double* __restrict__ partials, int blk, int nblk,
                                          double* s_red) {
  double ab = 0.0, ac = 0.0;
  for (size_t i = (size_t)blk * 256 + threadIdx.x; i < n; i += (size_t)nblk * 256) {
    const double av = a[i];
    ab += av * (double)b[i];
    if (c) ac += av * (double)c[i];
  }
  block_sum_to(ab, s_red, &partials[blk]);
  if (c) block_sum_to(ac, s_red, &partials[nblk + blk]);
}

template <class T>
__global__ __launch_bounds__(256) void dot2_kernel(const T* __restrict__ a, const T* __restrict__ b,
                                                   const T* __restrict__ c, size_t n,
                                                   double* __restrict__ partials) {
  __shared__ double s_red[256];
  dot2_body<T>(a, b, c, n, partials, blockIdx.x, gridDim.x, s_red);
}

__device__ __forceinline__ void cg_reset_body(double* sc) {
  sc[0] = 1.0;
  sc[1] = 0.0;
  sc[2] = 0.0;
  sc[3] = 0.0;
}

__global__ void cg_reset_kernel(double* sc) {
  if (threadIdx.x == 0) cg_reset_body(sc);
}

// mode 0: the partials hold z.r and z.q of the new preconditioned residual z,
//   q = -K p of the last direction; beta = alpha z.q / (r.z)_old, the
//   Polak-Ribiere form z.(r_new - r_old) / (r.z)_old, robust to a preconditioner
//   that is symmetric only up to rounding; zero on the first step (alpha = 0).
// mode 1: the partials hold p.q = -p.Kp; alpha = (r.z) / p.Kp, zero on breakdown.
// mode 2: the partials hold r.r after the update; sc[3] = r.r.
__device__ __forceinline__ void cg_coeff_body(const double* __restrict__ partials, size_t n_part,
                                              int mode, double* sc, double* s, double* tot) {
  sum_body(SumJob{partials, n_part, mode == 0 ? 2 : 1, tot}, s);
  if (threadIdx.x == 0) {
    if (mode == 0) {
      const double rz_old = sc[0], alpha = sc[1];
      sc[2] = (alpha != 0.0 && rz_old != 0.0) ? alpha * tot[1] / rz_old : 0.0;
      sc[0] = tot[0];
    } else if (mode == 1) {
      const double pkp = -tot[0];
      sc[1] = (pkp > 0.0 && isfinite(pkp)) ? sc[0] / pkp : 0.0;
    } else {
      sc[3] = tot[0];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void cg_coeff_kernel(const double* __restrict__ partials,
                                                       size_t n_part, int mode, double* sc) {
  __shared__ double s[256];
  __shared__ double tot[2];
  cg_coeff_body(partials, n_part, mode, sc, s, tot);
}

// p = z + beta p (p = z on the first step, so p need not start finite)
template <class T>
__device__ __forceinline__ void cg_direction_body(T* __restrict__ p, const T* __restrict__ z,
                                                  const double* __restrict__ sc, size_t n, int blk,
                                                  int nblk) {
  const T beta = (T)sc[2];
  for (size_t i = (size_t)blk * 256 + threadIdx.x; i < n; i += (size_t)nblk * 256)
    p[i] = beta == T(0) ? z[i] : z[i] + beta * p[i];
}

template <class T>
__global__ __launch_bounds__(256) void cg_direction_kernel(T* __restrict__ p, const T* __restrict__ z,
                                                           const double* __restrict__ sc, size_t n) {
  cg_direction_body<T>(p, z, sc, n, blockIdx.x, gridDim.x);
}

// e += alpha p; r += alpha q (q = -K p), with per-block partial sums of the new r.r
template <class T>
__device__ __forceinline__ void cg_update_body(T* __restrict__ e, const T* __restrict__ p,
                                               T* __restrict__ r, const T* __restrict__ q,
                                               const double* __restrict__ sc, size_t n,
                                               double* __restrict__ partials, int blk, int nblk,
                                               double* s_red) {
  const T alpha = (T)sc[1];
  double rr = 0.0;
  for (size_t i = (size_t)blk * 256 + threadIdx.x; i < n; i += (size_t)nblk * 256) {
    e[i] += alpha * p[i];
    const T rn = r[i] + alpha * q[i];
    r[i] = rn;
    rr += (double)rn * (double)rn;
  }
  block_sum_to(rr, s_red, &partials[blk]);
}

template <class T>
__global__ __launch_bounds__(256) void cg_update_kernel(T* __restrict__ e, const T* __restrict__ p,
                                                        T* __restrict__ r, const T* __restrict__ q,
                                                        const double* __restrict__ sc, size_t n,
                                                        double* __restrict__ partials) {
  __shared__ double s_red[256];
  cg_update_body<T>(e, p, r, q, sc, n, partials, blockIdx.x, gridDim.x, s_red);
}

// ---- batched forms: one work item is one block of one member's vector

template <class T>
__device__ __forceinline__ void dot2_item(const CgJob& C, int b) {
  __shared__ double s_red[256];
  dot2_body<T>(static_cast<const T*>(C.z), static_cast<const T*>(C.r), static_cast<const T*>(C.q), C.n,
               C.partials, b, C.nblocks, s_red);
}

template <class T>
__global__ __launch_bounds__(256) void dot2_batched(WorkList W) {
  MCW_BATCHED_LOOP(CgJob, dot2_item<T>)
}

template <class T>
__device__ __forceinline__ void direction_item(const CgJob& C, int b) {
  cg_direction_body<T>(static_cast<T*>(C.p), static_cast<const T*>(C.z), C.sc, C.n, b, C.nblocks);
}

template <class T>
__global__ __launch_bounds__(256) void cg_direction_batched(WorkList W) {
  MCW_BATCHED_LOOP(CgJob, direction_item<T>)
}

template <class T>
__device__ __forceinline__ void update_item(const CgJob& C, int b) {
  __shared__ double s_red[256];
  cg_update_body<T>(static_cast<T*>(C.e), static_cast<const T*>(C.p), static_cast<T*>(C.r),
                    static_cast<const T*>(C.q), C.sc, C.n, C.partials, b, C.nblocks, s_red);
}

template <class T>
__global__ __launch_bounds__(256) void cg_update_batched(WorkList W) {
  MCW_BATCHED_LOOP(CgJob, update_item<T>)
}

// one block per member; members whose flag is off keep their coefficients
__global__ __launch_bounds__(256) void cg_coeff_batched(const CgJob* __restrict__ jobs, int n, int mode,
                                                        const int* __restrict__ active) {
  __shared__ double s[256];
  __shared__ double tot[2];
  for (int j = blockIdx.x; j < n; j += gridDim.x) {
    if (!active[jobs[j].member]) continue;
    const size_t np = mode == 1 ? (size_t)jobs[j].res_blocks : (size_t)jobs[j].nblocks;
    cg_coeff_body(jobs[j].partials, np, mode, jobs[j].sc, s, tot);
  }
}

__global__ void cg_reset_batched(const CgJob* __restrict__ jobs, int n, const int* __restrict__ active) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n && active[jobs[j].member]) cg_reset_body(jobs[j].sc);
}

template <class T>
__global__ __launch_bounds__(256) void add_kernel(T* __restrict__ y, const T* __restrict__ x, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) y[i] += x[i];
}

}  // namespace

unsigned cg_blocks(size_t n) { return std::min<unsigned>(grid_stride_blocks(n), 2048); }

void launch_cg_reset(double* sc, hipStream_t s) {
  cg_reset_kernel<<<1, 64, 0, s>>>(sc);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_cg_beta(const T* z, const T* r, const T* q, size_t n, double* partials, size_t cap,
                    double* sc, hipStream_t s) {
  const unsigned blocks = cg_blocks(n);
  need_partials(2 * (size_t)blocks, cap);
  dot2_kernel<T><<<blocks, 256, 0, s>>>(z, r, q, n, partials);
  MCW_CHECK_LAUNCH();
  cg_coeff_kernel<<<1, 256, 0, s>>>(partials, blocks, 0, sc);
  MCW_CHECK_LAUNCH();
}

void launch_cg_alpha(size_t n_part, const double* partials, double* sc, hipStream_t s) {
  cg_coeff_kernel<<<1, 256, 0, s>>>(partials, n_part, 1, sc);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_add(T* y, const T* x, size_t n, hipStream_t s) {
  add_kernel<T><<<grid_stride_blocks(n), 256, 0, s>>>(y, x, n);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_cg_direction(T* p, const T* z, const double* sc, size_t n, hipStream_t s) {
  cg_direction_kernel<T><<<grid_stride_blocks(n), 256, 0, s>>>(p, z, sc, n);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_cg_update(T* e, const T* p, T* r, const T* q, double* sc, size_t n, double* partials,
                      size_t cap, hipStream_t s) {
  const unsigned blocks = cg_blocks(n);
  need_partials(blocks, cap);
  cg_update_kernel<T><<<blocks, 256, 0, s>>>(e, p, r, q, sc, n, partials);
  MCW_CHECK_LAUNCH();
  cg_coeff_kernel<<<1, 256, 0, s>>>(partials, blocks, 2, sc);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_residual(const Dims& d, const Faces& fc, StRef st, const T* x, const T* f, T* r,
                     double* partials, size_t* n_part, hipStream_t s, int by, size_t cap,
                     int last_colour_done) {
  ColJob J = col_job(d, fc, st, f, const_cast<T*>(x), r, -1, by);
  // the norm needs every node's residual in this launch
  if (last_colour_done && partials)
    throw Error{MCW_HIP_ERROR, "internal error: a residual norm needs every column's residual"};
  residual_skip(J, last_colour_done);
  if (partials) need_partials((size_t)J.nblocks, cap);
  const bool h16 = sizeof(T) == 4 && st.h16;
  if (partials && h16)
    residual_kernel<T, true, false, 1><<<J.nblocks, BX * by, 0, s>>>(J, partials);
  else if (partials)
    residual_kernel<T, true, false, 0><<<J.nblocks, BX * by, 0, s>>>(J, partials);
  else if (h16)
    residual_kernel<T, false, false, 1><<<J.nblocks, BX * by, 0, s>>>(J, nullptr);
  else
    residual_kernel<T, false, false, 0><<<J.nblocks, BX * by, 0, s>>>(J, nullptr);
  MCW_CHECK_LAUNCH();
  if (n_part) *n_part = J.nblocks;
}

// q = -K p with the per-block partial sums of p.q
template <class T>
void launch_neg_apply_dot(const Dims& d, const Faces& fc, StRef st, const T* p, T* q,
                          double* partials, size_t cap, size_t* n_part, hipStream_t s, int by) {
  const ColJob J = col_job(d, fc, st, nullptr, const_cast<T*>(p), q, -1, by);
  need_partials((size_t)J.nblocks, cap);
  if (sizeof(T) == 4 && st.h16)
    residual_kernel<T, true, true, 1><<<J.nblocks, BX * by, 0, s>>>(J, partials);
  else
    residual_kernel<T, true, true, 0><<<J.nblocks, BX * by, 0, s>>>(J, partials);
  MCW_CHECK_LAUNCH();
  *n_part = J.nblocks;
}

template <class T>
void launch_restrict(const Dims& df, const Dims& dc, const Faces& fc, const DirMapDev& mx,
                     const DirMapDev& my, const DirMapDev& mz, const T* r, T* rc, hipStream_t s) {
  const XferJob X = xfer_job(df, dc, fc, mx, my, mz, r, rc, true);
  restrict_kernel<T><<<X.nblocks, 256, 0, s>>>(X);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_prolong_dims(const Dims& df, const Dims& dc, const Faces& fc, const DirMapDev& mx,
                         const DirMapDev& my, const DirMapDev& mz, const T* e, T* x,
                         hipStream_t s) {
  const XferJob X = xfer_job(df, dc, fc, mx, my, mz, e, x, false);
  if (X.NXc != X.NXf) {
    // horizontally coarsened: one thread per coarse column, tiles over the coarse grid
    XferJob P = X;
    P.tiles_x = (P.NXc + BX - 1) / BX;
    P.nblocks = P.tiles_x * ((P.NYc + BY - 1) / BY);
    prolong_pairs_kernel<T, 4><<<P.nblocks, 256, 0, s>>>(P);
  } else {
    prolong_kernel<T><<<X.nblocks, 256, 0, s>>>(X);
  }
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_coarse_solve(int n, const double* inv, const int* idx, const T* r, T* e,
                         hipStream_t s) {
  const CoarseJob C = coarse_job(n, inv, idx, r, e);
  coarse_solve_kernel<T>
      <<<C.nblocks, 4 * COARSE_ROWS, (size_t)(n + 4 * COARSE_ROWS) * sizeof(double), s>>>(C);
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
  round_stencil_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(st64, st32, d.NX(), d.NY(), N);
  MCW_CHECK_LAUNCH();
}

void launch_unsplit_stencil(const Dims& d, const void* st, void* out, int kind, hipStream_t s,
                            float scale) {
  const size_t N = d.N();
  const unsigned blocks = (unsigned)((N * 27 + 255) / 256);
  if (kind == 1)
    unsplit_kernel<double><<<blocks, 256, 0, s>>>(static_cast<const double*>(st),
                                                  static_cast<double*>(out), d.NX(), d.NY(), N);
  else if (kind == 2)
    unsplit16_kernel<<<blocks, 256, 0, s>>>(static_cast<const _Float16*>(st),
                                            static_cast<float*>(out), d.NX(), d.NY(), N, scale);
  else
    unsplit_kernel<float><<<blocks, 256, 0, s>>>(static_cast<const float*>(st),
                                                 static_cast<float*>(out), d.NX(), d.NY(), N);
  MCW_CHECK_LAUNCH();
}

void launch_round_stencil16(const Dims& d, const double* st64, uint16_t* st16, double inv_scale,
                            hipStream_t s) {
  const size_t N = d.N();
  round_stencil16_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(
      st64, reinterpret_cast<_Float16*>(st16), d.NX(), d.NY(), N, inv_scale);
  MCW_CHECK_LAUNCH();
}

double stencil_absmax(const Dims& d, const double* st64, double* scratch, hipStream_t s) {
  const size_t N = d.N();
  const int blocks = (int)std::min<size_t>((N + 255) / 256, 1024);
  absmax_kernel<<<blocks, 256, 0, s>>>(st64, d.NX(), d.NY(), N, scratch);
  MCW_CHECK_LAUNCH();
  max_of_kernel<<<1, 256, 0, s>>>(scratch, blocks, scratch + blocks);
  MCW_CHECK_LAUNCH();
  double m = 0.0;
  MCW_HIP(hipMemcpyAsync(&m, scratch + blocks, sizeof(double), hipMemcpyDeviceToHost, s));
  MCW_HIP(hipStreamSynchronize(s));
  return m;
}

template <class T>
void launch_relayout(const Dims& d, const T* src, T* dst, bool to_split, hipStream_t s) {
  relayout_kernel<T><<<grid_stride_blocks(d.N()), 256, 0, s>>>(src, dst, d.N(), d.NX(), to_split ? 1 : 0);
  MCW_CHECK_LAUNCH();
}
template void launch_relayout<float>(const Dims&, const float*, float*, bool, hipStream_t);
template void launch_relayout<double>(const Dims&, const double*, double*, bool, hipStream_t);

void launch_scale_to_f32(const Dims& d, const double* r, const double* scale, float* r32,
                         hipStream_t s) {
  VecJob V = vec_job(r32, r, d.N(), scale);
  V.NX = d.NX();
  scale_kernel<<<V.nblocks, 256, 0, s>>>(V);
  MCW_CHECK_LAUNCH();
}

void launch_update_lambda(const Dims& d, const float* e, const double* scale, double* lam,
                          hipStream_t s) {
  VecJob V = vec_job(lam, e, d.N(), scale);
  V.NX = d.NX();
  update_kernel<<<V.nblocks, 256, 0, s>>>(V);
  MCW_CHECK_LAUNCH();
}

void launch_hash_fill(double* p, size_t n, unsigned long long seed, hipStream_t s) {
  hash_fill_kernel<<<grid_stride_blocks(n), 256, 0, s>>>(p, n, seed);
  MCW_CHECK_LAUNCH();
}

void launch_axpy64(size_t n, double alpha, const double* x, double* y, hipStream_t s) {
  axpy64_kernel<<<grid_stride_blocks(n), 256, 0, s>>>(alpha, x, y, n);
  MCW_CHECK_LAUNCH();
}

void launch_zero_fixed(const Dims& d, const Faces& fc, double* v, hipStream_t s) {
  VecJob V = vec_job(v, nullptr, d.N(), nullptr);
  V.NX = d.NX();
  V.NY = d.NY();
  V.NZ = d.NZ();
  V.fc = fc;
  zero_fixed_kernel<<<V.nblocks, 256, 0, s>>>(V);
  MCW_CHECK_LAUNCH();
}

void launch_sum_partials(const double* partials, size_t n_part, int width, double* out,
                         hipStream_t s) {
  const SumJob S{partials, n_part, width, out};
  sum_partials_kernel<<<1, 256, 0, s>>>(S);
  MCW_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- batched launches

template <class T, int SF>
void launch_gs_batched_f(const WorkList& W, hipStream_t s, int by, bool reverse, bool side) {
  if (side && !reverse)
    gs_pass_batched<T, SF, true><<<batched_grid(W.total), BX * by, 0, s>>>(W);
  else if (reverse)
    gs_pass_batched_rev<T, SF><<<batched_grid(W.total), BX * by, 0, s>>>(W);
  else
    gs_pass_batched<T, SF><<<batched_grid(W.total), BX * by, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_gs_batched(const WorkList& W, hipStream_t s, int by, bool reverse, bool h16, bool side) {
  if (W.total <= 0) return;
  if constexpr (sizeof(T) == 4) {
    if (h16) {
      launch_gs_batched_f<T, 1>(W, s, by, reverse, side);
      return;
    }
  }
  launch_gs_batched_f<T, 0>(W, s, by, reverse, side);
}

template <class T>
void launch_side_residual_batched(const WorkList& W, hipStream_t s, int by, bool h16) {
  if (W.total <= 0) return;
  if (sizeof(T) == 4 && h16)
    side_residual_batched<T, 1><<<batched_grid(W.total), BX * by, 0, s>>>(W);
  else
    side_residual_batched<T, 0><<<batched_grid(W.total), BX * by, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

template <class T, int SF>
void launch_gs_fused_batched_f(const WorkList& W, hipStream_t s, bool reverse, bool side) {
  if (side && !reverse)
    gs_fused_batched<T, false, SF, true><<<batched_grid(W.total), 256, 0, s>>>(W);
  else if (reverse)
    gs_fused_batched<T, true, SF><<<batched_grid(W.total), 256, 0, s>>>(W);
  else
    gs_fused_batched<T, false, SF><<<batched_grid(W.total), 256, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_gs_fused_batched(const WorkList& W, hipStream_t s, bool reverse, bool h16, bool side) {
  if (W.total <= 0) return;
  if constexpr (sizeof(T) == 4) {
    if (h16) {
      launch_gs_fused_batched_f<T, 1>(W, s, reverse, side);
      return;
    }
  }
  launch_gs_fused_batched_f<T, 0>(W, s, reverse, side);
}

template <class T>
void launch_dot2_batched(const WorkList& W, hipStream_t s) {
  if (W.total <= 0) return;
  dot2_batched<T><<<batched_grid(W.total), 256, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_cg_direction_batched(const WorkList& W, hipStream_t s) {
  if (W.total <= 0) return;
  cg_direction_batched<T><<<batched_grid(W.total), 256, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_cg_update_batched(const WorkList& W, hipStream_t s) {
  if (W.total <= 0) return;
  cg_update_batched<T><<<batched_grid(W.total), 256, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_neg_apply_dot_batched(const WorkList& W, hipStream_t s, int by, bool h16) {
  if (W.total <= 0) return;
  if (h16)
    residual_dot_batched<T, 1><<<batched_grid(W.total), BX * by, 0, s>>>(W);
  else
    residual_dot_batched<T, 0><<<batched_grid(W.total), BX * by, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

void launch_cg_coeff_batched(const CgJob* jobs, int n, int mode, const int* active, hipStream_t s) {
  if (n <= 0) return;
  cg_coeff_batched<<<(unsigned)n, 256, 0, s>>>(jobs, n, mode, active);
  MCW_CHECK_LAUNCH();
}

void launch_cg_reset_batched(const CgJob* jobs, int n, const int* active, hipStream_t s) {
  if (n <= 0) return;
  cg_reset_batched<<<(unsigned)((n + 63) / 64), 64, 0, s>>>(jobs, n, active);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_residual_batched(const WorkList& W, hipStream_t s, int by, bool h16) {
  if (W.total <= 0) return;
  if constexpr (sizeof(T) == 4) {
    if (h16) {
      residual_batched<T, 1><<<batched_grid(W.total), BX * by, 0, s>>>(W);
      MCW_CHECK_LAUNCH();
      return;
    }
  }
  residual_batched<T, 0><<<batched_grid(W.total), BX * by, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_restrict_batched(const WorkList& W, hipStream_t s) {
  if (W.total <= 0) return;
  restrict_batched<T><<<batched_grid(W.total), 256, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_prolong_batched(const WorkList& W, hipStream_t s) {
  if (W.total <= 0) return;
  prolong_batched<T><<<batched_grid(W.total), 256, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_coarse_batched(const WorkList& W, int max_n, hipStream_t s) {
  if (W.total <= 0) return;
  coarse_solve_batched<T><<<batched_grid(W.total), 4 * COARSE_ROWS,
                            (size_t)(max_n + 4 * COARSE_ROWS) * sizeof(double), s>>>(W);
  MCW_CHECK_LAUNCH();
}

template <class T>
void launch_fill_batched(const WorkList& W, hipStream_t s) {
  if (W.total <= 0) return;
  fill_batched<T><<<batched_grid(W.total), 256, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

void launch_scale_batched(const WorkList& W, hipStream_t s) {
  if (W.total <= 0) return;
  scale_batched<<<batched_grid(W.total), 256, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

void launch_update_batched(const WorkList& W, hipStream_t s) {
  if (W.total <= 0) return;
  update_batched<<<batched_grid(W.total), 256, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

void launch_zero_fixed_batched(const WorkList& W, hipStream_t s) {
  if (W.total <= 0) return;
  zero_fixed_batched<<<batched_grid(W.total), 256, 0, s>>>(W);
  MCW_CHECK_LAUNCH();
}

void launch_sum_batched(const SumJob* jobs, int n, hipStream_t s) {
  if (n <= 0) return;
  sum_partials_batched<<<(unsigned)n, 256, 0, s>>>(jobs, n);
  MCW_CHECK_LAUNCH();
}

#define MCW_INST(T)                                                                             \
  template int launch_smooth_sweep<T>(const Dims&, const Faces&, StRef, const T*, T*,           \
                                      hipStream_t, int, bool, T*, T*);                          \
  template void launch_cg_beta<T>(const T*, const T*, const T*, size_t, double*, size_t,       \
                                  double*, hipStream_t);                                        \
  template void launch_add<T>(T*, const T*, size_t, hipStream_t);                              \
  template void launch_cg_direction<T>(T*, const T*, const double*, size_t, hipStream_t);       \
  template void launch_cg_update<T>(T*, const T*, T*, const T*, double*, size_t, double*,      \
                                    size_t, hipStream_t);                                       \
  template void launch_neg_apply_dot<T>(const Dims&, const Faces&, StRef, const T*, T*,         \
                                        double*, size_t, size_t*, hipStream_t, int);            \
  template void launch_residual<T>(const Dims&, const Faces&, StRef, const T*, const T*, T*,    \
                                   double*, size_t*, hipStream_t, int, size_t, int);            \
  template void launch_restrict<T>(const Dims&, const Dims&, const Faces&, const DirMapDev&,    \
                                   const DirMapDev&, const DirMapDev&, const T*, T*,            \
                                   hipStream_t);                                                \
  template void launch_prolong_dims<T>(const Dims&, const Dims&, const Faces&,                  \
                                       const DirMapDev&, const DirMapDev&, const DirMapDev&,    \
                                       const T*, T*, hipStream_t);                              \
  template void launch_coarse_solve<T>(int, const double*, const int*, const T*, T*,            \
                                       hipStream_t);                                            \
  template void launch_fill<T>(T*, size_t, T, hipStream_t);                                     \
  template void launch_gs_batched<T>(const WorkList&, hipStream_t, int, bool, bool, bool);      \
  template void launch_side_residual_batched<T>(const WorkList&, hipStream_t, int, bool);       \
  template void launch_gs_fused_batched<T>(const WorkList&, hipStream_t, bool, bool, bool);     \
  template void launch_residual_batched<T>(const WorkList&, hipStream_t, int, bool);            \
  template void launch_restrict_batched<T>(const WorkList&, hipStream_t);                       \
  template void launch_prolong_batched<T>(const WorkList&, hipStream_t);                        \
  template void launch_coarse_batched<T>(const WorkList&, int, hipStream_t);                    \
  template void launch_fill_batched<T>(const WorkList&, hipStream_t);
MCW_INST(float)
MCW_INST(double)

template void launch_dot2_batched<float>(const WorkList&, hipStream_t);
template void launch_cg_direction_batched<float>(const WorkList&, hipStream_t);
template void launch_cg_update_batched<float>(const WorkList&, hipStream_t);
template void launch_neg_apply_dot_batched<float>(const WorkList&, hipStream_t, int, bool);
#undef MCW_INST

}  // namespace mcw
