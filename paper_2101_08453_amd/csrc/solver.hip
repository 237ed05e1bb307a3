// Host side of libmcwind: grid set-up (geometry check, fine stencil, coarse
// grid hierarchy, Galerkin operators, coarsest factorisation), the solve
// drivers (plain FP64 multigrid, and FP32 V-cycles inside FP64 iterative
// refinement), the adjoint, and the extern "C" entry points of mcwind.h.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <type_traits>
#include <sys/stat.h>
#include <unistd.h>

#include "mcw_internal.hpp"

using namespace mcw;

namespace {

thread_local std::string g_error;

struct Fail {
  static void arg(const std::string& m) { throw Error{MCW_INVALID_ARG, m}; }
};

void logf(const mcw_handle& h, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void logf(const mcw_handle& h, const char* fmt, ...) {
  if (!h.opt.verbose) return;
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "[mcwind] ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  va_end(ap);
}

// ---------------------------------------------------------------- hierarchy rule

// Counts of free nodes of a level.
size_t free_count(const Dims& d, const Faces& f) {
  auto cnt = [](int n, bool lo_fixed, bool hi_fixed) {
    return std::max(0, n - (lo_fixed ? 1 : 0) - (hi_fixed ? 1 : 0));
  };
  const size_t fx = cnt(d.NX(), f.x_fixed(0, d.NX()), f.x_fixed(d.NX() - 1, d.NX()));
  const size_t fy = cnt(d.NY(), f.y_fixed(0, d.NY()), f.y_fixed(d.NY() - 1, d.NY()));
  const int k0 = f.k_first(), k1 = f.k_last(d.NZ());
  const size_t fz = k1 >= k0 ? (size_t)(k1 - k0 + 1) : 0;
  return fx * fy * fz;
}

std::vector<int> keep_every_other(int n) {
  std::vector<int> k;
  for (int p = 0; p <= n; p += 2) k.push_back(p);
  if (k.back() != n) k.push_back(n);
  return k;
}

std::vector<int> keep_all(int n) {
  std::vector<int> k(n + 1);
  for (int p = 0; p <= n; ++p) k[p] = p;
  return k;
}

DirMap make_map(int n, const std::vector<int>& keep) {
  DirMap m;
  m.nf = n + 1;
  m.nc = (int)keep.size();
  std::vector<int> idx(n + 1, -1);
  for (int c = 0; c < m.nc; ++c) idx[keep[c]] = c;
  m.lo.resize(n + 1);
  m.hi.resize(n + 1);
  for (int p = 0; p <= n; ++p) {
    if (idx[p] >= 0) {
      m.lo[p] = m.hi[p] = idx[p];
    } else {
      m.lo[p] = idx[p - 1];
      m.hi[p] = idx[p + 1];
    }
  }
  m.ctr = keep;
  m.slo.resize(m.nc);
  m.shi.resize(m.nc);
  for (int c = 0; c < m.nc; ++c) {
    const int p = keep[c];
    m.slo[c] = (p - 1 >= 0 && idx[p - 1] < 0) ? p - 1 : p;
    m.shi[c] = (p + 1 <= n && idx[p + 1] < 0) ? p + 1 : p;
  }
  return m;
}

// Geometry kept on the host for the coarsening decisions: the bottom planes of
// X and Y and all of Z, addressed through the fine indices a level keeps.
struct HostGeom {
  int NX0 = 0, NY0 = 0;
  std::vector<double> X0, Y0, Z;
};

struct LevelIdx {
  std::vector<int> kx, ky, kz;  // level nodes as fine-grid indices
};

void spacings(const HostGeom& g, const LevelIdx& li, double& h1, double& h2,
              std::vector<double>& h3) {
  const int nxl = (int)li.kx.size() - 1, nyl = (int)li.ky.size() - 1, nzl = (int)li.kz.size() - 1;
  double sx = 0.0, sy = 0.0;
  for (int j : li.ky) sx += g.X0[(size_t)j * g.NX0 + li.kx.back()] - g.X0[(size_t)j * g.NX0 + li.kx.front()];
  for (int i : li.kx) sy += g.Y0[(size_t)li.ky.back() * g.NX0 + i] - g.Y0[(size_t)li.ky.front() * g.NX0 + i];
  h1 = sx / ((double)nxl * li.ky.size());
  h2 = sy / ((double)nyl * li.kx.size());
  h3.assign(nzl, 0.0);
  const size_t plane = (size_t)g.NX0 * g.NY0;
  for (int k = 0; k < nzl; ++k) {
    const double* zb = g.Z.data() + (size_t)li.kz[k] * plane;
    const double* zt = g.Z.data() + (size_t)li.kz[k + 1] * plane;
    double s = 0.0;
    for (int j : li.ky) {
      const size_t row = (size_t)j * g.NX0;
      for (int i : li.kx) s += zt[row + i] - zb[row + i];
    }
    h3[k] = s / ((double)li.kx.size() * li.ky.size());
  }
}

// Sec. 3 coarsening decision for one level; false when the level is the coarsest.
bool decide(const mcw_handle& h, const Dims& d, const Faces& fc, double h1, double h2,
            const std::vector<double>& h3, bool& ch, std::vector<int>& keep_z) {
  if ((long long)free_count(d, fc) <= (long long)h.opt.coarse_direct_max) return false;
  const bool can_h = d.nx >= 3 && d.ny >= 3;
  const double hh = std::sqrt(h1 * h2);
  const double ah = std::sqrt(h.a[0] * h.a[1]);
  auto ratio = [&](double t, double hhor) {
    return h.opt.coarsen_rule == MCW_COARSEN_LITERAL ? ah * t / (hhor * h.a[2])
                                                     : h.a[2] * t / (ah * hhor);
  };
  keep_z.clear();
  if (h.opt.coarsen_rule == MCW_COARSEN_FULL) {
    ch = can_h;
    keep_z = keep_every_other(d.nz);
  } else {
    ch = can_h && ratio(h3[0], hh) > 1.0 / 3.0;
    const double hh2 = (ch && h.opt.merge_spacing == MCW_MERGE_COARSENED_SPACING) ? 2.0 * hh : hh;
    keep_z.push_back(0);
    int k = 0;
    while (k < d.nz) {
      if (k + 1 < d.nz && ratio(h3[k], hh2) < 3.0) {
        keep_z.push_back(k + 2);
        k += 2;
      } else {
        keep_z.push_back(k + 1);
        k += 1;
      }
    }
  }
  // a coarse level keeps a free node: with both z faces fixed, dropping every interior
  // plane would leave none, so then all planes are kept
  const Dims dc{ch ? (int)keep_every_other(d.nx).size() - 1 : d.nx,
                ch ? (int)keep_every_other(d.ny).size() - 1 : d.ny, (int)keep_z.size() - 1};
  if (free_count(dc, fc) == 0) keep_z = keep_all(d.nz);
  if (!ch && (int)keep_z.size() == d.nz + 1) {
    if (!can_h) return false;
    ch = true;
  }
  return true;
}

void upload_maps(Level& L, hipStream_t s) {
  const DirMap* ms[3] = {&L.mx, &L.my, &L.mz};
  size_t total = 0;
  for (auto* m : ms) total += 2 * (size_t)m->nf + 3 * (size_t)m->nc;
  std::vector<int> host;
  host.reserve(total);
  size_t off[3][5];
  for (int d = 0; d < 3; ++d) {
    const DirMap& m = *ms[d];
    off[d][0] = host.size(); host.insert(host.end(), m.lo.begin(), m.lo.end());
    off[d][1] = host.size(); host.insert(host.end(), m.hi.begin(), m.hi.end());
    off[d][2] = host.size(); host.insert(host.end(), m.ctr.begin(), m.ctr.end());
    off[d][3] = host.size(); host.insert(host.end(), m.slo.begin(), m.slo.end());
    off[d][4] = host.size(); host.insert(host.end(), m.shi.begin(), m.shi.end());
  }
  L.maps.alloc(host.size() * sizeof(int));
  MCW_HIP(hipMemcpyAsync(L.maps.p, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice, s));
  MCW_HIP(hipStreamSynchronize(s));
  const int* base = L.maps.as<int>();
  DirMapDev* dm[3] = {&L.dmx, &L.dmy, &L.dmz};
  for (int d = 0; d < 3; ++d) {
    dm[d]->lo = base + off[d][0];
    dm[d]->hi = base + off[d][1];
    dm[d]->ctr = base + off[d][2];
    dm[d]->slo = base + off[d][3];
    dm[d]->shi = base + off[d][4];
  }
}

// ---------------------------------------------------------------- coarsest level

// Dense FP64 inverse of the coarsest operator on its free nodes (Cholesky).
void factor_coarsest(mcw_handle& h) {
  Level& L = h.levels.back();
  const Dims d = L.d;
  const size_t N = d.N();
  const StLayout SL = d.layout();
  std::vector<double> st(SW * SL.nodes);
  MCW_HIP(hipMemcpyAsync(st.data(), L.st64.p, st.size() * sizeof(double), hipMemcpyDeviceToHost,
                         h.stream));
  MCW_HIP(hipStreamSynchronize(h.stream));
  const int NX = d.NX(), NY = d.NY(), NZ = d.NZ();
  std::vector<int> pos(N, -1), idx, split_idx;  // natural and row-split node numbers
  const int k0 = h.faces.k_first(), k1 = h.faces.k_last(NZ);
  for (int k = 0; k < NZ; ++k)
    for (int j = 0; j < NY; ++j)
      for (int i = 0; i < NX; ++i) {
        if (h.faces.x_fixed(i, NX) || h.faces.y_fixed(j, NY) || k < k0 || k > k1) continue;
        const size_t n = (size_t)i + (size_t)NX * (j + (size_t)NY * k);
        pos[n] = (int)idx.size();
        idx.push_back((int)n);
        const int NXe = (NX + 1) >> 1;
        split_idx.push_back((int)(n - i + ((i & 1) ? NXe + (i >> 1) : (i >> 1))));
      }
  const int n = (int)idx.size();
  h.n_coarse = n;
  if (n == 0) return;  // every node is fixed: lambda = 0 and no level has anything to solve
  std::vector<double> A((size_t)n * n, 0.0);
  for (int r = 0; r < n; ++r) {
    const size_t nd = (size_t)idx[r];
    const int i = (int)(nd % NX), j = (int)((nd / NX) % NY), k = (int)(nd / ((size_t)NX * NY));
    const size_t sp = SL.node(i, j, k);
    for (int o = 0; o < 27; ++o) {
      const int ii = i + o % 3 - 1, jj = j + (o / 3) % 3 - 1, kk = k + o / 9 - 1;
      if (ii < 0 || ii >= NX || jj < 0 || jj >= NY || kk < 0 || kk >= NZ) continue;
      const int q = pos[(size_t)ii + (size_t)NX * (jj + (size_t)NY * kk)];
      if (q < 0) continue;
      A[(size_t)r * n + q] += st[st_entry<double>(sp, o)];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int q = r + 1; q < n; ++q) {
      const double s = 0.5 * (A[(size_t)r * n + q] + A[(size_t)q * n + r]);
      A[(size_t)r * n + q] = A[(size_t)q * n + r] = s;
    }
  // Cholesky A = L L^T, L stored in the lower triangle (row major)
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    const double* lj = &A[(size_t)j * n];
    for (int k = 0; k < j; ++k) s -= lj[k] * lj[k];
    if (!(s > 0.0)) throw Error{MCW_SINGULAR, "coarsest operator is not positive definite"};
    const double djj = std::sqrt(s);
    A[(size_t)j * n + j] = djj;
    for (int i = j + 1; i < n; ++i) {
      double* li = &A[(size_t)i * n];
      double t = li[j];
      for (int k = 0; k < j; ++k) t -= li[k] * lj[k];
      li[j] = t / djj;
    }
  }
  // W = L^{-1} (lower), stored transposed: Wt[c][r] = W[r][c] for r >= c
  std::vector<double> Wt((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    double* w = &Wt[(size_t)c * n];  // column c of W
    w[c] = 1.0 / A[(size_t)c * n + c];
    for (int r = c + 1; r < n; ++r) {
      const double* lr = &A[(size_t)r * n];
      double t = 0.0;
      for (int k = c; k < r; ++k) t -= lr[k] * w[k];
      w[r] = t / lr[r];
    }
  }
  // inverse = W^T W: inv[a][b] = sum_{r >= max(a,b)} W[r][a] W[r][b]
  std::vector<double> inv((size_t)n * n);
  for (int a = 0; a < n; ++a) {
    const double* wa = &Wt[(size_t)a * n];
    for (int b = a; b < n; ++b) {
      const double* wb = &Wt[(size_t)b * n];
      double t = 0.0;
      for (int r = b; r < n; ++r) t += wa[r] * wb[r];
      inv[(size_t)a * n + b] = inv[(size_t)b * n + a] = t;
    }
  }
  h.coarse_inv.alloc(inv.size() * sizeof(double));
  h.coarse_idx.alloc(split_idx.size() * sizeof(int));
  MCW_HIP(hipMemcpyAsync(h.coarse_inv.p, inv.data(), inv.size() * sizeof(double),
                         hipMemcpyHostToDevice, h.stream));
  MCW_HIP(hipMemcpyAsync(h.coarse_idx.p, split_idx.data(), split_idx.size() * sizeof(int),
                         hipMemcpyHostToDevice, h.stream));
  MCW_HIP(hipStreamSynchronize(h.stream));
}

// ---------------------------------------------------------------- reductions

// Sum `width` channels of per-block partials into h.scalars and return them on the host.
void reduce_to_host(mcw_handle& h, size_t n_part, int width, double* out) {
  launch_sum_partials(h.partials.as<double>(), n_part, width, h.scalars.as<double>(), h.stream);
  MCW_HIP(hipMemcpyAsync(h.host_scalars, h.scalars.p, width * sizeof(double), hipMemcpyDeviceToHost,
                         h.stream));
  MCW_HIP(hipStreamSynchronize(h.stream));
  for (int w = 0; w < width; ++w) out[w] = h.host_scalars[w];
}

// ---------------------------------------------------------------- V-cycle

// The stencil the V-cycle of precision T uses on level L: FP64, FP32, or FP16
// scaled by 1/st_scale (option stencil_fp16).
template <class T> StRef stencil_of(const Level& L);
template <> StRef stencil_of<double>(const Level& L) { return StRef(L.st64.p); }
template <> StRef stencil_of<float>(const Level& L) {
  if (!L.st16.p) return StRef(L.st32.p);
  StRef r(L.st16.p);
  r.h16 = 1;
  r.sc = L.st_scale;
  r.isc = 1.f / L.st_scale;
  return r;
}

// Scratch of the vertical line smoother (the level's residual vector, idle
// while smoothing), or null for the point smoother.
template <class T>
T* line_buf(const mcw_handle& h, Level& L) {
  return h.opt.smoother == MCW_SMOOTH_LINE ? L.r.as<T>() : nullptr;
}

template <class T>
void vcycle(mcw_handle& h, int l, T* x, const T* f) {
  Level& L = h.levels[l];
  if (l == (int)h.levels.size() - 1) {
    // no free node (every node fixed): nothing to solve
    if (h.n_coarse > 0)
      launch_coarse_solve<T>(h.n_coarse, h.coarse_inv.as<double>(), h.coarse_idx.as<int>(), f, x,
                             h.stream);
    return;
  }
  const StRef st = stencil_of<T>(L);
  // the last pre-smoothing sweep leaves the residual of the columns whose
  // residual it knows (its last colour, or every odd row) behind
  const int nu = h.opt.nu_pre;
  int known = 0;
  for (int s = 0; s < nu; ++s)
    known = launch_smooth_sweep<T>(L.d, h.faces, st, f, x, h.stream, L.by_gs, false, line_buf<T>(h, L),
                                   s == nu - 1 ? L.r.as<T>() : nullptr);
  launch_residual<T>(L.d, h.faces, st, x, f, L.r.as<T>(), nullptr, nullptr, h.stream, L.by_res, 0,
                     known);
  Level& C = h.levels[l + 1];
  launch_restrict<T>(L.d, C.d, h.faces, L.dmx, L.dmy, L.dmz, L.r.as<T>(), C.f.as<T>(), h.stream);
  launch_fill<T>(C.x.as<T>(), C.d.N(), T(0), h.stream);
  vcycle<T>(h, l + 1, C.x.as<T>(), C.f.as<T>());
  launch_prolong_dims<T>(L.d, C.d, h.faces, L.dmx, L.dmy, L.dmz, C.x.as<T>(), x, h.stream);
  // with krylov the post-smoother is the adjoint of the pre-smoother, so the cycle is symmetric
  for (int s = 0; s < h.opt.nu_post; ++s)
    launch_smooth_sweep<T>(L.d, h.faces, st, f, x, h.stream, L.by_gs, h.opt.krylov != 0, line_buf<T>(h, L));
}

// Run `record` on h.stream, or, with use_graph, replay the hipGraph it was
// captured into on the first call (the buffers it touches are fixed per handle).
template <class F>
void replay(mcw_handle& h, hipGraphExec_t& exec, bool& ready, F&& record) {
  if (!h.opt.use_graph) {
    record();
    return;
  }
  if (!ready) {
    hipGraph_t g = nullptr;
    MCW_HIP(hipStreamBeginCapture(h.stream, hipStreamCaptureModeThreadLocal));
    try {
      record();
    } catch (...) {
      (void)hipStreamEndCapture(h.stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    MCW_HIP(hipStreamEndCapture(h.stream, &g));
    const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    MCW_HIP(e);
    ready = true;
  }
  MCW_HIP(hipGraphLaunch(exec, h.stream));
}

// One FP32 V-cycle on the level-0 buffers, replayed from a hipGraph when enabled.
void vcycle_f32(mcw_handle& h) {
  Level& L0 = h.levels[0];
  replay(h, h.vgraph, h.vgraph_ready, [&] { vcycle<float>(h, 0, L0.x.as<float>(), L0.f.as<float>()); });
}

// ---------------------------------------------------------------- preconditioned CG

// Vectors of the inner CG solve of K e = r: r residual, z = B r (B one
// symmetric V-cycle from zero), p direction, q = -K p, e correction.
template <class T>
struct Krylov {
  T *r, *z, *p, *q, *e;
};

template <class T>
Krylov<T> krylov_vecs(mcw_handle& h) {
  Level& L0 = h.levels[0];
  if (std::is_same<T, float>::value)
    return {L0.f.as<T>(), L0.x.as<T>(), h.kp.as<T>(), h.kq.as<T>(), h.ke.as<T>()};
  return {h.kr.as<T>(), h.kz.as<T>(), h.kp.as<T>(), h.kq.as<T>(), h.ke.as<T>()};
}

// One CG step; the coefficients stay on the device (scalars 8..10), so the
// step is a fixed launch sequence without host synchronisation.
template <class T>
void pcg_step(mcw_handle& h, const Krylov<T>& v) {
  Level& L0 = h.levels[0];
  const size_t N = L0.d.N();
  double* sc = h.scalars.as<double>() + 8;
  double* part = h.partials.as<double>();
  launch_fill<T>(v.z, N, T(0), h.stream);
  vcycle<T>(h, 0, v.z, v.r);
  launch_cg_beta<T>(v.z, v.r, v.q, N, part, h.n_partials, sc, h.stream);
  launch_cg_direction<T>(v.p, v.z, sc, N, h.stream);
  size_t np = 0;
  launch_neg_apply_dot<T>(L0.d, h.faces, stencil_of<T>(L0), v.p, v.q, part, h.n_partials, &np,
                          h.stream, L0.by_res);
  launch_cg_alpha(np, part, sc, h.stream);
  launch_cg_update<T>(v.e, v.p, v.r, v.q, sc, N, part, h.n_partials, h.stream);
}

// CG steps from e = 0 on the residual in v.r (overwritten): at most m_max, and
// with rr_stop > 0 only until the recursive r.r falls to rr_stop (read back
// after every step; one V-cycle outweighs the synchronisation by far).
// Returns the number of steps taken.
template <class T>
int pcg_inner(mcw_handle& h, const Krylov<T>& v, int m_max, double rr_stop) {
  double* sc = h.scalars.as<double>() + 8;
  launch_cg_reset(sc, h.stream);
  launch_fill<T>(v.e, h.levels[0].d.N(), T(0), h.stream);
  int c = 0;
  while (c < m_max) {
    replay(h, h.kgraph, h.kgraph_ready, [&] { pcg_step<T>(h, v); });
    ++c;
    if (rr_stop > 0.0) {
      MCW_HIP(hipMemcpyAsync(h.host_scalars + 3, sc + 3, sizeof(double), hipMemcpyDeviceToHost,
                             h.stream));
      MCW_HIP(hipStreamSynchronize(h.stream));
      const double rr = h.host_scalars[3];
      if (!(rr > rr_stop)) break;  // reached, or not finite (the outer residual reports it)
    }
  }
  return c;
}

// Steps for the next inner solve: enough to reduce the residual by `target`
// at the measured rate, within [1, cap].
// At most this many FP32 V-cycles per refinement step: enough for the 3e-5
// reduction an FP32 inner solve is asked for at rates up to about 0.6 (18 at
// 0.55), so that a slow solve needs no extra FP64 residual evaluations.
constexpr int kMaxInnerCycles = 20;

// The smallest reduction of the true residual one refinement step is asked for:
// what the V-cycle's operator resolves.  FP32 stencils: 3e-5.  FP16 stencils
// perturb the operator by about 1e-4 relative per coefficient, and one step
// then reduces the FP64 residual by about 1e-3 at best, however many V-cycles
// it runs (measured with the oracle's multigrid on a 64x64x15 fractal grid).
double inner_floor(const mcw_handle& h) { return h.opt.stencil_fp16 ? 1e-3 : 3e-5; }

int inner_steps(double target, double rho, int cap) {
  const int m = (int)std::ceil(std::log(target) / std::log(rho));
  return std::max(1, std::min(m, cap));
}

// Cycles of a refinement step before the handle's V-cycle rate is known: the
// FP64 residual after them measures it.
constexpr int kProbeCycles = 3;

// Cycles of the next FP32 refinement step at relative residual rel: enough to
// reach the tolerance at the rate rho (0 = not measured yet), but no further
// than the FP32 operator resolves.  *aimed_floor tells whether that floor, not
// the tolerance, set the target.
int step_cycles(const mcw_handle& h, double rho, double rel, bool* aimed_floor) {
  const double floor = inner_floor(h);
  *aimed_floor = h.opt.rtol / rel <= floor;
  if (h.opt.inner_cycles > 0) return h.opt.inner_cycles;
  if (!(rho > 0.0)) return kProbeCycles;
  return inner_steps(std::max(h.opt.rtol / rel, floor), rho, kMaxInnerCycles);
}

// The rate after a step of m cycles that reduced the FP64 residual by red.  A
// step aimed at the FP32 floor may have been limited by it rather than by the
// cycle, so its reduction can only raise a known estimate.
double update_rate(double rho, double red, int m, bool aimed_floor) {
  const double r = std::min(0.95, std::max(0.02, std::pow(std::max(red, 1e-300), 1.0 / m)));
  if (!(rho > 0.0) || !aimed_floor || r > rho) return r;
  return rho;
}

// The FP32 V-cycle's rate on the handle's operator: from a fixed pseudo-random
// right-hand side and x = 0, the FP32 residual norm after the first and after
// the fourth cycle, (r4 / r1)^(1/3).  Four cycles keep the reduction well above
// what the FP32 (or FP16) operator resolves at the rates met here.  Measured
// once at set-up, so that every solve on the handle runs the same cycle
// schedule for the same input.
constexpr int kRateCycles = 4;

double measure_rate(mcw_handle& h) {
  if (h.levels.size() < 2) return 0.02;  // one level: the cycle is the direct solve
  Level& L0 = h.levels[0];
  const size_t N = h.d.N();
  launch_hash_fill(h.r64.as<double>(), N, 0x6d63776eull, h.stream);
  h.host_scalars[7] = 1.0;
  double* scale_dev = h.scalars.as<double>() + 7;
  MCW_HIP(hipMemcpyAsync(scale_dev, &h.host_scalars[7], sizeof(double), hipMemcpyHostToDevice,
                         h.stream));
  launch_scale_to_f32(h.d, h.r64.as<double>(), scale_dev, L0.f.as<float>(), h.stream);
  launch_fill<float>(L0.x.as<float>(), N, 0.f, h.stream);
  double rn[2] = {0.0, 0.0};
  for (int c = 1; c <= kRateCycles; ++c) {
    vcycle_f32(h);
    if (c != 1 && c != kRateCycles) continue;
    size_t np = 0;
    launch_residual<float>(L0.d, h.faces, stencil_of<float>(L0), L0.x.as<float>(), L0.f.as<float>(),
                           L0.r.as<float>(), h.partials.as<double>(), &np, h.stream, L0.by_res,
                           h.n_partials);
    reduce_to_host(h, np, 1, &rn[c == 1 ? 0 : 1]);
  }
  if (!(rn[0] > 0.0) || !std::isfinite(rn[1])) return 0.0;
  const double r = std::pow(std::sqrt(rn[1] / rn[0]), 1.0 / (kRateCycles - 1));
  return std::min(0.95, std::max(0.02, r));
}

// ---------------------------------------------------------------- solve drivers

struct Progress {
  int outer = 0, cycles = 0;
  double rel = 0.0;
  std::vector<double> hist;
  float ms_outer = 0.f;
};

// Solve K lam = h.f64 (free nodes) from the starting lam; fnorm = ||f||.
mcw_status iterate(mcw_handle& h, double* lam, double fnorm, Progress& pg) {
  Level& L0 = h.levels[0];
  const size_t N = h.d.N();
  const double tol = h.opt.rtol;
  size_t np = 0;
  double rr = 0.0;
  if (h.opt.precision == MCW_FP64) {
    // the V-cycle works on row-split copies of lambda and f
    double* x0 = L0.x.as<double>();
    double* f0 = L0.f.as<double>();
    launch_relayout<double>(h.d, lam, x0, true, h.stream);
    launch_relayout<double>(h.d, h.f64.as<double>(), f0, true, h.stream);
    const Krylov<double> kv = krylov_vecs<double>(h);
    double prev_rel = -1.0;
    mcw_status st = MCW_OK;
    for (;;) {
      // with krylov the residual is the right-hand side of the next inner CG solve
      launch_residual<double>(L0.d, h.faces, L0.st64.as<double>(), x0, f0,
                              h.opt.krylov ? kv.r : L0.r.as<double>(), h.partials.as<double>(), &np,
                              h.stream, L0.by_res, h.n_partials);
      reduce_to_host(h, np, 1, &rr);
      pg.rel = std::sqrt(rr) / fnorm;
      pg.hist.push_back(pg.rel);
      ++pg.outer;
      logf(h, "fp64 cycle %d  rel residual %.3e", pg.cycles, pg.rel);
      if (!std::isfinite(pg.rel)) { st = MCW_NONFINITE; break; }
      if (pg.rel <= tol) break;
      if (pg.cycles >= h.opt.max_cycles) { st = MCW_NOT_CONVERGED; break; }
      if (!h.opt.krylov) {
        vcycle<double>(h, 0, x0, f0);
        ++pg.cycles;
        continue;
      }
      // an inner solve that no longer reduces the true residual has stagnated
      if (prev_rel > 0.0 && pg.rel > 0.95 * prev_rel) { st = MCW_NOT_CONVERGED; break; }
      // fixed inner_cycles, or until the recursive residual is half the tolerance
      const int m_max = std::min(h.opt.inner_cycles > 0 ? h.opt.inner_cycles : 100,
                                 h.opt.max_cycles - pg.cycles);
      const double stop = h.opt.inner_cycles > 0 ? 0.0 : 0.5 * tol * fnorm;
      const int m = pcg_inner<double>(h, kv, m_max, stop * stop);
      launch_add<double>(x0, kv.e, N, h.stream);
      pg.cycles += m;
      prev_rel = pg.rel;
    }
    launch_relayout<double>(h.d, x0, lam, false, h.stream);
    return st;
  }
  // FP32 V-cycles inside FP64 iterative refinement; the V-cycle rate measured
  // at set-up sets the first cycle count, the solve's own steps the later ones
  double rho_est = h.rho_setup, prev_rel = -1.0;
  int prev_m = 0, stall = 0;
  bool prev_floor = false;
  const double nfree = (double)std::max<size_t>(free_count(h.d, h.faces), 1);
  for (;;) {
    MCW_HIP(hipEventRecord(h.ev[4], h.stream));
    launch_apply(h, lam, h.f64.as<double>(), h.r64.as<double>(), 1, h.partials.as<double>(), &np);
    MCW_HIP(hipEventRecord(h.ev[5], h.stream));
    reduce_to_host(h, np, 1, &rr);
    float ms = 0.f;
    MCW_HIP(hipEventElapsedTime(&ms, h.ev[4], h.ev[5]));
    pg.ms_outer += ms;
    pg.rel = std::sqrt(rr) / fnorm;
    pg.hist.push_back(pg.rel);
    ++pg.outer;
    logf(h, "refine step %d after %d cycles  rel residual %.3e", pg.outer, pg.cycles, pg.rel);
    if (!std::isfinite(pg.rel)) return MCW_NONFINITE;
    if (prev_rel > 0.0 && prev_m > 0 && !h.opt.krylov)
      rho_est = update_rate(rho_est, pg.rel / prev_rel, prev_m, prev_floor);
    if (pg.rel <= tol) return MCW_OK;
    if (pg.cycles >= h.opt.max_cycles) return MCW_NOT_CONVERGED;
    if (prev_rel > 0.0 && prev_m > 0) {
      if (pg.rel / prev_rel > 0.95) {
        if (++stall >= 3) return MCW_NOT_CONVERGED;
      } else {
        stall = 0;
      }
    }
    // reduce to the tolerance in one step, but not below what FP32 can resolve.
    // (Aiming lower, at half the tolerance, trades a refinement step of one FP64
    // residual for an extra V-cycle, which costs about four times as much.)
    int m = step_cycles(h, rho_est, pg.rel, &prev_floor);
    m = std::min(m, h.opt.max_cycles - pg.cycles);
    // scale the residual by a power of two to O(1) before rounding it to FP32
    const double rms = std::sqrt(rr / nfree);
    h.host_scalars[7] = std::ldexp(1.0, -std::ilogb(rms));
    double* scale_dev = h.scalars.as<double>() + 7;
    MCW_HIP(hipMemcpyAsync(scale_dev, &h.host_scalars[7], sizeof(double), hipMemcpyHostToDevice,
                           h.stream));
    launch_scale_to_f32(h.d, h.r64.as<double>(), scale_dev, L0.f.as<float>(), h.stream);
    if (h.opt.krylov) {
      // until the scaled FP32 residual has dropped by the same target as above
      const Krylov<float> kv = krylov_vecs<float>(h);
      const double target = std::max(tol / pg.rel, inner_floor(h));
      const double r0 = std::sqrt(rr) * h.host_scalars[7];
      const int m_max = std::min(h.opt.inner_cycles > 0 ? h.opt.inner_cycles : 30,
                                 h.opt.max_cycles - pg.cycles);
      const double stop = h.opt.inner_cycles > 0 ? 0.0 : target * r0;
      m = pcg_inner<float>(h, kv, m_max, stop * stop);
      launch_update_lambda(h.d, kv.e, scale_dev, lam, h.stream);
    } else {
      launch_fill<float>(L0.x.as<float>(), N, 0.f, h.stream);
      for (int c = 0; c < m; ++c) vcycle_f32(h);
      launch_update_lambda(h.d, L0.x.as<float>(), scale_dev, lam, h.stream);
    }
    pg.cycles += m;
    prev_m = m;
    prev_rel = pg.rel;
  }
}

void fill_info(const mcw_handle& h, const Progress& pg, mcw_info* info) {
  if (!info) return;
  info->outer_steps = pg.outer;
  info->cycles = pg.cycles;
  info->rel_residual = pg.rel;
  info->n_levels = (int)h.levels.size();
  for (int l = 0; l < info->n_levels && l < MCW_MAX_LEVELS; ++l) {
    info->level_dims[l][0] = h.levels[l].d.nx;
    info->level_dims[l][1] = h.levels[l].d.ny;
    info->level_dims[l][2] = h.levels[l].d.nz;
  }
  info->n_history = (int)std::min<size_t>(pg.hist.size(), MCW_HISTORY);
  for (int i = 0; i < info->n_history; ++i) info->history[i] = pg.hist[i];
  info->rho = 0.0;
  if (pg.cycles > 0 && !pg.hist.empty() && pg.hist.front() > 0.0 && pg.hist.back() > 0.0)
    info->rho = std::pow(pg.hist.back() / pg.hist.front(), 1.0 / pg.cycles);
  info->ms_outer = pg.ms_outer;
}

mcw_status solve_impl(mcw_handle& h, const double* u0, double* lam, double* u, mcw_info* info) {
  if (!u0 || !lam) Fail::arg("u0 and lambda must be non-null");
  if (info) std::memset(info, 0, sizeof(*info));
  const size_t N = h.d.N();
  const size_t E = (size_t)h.d.nx * h.d.ny * h.d.nz;
  MCW_HIP(hipEventRecord(h.ev[0], h.stream));
  launch_zero_fixed(h.d, h.faces, lam, h.stream);
  size_t np = 0;
  double ff = 0.0;
  launch_rhs(h, u0, h.f64.as<double>(), h.partials.as<double>(), &np);
  MCW_HIP(hipEventRecord(h.ev[1], h.stream));
  reduce_to_host(h, np, 1, &ff);
  const double fnorm = std::sqrt(ff);
  Progress pg;
  mcw_status st = MCW_OK;
  if (!std::isfinite(fnorm)) {
    st = MCW_NONFINITE;
    h.last_error = "non-finite right-hand side (check u0)";
  } else if (fnorm == 0.0) {
    launch_fill<double>(lam, N, 0.0, h.stream);
  } else {
    st = iterate(h, lam, fnorm, pg);
    if (st == MCW_NOT_CONVERGED)
      h.last_error = "not converged: relative residual " + std::to_string(pg.rel);
    if (st == MCW_NONFINITE) h.last_error = "non-finite residual";
  }
  MCW_HIP(hipEventRecord(h.ev[2], h.stream));
  double div[2] = {0.0, 0.0};
  if (st == MCW_OK || st == MCW_NOT_CONVERGED) {
    // one element-tile launch recovers u (when wanted) and checks the divergence
    launch_divergence(h, u0, lam, h.t64.as<double>(), h.partials.as<double>(), &np, u);
    reduce_to_host(h, np, 2, div);
  } else if (u) {
    MCW_HIP(hipMemcpyAsync(u, u0, 3 * E * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
  }
  MCW_HIP(hipEventRecord(h.ev[3], h.stream));
  MCW_HIP(hipEventSynchronize(h.ev[3]));
  if (info) {
    fill_info(h, pg, info);
    info->f_norm = fnorm;
    info->rel_divergence = div[1] > 0.0 ? std::sqrt(div[0] / div[1]) : std::sqrt(div[0]);
    float t = 0.f;
    MCW_HIP(hipEventElapsedTime(&t, h.ev[0], h.ev[3])); info->ms_total = t;
    MCW_HIP(hipEventElapsedTime(&t, h.ev[0], h.ev[1])); info->ms_rhs = t;
    MCW_HIP(hipEventElapsedTime(&t, h.ev[1], h.ev[2])); info->ms_cycles = t - pg.ms_outer;
    MCW_HIP(hipEventElapsedTime(&t, h.ev[2], h.ev[3])); info->ms_finish = t;
    info->status = st;
  }
  return st;
}

// ---------------------------------------------------------------- tile-shape autotuner

// Cache of tuned tile rows, one `"key": rows` pair per line of a JSON object.
class TuneCache {
 public:
  explicit TuneCache(const std::string* given) {
    const char* env = std::getenv("MCW_TUNE_CACHE");
    if (given) {
      path_ = *given;  // "" = no cache
      if (path_.empty()) return;
    } else if (env && *env) {
      path_ = env;
    } else if (const char* home = std::getenv("HOME")) {
      const std::string dir = std::string(home) + "/.cache/mcwind";
      (void)mkdir((std::string(home) + "/.cache").c_str(), 0755);
      (void)mkdir(dir.c_str(), 0755);
      path_ = dir + "/tune.json";
    }
    std::ifstream in(path_);
    std::string line;
    while (std::getline(in, line)) {
      const size_t a = line.find('"'), b = line.find('"', a + 1), c = line.find(':', b + 1);
      if (a == std::string::npos || b == std::string::npos || c == std::string::npos) continue;
      m_[line.substr(a + 1, b - a - 1)] = std::atoi(line.c_str() + c + 1);
    }
  }
  bool get(const std::string& k, int& v) const {
    auto it = m_.find(k);
    if (it == m_.end()) return false;
    v = it->second;
    return true;
  }
  void put(const std::string& k, int v) {
    m_[k] = v;
    dirty_ = true;
  }
  void save() {
    if (!dirty_ || path_.empty()) return;
    const std::string tmp = path_ + ".tmp" + std::to_string(getpid());
    {
      std::ofstream out(tmp);
      if (!out) return;
      out << "{\n";
      size_t i = 0;
      for (auto& kv : m_) out << "  \"" << kv.first << "\": " << kv.second << (++i < m_.size() ? ",\n" : "\n");
      out << "}\n";
    }
    (void)std::rename(tmp.c_str(), path_.c_str());
  }

 private:
  std::string path_;
  std::map<std::string, int> m_;
  bool dirty_ = false;
};

// Where a level's stencil and vectors sit in physical memory moves its
// colour pass and residual by up to about 15 %: at 3000 x 3000 x 15 the same
// buffers in different allocations took 2.70-3.22 ms per sweep and 2.89-3.45
// ms per residual, each allocation keeping its speed, and neither the virtual
// addresses nor fixed offsets inside one allocation predicted it.  So set-up
// times a few placements of every level with at least 2^22 nodes (fresh
// allocations, the stencil copied over) and keeps the fastest; all placements
// give the same results.  Rejected placements are held until the level's
// probing ends, so that every trial gets new memory, and probing stops early
// when free memory runs short.
constexpr int kPlacementTrials = 6;

template <class T>
void probe_placement(mcw_handle& h, size_t l) {
  if (l + 1 >= h.levels.size()) return;  // the coarsest level has no smoother
  Level& L = h.levels[l];
  const size_t n = L.d.N();
  if (n < ((size_t)1 << 22)) return;
  DevBuf& st = L.st16.p ? L.st16 : (L.st32.p ? L.st32 : L.st64);
  const size_t vb = n * sizeof(T), need = st.bytes + 3 * vb;
  const int nu = std::max(1, h.opt.nu_pre + h.opt.nu_post);
  auto timed = [&](auto&& fn) {
    fn();
    MCW_HIP(hipEventRecord(h.ev[6], h.stream));
    for (int r = 0; r < 3; ++r) fn();
    MCW_HIP(hipEventRecord(h.ev[7], h.stream));
    MCW_HIP(hipEventSynchronize(h.ev[7]));
    float ms = 0.f;
    MCW_HIP(hipEventElapsedTime(&ms, h.ev[6], h.ev[7]));
    return ms / 3;
  };
  // one V-cycle's work on this level: nu sweeps and one residual
  auto cost = [&](float* sweep_ms, float* res_ms) {
    launch_fill<T>(L.f.as<T>(), n, T(0), h.stream);
    launch_fill<T>(L.x.as<T>(), n, T(0), h.stream);
    const StRef sr = stencil_of<T>(L);
    *sweep_ms = timed([&] {
      launch_smooth_sweep<T>(L.d, h.faces, sr, L.f.as<T>(), L.x.as<T>(), h.stream, L.by_gs, false,
                             line_buf<T>(h, L));
    });
    *res_ms = timed([&] {
      launch_residual<T>(L.d, h.faces, sr, L.x.as<T>(), L.f.as<T>(), L.r.as<T>(), nullptr, nullptr,
                         h.stream, L.by_res);
    });
    return nu * *sweep_ms + *res_ms;
  };
  float sw = 0.f, rs = 0.f;
  float best = cost(&sw, &rs);
  std::string log = std::to_string(sw).substr(0, 5) + "/" + std::to_string(rs).substr(0, 5);
  std::vector<DevBuf> held;
  for (int t = 1; t < kPlacementTrials; ++t) {
    size_t free_b = 0, total_b = 0;
    MCW_HIP(hipMemGetInfo(&free_b, &total_b));
    if (free_b < 2 * need + ((size_t)4 << 30)) break;
    DevBuf s2, x2, f2, r2;
    try {
      s2.alloc(st.bytes);
      x2.alloc(vb);
      f2.alloc(vb);
      r2.alloc(vb);
    } catch (const Error& e) {
      if (e.status != MCW_OOM) throw;
      (void)hipGetLastError();  // a failed trial only ends the probing
      break;
    }
    MCW_HIP(hipMemcpyAsync(s2.p, st.p, st.bytes, hipMemcpyDeviceToDevice, h.stream));
    std::swap(st, s2);
    std::swap(L.x, x2);
    std::swap(L.f, f2);
    std::swap(L.r, r2);
    const float c = cost(&sw, &rs);
    log += " " + std::to_string(sw).substr(0, 5) + "/" + std::to_string(rs).substr(0, 5);
    if (c < best) {
      best = c;
    } else {
      std::swap(st, s2);
      std::swap(L.x, x2);
      std::swap(L.f, f2);
      std::swap(L.r, r2);
    }
    held.push_back(std::move(s2));
    held.push_back(std::move(x2));
    held.push_back(std::move(f2));
    held.push_back(std::move(r2));
  }
  MCW_HIP(hipStreamSynchronize(h.stream));
  launch_fill<T>(L.x.as<T>(), n, T(0), h.stream);
  logf(h, "level %zu placements, ms per sweep/residual: %s; kept %.3f ms per cycle", l, log.c_str(), best);
}

// Time rows-per-block candidates of the colour pass and the residual on every
// level large enough for the shape to matter, on the level's own buffers.
template <class T>
void autotune_levels(mcw_handle& h) {
  hipDeviceProp_t prop;
  MCW_HIP(hipGetDeviceProperties(&prop, h.device));
  const std::string arch = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':'));
  TuneCache cache(h.tune_cache_set ? &h.tune_cache : nullptr);
  // colour pass: 0 = fused two-colour pass (one block per row), or 1, 2, 4 rows
  // of 64 columns per block of the four separate passes; residual: 1, 2, 4 rows
  const std::vector<int> cand_gs = {0, 1, 2, 4}, cand_res = {1, 2, 4};
  for (auto& L : h.levels) {
    if (L.d.N() < (size_t)1 << 16) continue;
    const std::string dims = std::to_string(L.d.NX()) + "x" + std::to_string(L.d.NY()) + "x" +
                             std::to_string(L.d.NZ()) +
                             (sizeof(T) == 8 ? "|f64" : (L.st16.p ? "|h16" : "|f32"));
    int v = 0;
    const std::string gs_key = arch + (h.opt.smoother == MCW_SMOOTH_LINE ? "|gsl|" : "|gsf|") + dims;
    const bool have_gs = cache.get(gs_key, v);
    if (have_gs) L.by_gs = v;
    const bool have_res = cache.get(arch + "|res|" + dims, v);
    if (have_res) L.by_res = v;
    if (have_gs && have_res) continue;
    launch_fill<T>(L.f.as<T>(), L.d.N(), T(0), h.stream);
    launch_fill<T>(L.x.as<T>(), L.d.N(), T(0), h.stream);
    const StRef st = stencil_of<T>(L);
    for (int which = 0; which < 2; ++which) {
      if ((which == 0 && have_gs) || (which == 1 && have_res)) continue;
      float best = 1e30f;
      int best_by = which == 0 ? 0 : 4;
      std::string times;
      for (int by : which == 0 ? cand_gs : cand_res) {
        auto run = [&] {
          if (which == 0)
            launch_smooth_sweep<T>(L.d, h.faces, st, L.f.as<T>(), L.x.as<T>(), h.stream, by, false,
                                   line_buf<T>(h, L));
          else
            launch_residual<T>(L.d, h.faces, st, L.x.as<T>(), L.f.as<T>(), L.r.as<T>(), nullptr, nullptr,
                               h.stream, by);
        };
        run();
        MCW_HIP(hipEventRecord(h.ev[6], h.stream));
        for (int r = 0; r < 3; ++r) run();
        MCW_HIP(hipEventRecord(h.ev[7], h.stream));
        MCW_HIP(hipEventSynchronize(h.ev[7]));
        float ms = 0.f;
        MCW_HIP(hipEventElapsedTime(&ms, h.ev[6], h.ev[7]));
        char buf[48];
        std::snprintf(buf, sizeof buf, " %d:%.3f", by, ms / 3);
        times += buf;
        if (ms < best) {
          best = ms;
          best_by = by;
        }
      }
      if (which == 0) {
        L.by_gs = best_by;
        cache.put(gs_key, best_by);
      } else {
        L.by_res = best_by;
        cache.put(arch + "|res|" + dims, best_by);
      }
      logf(h, "autotune %s %s: %d rows per block (0: fused rows); ms per %s:%s",
           which == 0 ? "gs" : "res", dims.c_str(), best_by, which == 0 ? "sweep" : "launch", times.c_str());
    }
  }
  cache.save();
}

// ---------------------------------------------------------------- set-up

void validate_grid(const mcw_grid_desc* g) {
  if (!g) Fail::arg("grid descriptor is null");
  if (!g->X || !g->Y || !g->Z) Fail::arg("node coordinate arrays must be non-null");
  if (g->nx < 2 || g->ny < 2 || g->nz < 1) Fail::arg("need nx >= 2, ny >= 2, nz >= 1");
  if ((long long)(g->nx + 1) * (g->ny + 1) > (1LL << 30) || g->nz > 4096)
    Fail::arg("grid too large");
  // element-column kernels launch ceil(ny / 4) blocks along y
  if (g->ny > 4 * 65535) Fail::arg("ny must be at most 262140");
  for (int d = 0; d < 3; ++d)
    if (!(g->a[d] > 0.0) || !std::isfinite(g->a[d])) Fail::arg("penalty constants must be finite and > 0");
  if (g->gamma_faces > 63u) Fail::arg("gamma_faces has bits beyond the six faces");
}

void validate(const mcw_grid_desc* g, const mcw_options& o) {
  validate_grid(g);
  if (o.precision != MCW_FP64 && o.precision != MCW_FP32_REFINE) Fail::arg("bad precision");
  if (!(o.rtol > 0.0) || !(o.rtol < 1.0)) Fail::arg("rtol must be in (0, 1)");
  if (o.max_cycles < 1 || o.nu_pre < 0 || o.nu_post < 0 || o.nu_pre + o.nu_post < 1)
    Fail::arg("bad cycle or smoothing counts");
  if (o.coarsen_rule < 0 || o.coarsen_rule > 2) Fail::arg("bad coarsening rule");
  if (o.coarse_direct_max < 1 || o.coarse_direct_max > 4096) Fail::arg("coarse_direct_max must be in [1, 4096]");
  if (o.krylov != 0 && o.krylov != 1) Fail::arg("krylov must be 0 or 1");
  if (o.krylov && o.nu_pre != o.nu_post) Fail::arg("krylov needs nu_pre == nu_post (a symmetric V-cycle)");
  if (o.smoother != MCW_SMOOTH_POINT && o.smoother != MCW_SMOOTH_LINE) Fail::arg("bad smoother");
  if (o.stencil_fp16 != 0 && o.stencil_fp16 != 1) Fail::arg("stencil_fp16 must be 0 or 1");
  if (o.stencil_fp16 && o.precision != MCW_FP32_REFINE)
    Fail::arg("stencil_fp16 needs precision FP32_REFINE");
  if (o.merge_spacing != MCW_MERGE_LEVEL_SPACING && o.merge_spacing != MCW_MERGE_COARSENED_SPACING)
    Fail::arg("bad merge_spacing");
}

void create_impl(const mcw_grid_desc* g, const mcw_options& opt, void* stream, mcw_handle& h) {
  validate(g, opt);
  if (g->gamma_faces == 63u)
    throw Error{MCW_SINGULAR, "Gamma covers every face: lambda is only defined up to a constant"};
  h.opt = opt;
  h.tune_cache_set = opt.tune_cache != nullptr;
  if (h.tune_cache_set) h.tune_cache = opt.tune_cache;
  h.opt.tune_cache = nullptr;  // the caller's string need not outlive this call
  MCW_HIP(hipGetDevice(&h.device));
  h.stream = static_cast<hipStream_t>(stream);
  if (!h.stream) {
    // a stream of our own (graph capture needs one); it synchronises with the default stream
    MCW_HIP(hipStreamCreate(&h.stream));
    h.own_stream = true;
  }
  h.d = Dims{g->nx, g->ny, g->nz};
  h.faces = Faces{g->gamma_faces};
  for (int d = 0; d < 3; ++d) {
    h.a[d] = g->a[d];
    h.c[d] = 1.0 / (g->a[d] * g->a[d]);
  }
  for (auto& e : h.ev) MCW_HIP(hipEventCreate(&e));
  const size_t N = h.d.N();
  h.X.alloc(N * sizeof(double));
  h.Y.alloc(N * sizeof(double));
  h.Z.alloc(N * sizeof(double));
  MCW_HIP(hipMemcpyAsync(h.X.p, g->X, N * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
  MCW_HIP(hipMemcpyAsync(h.Y.p, g->Y, N * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
  MCW_HIP(hipMemcpyAsync(h.Z.p, g->Z, N * sizeof(double), hipMemcpyDeviceToDevice, h.stream));

  // a1: geometry
  h.flag.alloc(sizeof(unsigned long long));
  const unsigned long long none = ~0ULL;
  MCW_HIP(hipMemcpyAsync(h.flag.p, &none, sizeof(none), hipMemcpyHostToDevice, h.stream));
  launch_geometry_check(h, h.flag.as<long long>());
  unsigned long long bad = 0;
  MCW_HIP(hipMemcpyAsync(&bad, h.flag.p, sizeof(bad), hipMemcpyDeviceToHost, h.stream));
  MCW_HIP(hipStreamSynchronize(h.stream));
  if (bad != none) {
    const unsigned long long nx = g->nx, ny = g->ny;
    throw Error{MCW_BAD_GEOMETRY, "det J <= 0 in element (" + std::to_string(bad % nx) + ", " +
                                      std::to_string((bad / nx) % ny) + ", " +
                                      std::to_string(bad / (nx * ny)) + ")"};
  }

  // terrain-following grids (x of a node depends on i only, y on j only) take
  // the element kernels' shorter path
  const int zero = 0;
  MCW_HIP(hipMemcpyAsync(h.flag.p, &zero, sizeof(zero), hipMemcpyHostToDevice, h.stream));
  launch_structure_check(h.X.as<double>(), h.Y.as<double>(), h.d, h.flag.as<int>(), h.stream);
  int not_tf = 1;
  MCW_HIP(hipMemcpyAsync(&not_tf, h.flag.p, sizeof(not_tf), hipMemcpyDeviceToHost, h.stream));
  MCW_HIP(hipStreamSynchronize(h.stream));
  h.terrain = not_tf == 0;
  logf(h, "terrain-following grid: %s", h.terrain ? "yes" : "no");

  // host geometry for the coarsening decisions
  HostGeom hg;
  hg.NX0 = h.d.NX();
  hg.NY0 = h.d.NY();
  const size_t plane = (size_t)hg.NX0 * hg.NY0;
  hg.X0.resize(plane);
  hg.Y0.resize(plane);
  hg.Z.resize(N);
  MCW_HIP(hipMemcpyAsync(hg.X0.data(), h.X.p, plane * sizeof(double), hipMemcpyDeviceToHost, h.stream));
  MCW_HIP(hipMemcpyAsync(hg.Y0.data(), h.Y.p, plane * sizeof(double), hipMemcpyDeviceToHost, h.stream));
  MCW_HIP(hipMemcpyAsync(hg.Z.data(), h.Z.p, N * sizeof(double), hipMemcpyDeviceToHost, h.stream));
  MCW_HIP(hipStreamSynchronize(h.stream));

  // a3: the hierarchy of logically Cartesian coarse grids
  LevelIdx li{keep_all(h.d.nx), keep_all(h.d.ny), keep_all(h.d.nz)};
  h.levels.clear();
  h.levels.emplace_back();
  h.levels[0].d = h.d;
  for (;;) {
    Level& L = h.levels.back();
    spacings(hg, li, L.h1, L.h2, L.h3);
    bool ch = false;
    std::vector<int> kz;
    if ((int)h.levels.size() >= MCW_MAX_LEVELS || !decide(h, L.d, h.faces, L.h1, L.h2, L.h3, ch, kz))
      break;
    L.coarsen_h = ch ? 1 : 0;
    L.keep_z = kz;
    const std::vector<int> kx = ch ? keep_every_other(L.d.nx) : keep_all(L.d.nx);
    const std::vector<int> ky = ch ? keep_every_other(L.d.ny) : keep_all(L.d.ny);
    L.mx = make_map(L.d.nx, kx);
    L.my = make_map(L.d.ny, ky);
    L.mz = make_map(L.d.nz, kz);
    LevelIdx nl;
    for (int p : kx) nl.kx.push_back(li.kx[p]);
    for (int p : ky) nl.ky.push_back(li.ky[p]);
    for (int p : kz) nl.kz.push_back(li.kz[p]);
    li = nl;
    Level C;
    C.d = Dims{(int)kx.size() - 1, (int)ky.size() - 1, (int)kz.size() - 1};
    h.levels.push_back(std::move(C));
  }
  hg = HostGeom();
  for (size_t l = 0; l + 1 < h.levels.size(); ++l) upload_maps(h.levels[l], h.stream);

  // a2 + a4: fine stencil by 2x2x2 Gauss, Galerkin coarse operators in FP64
  const bool f32 = opt.precision == MCW_FP32_REFINE;
  Level& L0 = h.levels[0];
  L0.st64.alloc(SW * h.d.layout().nodes * sizeof(double));
  launch_fill<double>(L0.st64.as<double>(), SW * h.d.layout().nodes, 0.0, h.stream);
  launch_assemble_stencil(h, L0.st64.as<double>());
  for (size_t l = 0; l < h.levels.size(); ++l) {
    Level& L = h.levels[l];
    if (l + 1 < h.levels.size()) {
      Level& C = h.levels[l + 1];
      C.st64.alloc(SW * C.d.layout().nodes * sizeof(double));
      launch_rap(L.d, C.d, L.dmx, L.dmy, L.dmz, L.st64.as<double>(), C.st64.as<double>(), h.stream);
    }
    if (f32 && opt.stencil_fp16) {
      // FP16 off-diagonals divided by a power of two at least the level's largest magnitude
      DevBuf scratch;
      scratch.alloc(1025 * sizeof(double));
      const double amax = stencil_absmax(L.d, L.st64.as<double>(), scratch.as<double>(), h.stream);
      const double scale = amax > 0.0 ? std::ldexp(1.0, std::ilogb(amax) + 1) : 1.0;
      L.st_scale = (float)scale;
      L.st16.alloc(SW16 * L.d.layout().nodes * sizeof(uint16_t));
      launch_round_stencil16(L.d, L.st64.as<double>(), L.st16.as<uint16_t>(), 1.0 / scale, h.stream);
    } else if (f32) {
      L.st32.alloc(SW32 * L.d.layout().nodes * sizeof(float));
      launch_round_stencil(L.d, L.st64.as<double>(), L.st32.as<float>(), h.stream);
    }
    if (f32) {
      if (l + 1 < h.levels.size()) {
        MCW_HIP(hipStreamSynchronize(h.stream));
        L.st64.release();
      }
    }
  }
  // a5: coarsest direct solve
  factor_coarsest(h);
  if (f32) h.levels.back().st64.release();

  // level vectors
  for (size_t l = 0; l < h.levels.size(); ++l) {
    Level& L = h.levels[l];
    const size_t n = L.d.N();
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    L.x.alloc(n * es);
    L.f.alloc(n * es);
    L.r.alloc(n * es);
    if (f32) launch_fill<float>(L.x.as<float>(), n, 0.f, h.stream);
    else launch_fill<double>(L.x.as<double>(), n, 0.0, h.stream);
  }
  h.f64.alloc(N * sizeof(double));
  h.r64.alloc(N * sizeof(double));
  h.t64.alloc(N * sizeof(double));
  {
    const Level& F = h.levels[0];
    const void* st = F.st32.p ? F.st32.p : (F.st16.p ? F.st16.p : F.st64.p);
    logf(h, "level 0 buffers: stencil %p x %p f %p r %p", st, F.x.p, F.f.p, F.r.p);
  }
  // per-block partial sums: the largest user is the element-tile grid (2 channels)
  const size_t tiles = (size_t)((h.d.NX() + 14) / 15) * ((h.d.NY() + 14) / 15);
  // fine-level column blocks at the smallest tile shape (one row of 64 columns)
  const size_t cols = (size_t)((h.d.NX() + 63) / 64) * h.d.NY();
  const size_t ecols = (size_t)((h.d.nx + 63) / 64) * ((h.d.ny + 3) / 4);
  h.n_partials = std::max({2 * tiles, cols, 3 * ecols, (size_t)4096});
  h.partials.alloc(h.n_partials * sizeof(double));
  if (opt.krylov) {
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    if (!f32) {
      h.kr.alloc(N * es);
      h.kz.alloc(N * es);
    }
    h.kp.alloc(N * es);
    h.kq.alloc(N * es);
    h.ke.alloc(N * es);
  }
  h.scalars.alloc(16 * sizeof(double));
  MCW_HIP(hipHostMalloc((void**)&h.host_scalars, 8 * sizeof(double), hipHostMallocDefault));
  if (opt.autotune) {
    for (size_t l = 0; l < h.levels.size(); ++l) {
      if (f32) probe_placement<float>(h, l);
      else probe_placement<double>(h, l);
    }
    if (f32) autotune_levels<float>(h);
    else autotune_levels<double>(h);
  }
  if (f32 && !opt.krylov) h.rho_setup = measure_rate(h);
  MCW_HIP(hipStreamSynchronize(h.stream));
  if (opt.verbose) {
    for (size_t l = 0; l < h.levels.size(); ++l) {
      const Level& L = h.levels[l];
      logf(h, "level %zu: %d x %d x %d elements, h1 %.3g, h3[0] %.3g, coarsen_h %d, planes kept %zu", l,
           L.d.nx, L.d.ny, L.d.nz, L.h1, L.h3.empty() ? 0.0 : L.h3[0], L.coarsen_h, L.keep_z.size());
    }
    logf(h, "coarsest free unknowns %d; V-cycle rate at set-up %.3f", h.n_coarse, h.rho_setup);
  }
}

void destroy_impl(mcw_handle* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  if (h->vgraph) (void)hipGraphExecDestroy(h->vgraph);
  if (h->kgraph) (void)hipGraphExecDestroy(h->kgraph);
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  if (h->host_scalars) (void)hipHostFree(h->host_scalars);
  const bool own = h->own_stream;
  hipStream_t s = h->stream;
  delete h;
  if (own && s) (void)hipStreamDestroy(s);
}

template <class F>
mcw_status guarded(mcw_handle* h, F&& fn) {
  try {
    return fn();
  } catch (const Error& e) {
    if (h) h->last_error = e.msg;
    g_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    if (h) h->last_error = "host allocation failed";
    g_error = "host allocation failed";
    return MCW_OOM;
  } catch (...) {
    if (h) h->last_error = "unexpected exception";
    g_error = "unexpected exception";
    return MCW_HIP_ERROR;
  }
}

Level& level_at(mcw_handle* h, int l, bool need_coarser) {
  if (l < 0 || l >= (int)h->levels.size() || (need_coarser && l + 1 >= (int)h->levels.size()))
    Fail::arg("level index out of range");
  return h->levels[l];
}

bool is_f32(const mcw_handle* h) { return h->opt.precision == MCW_FP32_REFINE; }

// Single-step entry points take natural-order vectors; the level buffers hold
// the row-split copies the kernels work on.
template <class T>
void smooth_t(mcw_handle& h, int l, T* x, const T* f, int sweeps) {
  Level& L = level_at(&h, l, false);
  launch_relayout<T>(L.d, x, L.x.as<T>(), true, h.stream);
  launch_relayout<T>(L.d, f, L.f.as<T>(), true, h.stream);
  const bool reverse = sweeps < 0;
  for (int s = 0; s < std::abs(sweeps); ++s)
    launch_smooth_sweep<T>(L.d, h.faces, stencil_of<T>(L), L.f.as<T>(), L.x.as<T>(), h.stream,
                           L.by_gs, reverse, line_buf<T>(h, L));
  launch_relayout<T>(L.d, L.x.as<T>(), x, false, h.stream);
}

template <class T>
void residual_t(mcw_handle& h, int l, const T* x, const T* f, T* r) {
  Level& L = level_at(&h, l, false);
  launch_relayout<T>(L.d, x, L.x.as<T>(), true, h.stream);
  launch_relayout<T>(L.d, f, L.f.as<T>(), true, h.stream);
  launch_residual<T>(L.d, h.faces, stencil_of<T>(L), L.x.as<T>(), L.f.as<T>(), L.r.as<T>(), nullptr,
                     nullptr, h.stream);
  launch_relayout<T>(L.d, L.r.as<T>(), r, false, h.stream);
}

template <class T>
void restrict_t(mcw_handle& h, int l, const T* r, T* rc) {
  Level& L = level_at(&h, l, true);
  Level& C = h.levels[l + 1];
  launch_relayout<T>(L.d, r, L.r.as<T>(), true, h.stream);
  launch_restrict<T>(L.d, C.d, h.faces, L.dmx, L.dmy, L.dmz, L.r.as<T>(), C.f.as<T>(), h.stream);
  launch_relayout<T>(C.d, C.f.as<T>(), rc, false, h.stream);
}

template <class T>
void prolong_t(mcw_handle& h, int l, const T* e, T* x) {
  Level& L = level_at(&h, l, true);
  Level& C = h.levels[l + 1];
  launch_relayout<T>(C.d, e, C.x.as<T>(), true, h.stream);
  launch_relayout<T>(L.d, x, L.x.as<T>(), true, h.stream);
  launch_prolong_dims<T>(L.d, C.d, h.faces, L.dmx, L.dmy, L.dmz, C.x.as<T>(), L.x.as<T>(), h.stream);
  launch_relayout<T>(L.d, L.x.as<T>(), x, false, h.stream);
}

template <class T>
void coarse_t(mcw_handle& h, const T* r, T* e) {
  Level& L = h.levels.back();
  launch_relayout<T>(L.d, r, L.f.as<T>(), true, h.stream);
  launch_fill<T>(L.x.as<T>(), L.d.N(), T(0), h.stream);
  if (h.n_coarse > 0)
    launch_coarse_solve<T>(h.n_coarse, h.coarse_inv.as<double>(), h.coarse_idx.as<int>(),
                           L.f.as<T>(), L.x.as<T>(), h.stream);
  launch_relayout<T>(L.d, L.x.as<T>(), e, false, h.stream);
}

template <class T>
void vcycle_t(mcw_handle& h, T* x, const T* f) {
  Level& L = h.levels[0];
  launch_relayout<T>(L.d, x, L.x.as<T>(), true, h.stream);
  launch_relayout<T>(L.d, f, L.f.as<T>(), true, h.stream);
  vcycle<T>(h, 0, L.x.as<T>(), L.f.as<T>());
  launch_relayout<T>(L.d, L.x.as<T>(), x, false, h.stream);
}


}  // namespace

// ---------------------------------------------------------------- batched solves

// Per-member state of the refinement loop (mirrors iterate()).
struct MemberState {
  mcw_status st = MCW_OK;
  bool active = false, prev_floor = false;
  double fnorm = 0.0, rel = 0.0, prev_rel = -1.0, rho_est = 0.0;
  int outer = 0, cycles = 0, prev_m = 0, stall = 0;
  std::vector<double> hist;
};

// Device-side job tables of one batch: every phase has a work list over the
// members that take part in it; all lists share one active-flag array.
class Batch {
 public:
  Batch(std::vector<mcw_handle*> hs) : hs_(std::move(hs)), m_((int)hs_.size()), s_(hs_[0]->stream) {}
  ~Batch() {
    if (graph_) (void)hipGraphExecDestroy(graph_);
    if (cg_graph_) (void)hipGraphExecDestroy(cg_graph_);
    if (host_sums_) (void)hipHostFree(host_sums_);
    if (host_cg_) (void)hipHostFree(host_cg_);
  }

  void build() {
    krylov_ = hs_[0]->opt.krylov != 0;
    depth_ = 0;
    for (auto* h : hs_) depth_ = std::max(depth_, (int)h->levels.size());
    gs_.assign(depth_, {});
    gs2r_.assign(depth_, {});
    gs3r_.assign(depth_, {});
    gsf_.assign(depth_, {});
    gsfr_.assign(depth_, {});
    gsf3r_.assign(depth_, {});
    fused_.assign(depth_, 0);
    by_gs_.assign(depth_, 4);
    by_res_.assign(depth_, 4);
    res_.assign(depth_, {});
    resv_.assign(depth_, {});
    const bool r_last = hs_[0]->opt.nu_pre > 0;
    restr_.assign(depth_, {});
    fillx_.assign(depth_, {});
    prol_.assign(depth_, {});
    coarse_.assign(depth_, {});
    for (int d = 0; d < depth_; ++d) {
      std::vector<ColJob> gsj[4], rj, g2r, g3r, rvj;
      std::vector<FusedJob> fj2[2], fr2[2], f3r;
      std::vector<int> fm2[2], frm2[2];
      std::vector<XferJob> rsj, pj;
      std::vector<VecJob> fj;
      std::vector<CoarseJob> cj;
      std::vector<int> gsm[4], rm, rsm, pm, fm, cm;
      // tile rows of this depth: the tuned shapes of its largest member
      size_t big = 0;
      for (int i = 0; i < m_; ++i) {
        mcw_handle& h = *hs_[i];
        if (d + 1 < (int)h.levels.size() && h.levels[d].d.N() > big) {
          big = h.levels[d].d.N();
          by_gs_[d] = std::max(1, h.levels[d].by_gs);  // per-colour passes: tiles of rows
          by_res_[d] = h.levels[d].by_res;
          // where the largest member's tuned pass is the fused one, so is the batch's
          fused_[d] = h.levels[d].by_gs == 0 ? 1 : 0;
        }
      }
      for (int i = 0; i < m_; ++i) {
        mcw_handle& h = *hs_[i];
        const int L = (int)h.levels.size();
        if (d >= L) continue;
        Level& V = h.levels[d];
        if (d == L - 1) {
          max_coarse_ = std::max(max_coarse_, h.n_coarse);
          cj.push_back(coarse_job(h.n_coarse, h.coarse_inv.as<double>(), h.coarse_idx.as<int>(),
                                  V.f.p, V.x.p));
          cm.push_back(i);
          continue;
        }
        Level& C = h.levels[d + 1];
        for (int c = 0; c < 4; ++c) {
          const ColJob J = col_job(V.d, h.faces, stencil_of<float>(V), V.f.p, V.x.p, nullptr, c, by_gs_[d]);
          if (J.nblocks > 0) {
            gsj[c].push_back(J);
            gsm[c].push_back(i);
            if (c == 2) {
              // colour (0,1) of the last pre-smoothing sweep writes the part of its
              // residual its own updates leave (the rest follows the (1,1) pass)
              g2r.push_back(J);
              g2r.back().rlast = r_last ? V.r.p : nullptr;
            }
            if (c == 3) {
              // the last colour of the last pre-smoothing sweep writes its residual
              // and the side sums of the (0,1) columns
              g3r.push_back(J);
              g3r.back().rlast = r_last ? V.r.p : nullptr;
              g3r.back().rside = r_last ? V.r.p : nullptr;
            }
          }
        }
        // the two-colour passes: (0,0),(1,0) on even rows, (0,1),(1,1) on odd
        // rows; reversed (1,1),(0,1) then (1,0),(0,0)
        for (int pr = 0; pr < 2; ++pr) {
          FusedJob F{};
          F.J0 = col_job(V.d, h.faces, stencil_of<float>(V), V.f.p, V.x.p, nullptr, 2 * pr, 1);
          F.J1 = col_job(V.d, h.faces, stencil_of<float>(V), V.f.p, V.x.p, nullptr, 2 * pr + 1, 1);
          F.nblocks = std::max(0, F.J0.ncy);
          if (F.nblocks > 0) {
            fj2[pr].push_back(F);
            fm2[pr].push_back(i);
            if (pr == 1) {
              // the odd rows of the last pre-smoothing sweep leave their residual
              // (gs_fused_kernel with SIDE)
              f3r.push_back(F);
              f3r.back().J0.rlast = r_last ? V.r.p : nullptr;
              f3r.back().J1.rlast = r_last ? V.r.p : nullptr;
              f3r.back().J1.rside = r_last ? V.r.p : nullptr;
            }
          }
          FusedJob R{};
          R.J0 = col_job(V.d, h.faces, stencil_of<float>(V), V.f.p, V.x.p, nullptr, 3 - 2 * pr, 1);
          R.J1 = col_job(V.d, h.faces, stencil_of<float>(V), V.f.p, V.x.p, nullptr, 2 - 2 * pr, 1);
          R.nblocks = std::max(0, R.J0.ncy);
          if (R.nblocks > 0) {
            fr2[pr].push_back(R);
            frm2[pr].push_back(i);
          }
        }
        rj.push_back(col_job(V.d, h.faces, stencil_of<float>(V), V.f.p, V.x.p, V.r.p, -1, by_res_[d]));
        rvj.push_back(rj.back());
        residual_skip(rvj.back(), r_last ? 2 : 0);
        rm.push_back(i);
        rsj.push_back(xfer_job(V.d, C.d, h.faces, V.dmx, V.dmy, V.dmz, V.r.p, C.f.p, true));
        rsm.push_back(i);
        pj.push_back(xfer_job(V.d, C.d, h.faces, V.dmx, V.dmy, V.dmz, C.x.p, V.x.p, false));
        pm.push_back(i);
        fj.push_back(vec_job(C.x.p, nullptr, C.d.N(), nullptr));
        fm.push_back(i);
      }
      for (int c = 0; c < 4; ++c) gs_[d][c] = add_split(gsj[c], gsm[c]);
      gs2r_[d] = add_split(g2r, gsm[2]);
      gs3r_[d] = add_split(g3r, gsm[3]);
      for (int pr = 0; pr < 2; ++pr) {
        gsf_[d][pr] = add_split(fj2[pr], fm2[pr]);
        if (krylov_) gsfr_[d][pr] = add_split(fr2[pr], frm2[pr]);
      }
      gsf3r_[d] = add_split(f3r, fm2[1]);
      res_[d] = add_split(rj, rm);
      resv_[d] = add_split(rvj, rm);
      restr_[d] = add(rsj, rsm);
      prol_[d] = add(pj, pm);
      fillx_[d] = add(fj, fm);
      coarse_[d] = add(cj, cm);
    }
    // outer-loop phases over all members
    std::vector<TileJob> rhs, res64, div;
    std::vector<RecoverJob> rec;
    std::vector<VecJob> zf, sc, f0, up;
    std::vector<SumJob> s1, s2;
    std::vector<int> all(m_);
    for (int i = 0; i < m_; ++i) all[i] = i;
    zero_slot_ = alloc_host(sizeof(double));  // float and double zero
    scales_slot_ = alloc_host(m_ * sizeof(double));
    sums_slot_ = alloc_host((size_t)m_ * 4 * sizeof(double));
    for (int i = 0; i < m_; ++i) {
      mcw_handle& h = *hs_[i];
      const size_t N = h.d.N();
      VecJob z = vec_job(nullptr, nullptr, N, nullptr);
      z.NX = h.d.NX();
      z.NY = h.d.NY();
      z.NZ = h.d.NZ();
      z.fc = h.faces;
      zf.push_back(z);
      TileJob A = tile_job(h);
      A.f = h.f64.as<double>();
      A.out = nullptr;
      A.partials = h.partials.as<double>();
      rhs.push_back(A);
      res64.push_back(A);
      div.push_back(A);
      rec.push_back(recover_job(h, nullptr, nullptr, nullptr));
      sc.push_back(vec_job(h.levels[0].f.p, h.r64.p, N, nullptr));
      sc.back().NX = h.d.NX();
      f0.push_back(vec_job(h.levels[0].x.p, nullptr, N, nullptr));
      // the correction: the V-cycles' x, or the CG solution e
      up.push_back(vec_job(nullptr, krylov_ ? h.ke.p : h.levels[0].x.p, N, nullptr));
      up.back().NX = h.d.NX();
      s1.push_back(SumJob{h.partials.as<double>(), (size_t)A.gx * A.gy, 1, nullptr});
      s2.push_back(SumJob{h.partials.as<double>(), (size_t)A.gx * A.gy, 2, nullptr});
    }
    zf_jobs_ = zf;
    rhs_jobs_ = rhs;
    res_jobs_ = res64;
    div_jobs_ = div;
    rec_jobs_ = rec;
    sc_jobs_ = sc;
    f0_jobs_ = f0;
    up_jobs_ = up;
    s1_jobs_ = s1;
    s2_jobs_ = s2;
    all_ = all;
    // job tables whose pointers change per call are filled in solve(); reserve their space now
    zf_ = add(zf, all);
    rhs_ = add(rhs, all);
    res64_ = add(res64, all);
    div_ = add(div, all);
    rec_ = add(rec, all);
    sc_ = add(sc, all);
    f0_ = add(f0, all);
    up_ = add(up, all);
    s1_off_ = add_raw(s1.data(), s1.size() * sizeof(SumJob));
    s2_off_ = add_raw(s2.data(), s2.size() * sizeof(SumJob));
    active_off_ = add_raw(nullptr, m_ * sizeof(int));
    if (krylov_) build_cg(all);
    blob_.alloc(host_.size());
    base_ = blob_.as<char>();
    MCW_HIP(hipHostMalloc((void**)&host_sums_, (size_t)m_ * 4 * sizeof(double), hipHostMallocDefault));
    if (krylov_) {
      // the coefficient slots live in the blob: point the jobs at them
      for (int i = 0; i < m_; ++i) cg_jobs_[i].sc = dev<double>(cg_slot_) + 4 * i;
      put(cgvec_, cg_jobs_);
      std::memcpy(&host_[cgtab_off_], cg_jobs_.data(), cg_jobs_.size() * sizeof(CgJob));
      MCW_HIP(hipHostMalloc((void**)&host_cg_, (size_t)m_ * 4 * sizeof(double), hipHostMallocDefault));
    }
  }

  // Work lists of the batched conjugate gradients: the vector kernels over
  // every member's level-0 vectors, q = -K p with p.q, and the fill of e.
  void build_cg(const std::vector<int>& all) {
    std::vector<ColJob> cr;
    std::vector<VecJob> fe;
    cg_jobs_.clear();
    for (int i = 0; i < m_; ++i) {
      mcw_handle& h = *hs_[i];
      Level& V = h.levels[0];
      const size_t N = V.d.N();
      ColJob J = col_job(V.d, h.faces, stencil_of<float>(V), nullptr, h.kp.p, h.kq.p, -1, by_res_[0]);
      J.part = h.partials.as<double>();
      need_partials((size_t)J.nblocks, h.n_partials);
      need_partials(2 * (size_t)cg_blocks(N), h.n_partials);
      cr.push_back(J);
      CgJob C{};
      C.e = h.ke.p;
      C.p = h.kp.p;
      C.z = V.x.p;
      C.r = V.f.p;
      C.q = h.kq.p;
      C.partials = h.partials.as<double>();
      C.n = N;
      C.nblocks = (int)cg_blocks(N);
      C.res_blocks = J.nblocks;
      C.member = i;
      cg_jobs_.push_back(C);
      fe.push_back(vec_job(h.ke.p, nullptr, N, nullptr));
    }
    cg_slot_ = alloc_host((size_t)m_ * 4 * sizeof(double));
    cgvec_ = add(cg_jobs_, all);
    cgres_ = add_split(cr, all);
    cgfill_ = add(fe, all);
    cgtab_off_ = add_raw(cg_jobs_.data(), cg_jobs_.size() * sizeof(CgJob));
  }

  // Solve all members; returns the first non-OK member status.
  mcw_status solve(const double* const* u0, double* const* lam, double* const* u, mcw_info* infos) {
    mcw_handle& h0 = *hs_[0];
    const bool timing = true;
    MCW_HIP(hipEventRecord(h0.ev[0], s_));
    // per-call pointers
    for (int i = 0; i < m_; ++i) {
      zf_jobs_[i].p = lam[i];
      rhs_jobs_[i].ue = u0[i];
      rhs_jobs_[i].out = hs_[i]->f64.as<double>();
      res_jobs_[i].v = lam[i];
      res_jobs_[i].out = hs_[i]->r64.as<double>();
      div_jobs_[i].ue = u0[i];
      div_jobs_[i].v = lam[i];
      div_jobs_[i].out = hs_[i]->t64.as<double>();
      rec_jobs_[i].u0 = u0[i];
      rec_jobs_[i].lam = lam[i];
      rec_jobs_[i].u = u ? u[i] : nullptr;
      sc_jobs_[i].scale = dev<double>(scales_slot_) + i;
      up_jobs_[i].p = lam[i];
      up_jobs_[i].scale = dev<double>(scales_slot_) + i;
      s1_jobs_[i].out = dev<double>(sums_slot_) + 4 * i;
      s2_jobs_[i].out = dev<double>(sums_slot_) + 4 * i;
    }
    put(zf_, zf_jobs_);
    put(rhs_, rhs_jobs_);
    put(res64_, res_jobs_);
    put(div_, div_jobs_);
    put(rec_, rec_jobs_);
    put(sc_, sc_jobs_);
    put(f0_, f0_jobs_);
    put(up_, up_jobs_);
    std::memcpy(&host_[s1_off_], s1_jobs_.data(), s1_jobs_.size() * sizeof(SumJob));
    std::memcpy(&host_[s2_off_], s2_jobs_.data(), s2_jobs_.size() * sizeof(SumJob));
    std::memset(&host_[zero_slot_], 0, sizeof(double));
    std::vector<MemberState> ms(m_);
    for (int i = 0; i < m_; ++i) ms[i].rho_est = hs_[i]->rho_setup;
    set_active(std::vector<int>(m_, 1));
    upload();

    launch_zero_fixed_batched(fix(zf_), s_);
    launch_tile_batched(M_RHS, fix(rhs_), s_);
    launch_sum_batched(dev<SumJob>(s1_off_), m_, s_);
    fetch_sums();
    std::vector<int> act(m_, 0);
    for (int i = 0; i < m_; ++i) {
      ms[i].fnorm = std::sqrt(host_sums_[4 * i]);
      if (!std::isfinite(ms[i].fnorm)) {
        ms[i].st = MCW_NONFINITE;
      } else if (ms[i].fnorm == 0.0) {
        launch_fill<double>(lam[i], hs_[i]->d.N(), 0.0, s_);
      } else {
        ms[i].active = true;
        act[i] = 1;
      }
    }
    MCW_HIP(hipEventRecord(h0.ev[1], s_));
    std::vector<double> cg_stop2(m_, 0.0);
    std::vector<int> cg_mmax(m_, 0), want_of(m_, 0);
    for (;;) {
      set_active(act);
      upload_active();
      launch_tile_batched(M_RESID, fix(res64_), s_);
      launch_sum_batched(dev<SumJob>(s1_off_), m_, s_);
      fetch_sums();
      int want = 0;
      for (int i = 0; i < m_; ++i) {
        MemberState& S = ms[i];
        if (!S.active) continue;
        mcw_handle& h = *hs_[i];
        const double tol = h.opt.rtol;  // each member stops on its own tolerance
        const double rr = host_sums_[4 * i];
        S.rel = std::sqrt(rr) / S.fnorm;
        S.hist.push_back(S.rel);
        ++S.outer;
        if (std::isfinite(S.rel) && S.prev_rel > 0.0 && S.prev_m > 0 && !krylov_)
          S.rho_est = update_rate(S.rho_est, S.rel / S.prev_rel, S.prev_m, S.prev_floor);
        if (!std::isfinite(S.rel)) { S.st = MCW_NONFINITE; S.active = false; }
        else if (S.rel <= tol) { S.active = false; }
        else if (S.cycles >= h.opt.max_cycles) { S.st = MCW_NOT_CONVERGED; S.active = false; }
        if (S.active && S.prev_rel > 0.0 && S.prev_m > 0) {
          if (S.rel / S.prev_rel > 0.95) {
            if (++S.stall >= 3) { S.st = MCW_NOT_CONVERGED; S.active = false; }
          } else {
            S.stall = 0;
          }
        }
        if (!S.active) continue;
        int mi = step_cycles(h, S.rho_est, S.rel, &S.prev_floor);
        mi = std::min(mi, h.opt.max_cycles - S.cycles);
        want_of[i] = mi;
        want = std::max(want, mi);
        const double nfree = (double)std::max<size_t>(free_count(h.d, h.faces), 1);
        const double scale = std::ldexp(1.0, -std::ilogb(std::sqrt(rr / nfree)));
        reinterpret_cast<double*>(&host_[scales_slot_])[i] = scale;
        // CG stops on its own residual: the same target, in the scaled FP32 units
        cg_mmax[i] = std::min(h.opt.inner_cycles > 0 ? h.opt.inner_cycles : 30, h.opt.max_cycles - S.cycles);
        const double stop = h.opt.inner_cycles > 0 ? 0.0 : std::max(tol / S.rel, inner_floor(h)) * std::sqrt(rr) * scale;
        cg_stop2[i] = stop * stop;
      }
      for (int i = 0; i < m_; ++i) act[i] = ms[i].active ? 1 : 0;
      if (want == 0) break;
      set_active(act);
      MCW_HIP(hipMemcpyAsync(base_ + scales_slot_, &host_[scales_slot_], m_ * sizeof(double),
                             hipMemcpyHostToDevice, s_));
      upload_active();
      launch_scale_batched(fix(sc_), s_);
      std::vector<int> took = want_of;
      if (krylov_) {
        took = cg_inner(act, cg_stop2, cg_mmax);
      } else {
        launch_fill_batched<float>(fix(f0_), s_);
        // each member runs its own cycle count: it leaves the active set (read
        // by every batched kernel) once its count is done
        std::vector<int> a = act;
        for (int c = 0; c < want; ++c) {
          bool change = false;
          for (int i = 0; i < m_; ++i)
            if (a[i] && want_of[i] <= c) { a[i] = 0; change = true; }
          if (change) {
            MCW_HIP(hipStreamSynchronize(s_));  // the previous upload has read host_
            set_active(a);
            upload_active();
          }
          vcycle();
        }
        if (a != act) {
          MCW_HIP(hipStreamSynchronize(s_));
          set_active(act);
          upload_active();
        }
      }
      launch_update_batched(fix(up_), s_);
      for (int i = 0; i < m_; ++i)
        if (ms[i].active) {
          ms[i].cycles += took[i];
          ms[i].prev_m = took[i];
          ms[i].prev_rel = ms[i].rel;
        }
      MCW_HIP(hipStreamSynchronize(s_));  // host_ staging is rewritten next step
    }
    MCW_HIP(hipEventRecord(h0.ev[2], s_));
    // recovery and divergence check for every member that has an iterate
    std::vector<int> fin(m_, 0), rec(m_, 0);
    bool any_rec = false;
    for (int i = 0; i < m_; ++i) {
      fin[i] = (ms[i].st == MCW_OK || ms[i].st == MCW_NOT_CONVERGED) ? 1 : 0;
      rec[i] = fin[i] && u && u[i] ? 1 : 0;  // a member without an output wind skips recovery
      any_rec = any_rec || rec[i];
    }
    if (any_rec) {
      set_active(rec);
      upload_active();
      launch_recover_batched(fix(rec_), s_);
      MCW_HIP(hipStreamSynchronize(s_));  // the upload has read host_
    }
    set_active(fin);
    upload_active();
    launch_tile_batched(M_DIV, fix(div_), s_);
    launch_sum_batched(dev<SumJob>(s2_off_), m_, s_);
    for (int i = 0; i < m_; ++i)
      if (!fin[i] && u && u[i])
        MCW_HIP(hipMemcpyAsync(u[i], u0[i], 3 * (size_t)hs_[i]->d.nx * hs_[i]->d.ny * hs_[i]->d.nz *
                                               sizeof(double), hipMemcpyDeviceToDevice, s_));
    fetch_sums();
    MCW_HIP(hipEventRecord(h0.ev[3], s_));
    MCW_HIP(hipEventSynchronize(h0.ev[3]));
    float t_all = 0.f, t_rhs = 0.f, t_iter = 0.f, t_fin = 0.f;
    if (timing) {
      MCW_HIP(hipEventElapsedTime(&t_all, h0.ev[0], h0.ev[3]));
      MCW_HIP(hipEventElapsedTime(&t_rhs, h0.ev[0], h0.ev[1]));
      MCW_HIP(hipEventElapsedTime(&t_iter, h0.ev[1], h0.ev[2]));
      MCW_HIP(hipEventElapsedTime(&t_fin, h0.ev[2], h0.ev[3]));
    }
    mcw_status first = MCW_OK;
    for (int i = 0; i < m_; ++i) {
      MemberState& S = ms[i];
      if (S.st != MCW_OK && first == MCW_OK) first = S.st;
      if (S.st == MCW_NOT_CONVERGED)
        hs_[i]->last_error = "not converged: relative residual " + std::to_string(S.rel);
      if (!infos) continue;
      mcw_info* info = &infos[i];
      std::memset(info, 0, sizeof(*info));
      Progress pg;
      pg.outer = S.outer;
      pg.cycles = S.cycles;
      pg.rel = S.rel;
      pg.hist = S.hist;
      fill_info(*hs_[i], pg, info);
      info->f_norm = S.fnorm;
      const double d0 = host_sums_[4 * i], d1 = host_sums_[4 * i + 1];
      info->rel_divergence = d1 > 0.0 ? std::sqrt(d0 / d1) : std::sqrt(d0);
      info->ms_total = t_all;
      info->ms_rhs = t_rhs;
      info->ms_cycles = t_iter;
      info->ms_finish = t_fin;
      info->status = S.st;
    }
    return first;
  }

  // For timing: `reps` launches of one batched phase over every member's finest
  // level on the members' own buffers (their current contents), all members
  // taking part.  kernel 0: one Gauss-Seidel sweep (two fused two-colour
  // launches, or four colour passes), 1: the residual.  Returns the device ms
  // per repetition (HIP events on the batch's stream around the launches) and
  // the launches per repetition of each stencil format present.
  std::pair<float, int> run_fine(int kernel, int reps) {
    set_active(std::vector<int>(m_, 1));
    upload();
    struct Events {  // destroyed on every way out
      hipEvent_t e[2] = {nullptr, nullptr};
      ~Events() {
        for (hipEvent_t x : e)
          if (x) (void)hipEventDestroy(x);
      }
    } ev;
    MCW_HIP(hipEventCreate(&ev.e[0]));
    MCW_HIP(hipEventCreate(&ev.e[1]));
    hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
    int launches = 0;
    MCW_HIP(hipEventRecord(e0, s_));
    for (int r = 0; r < reps; ++r) {
      if (kernel == 0 && fused_[0]) {
        for (int pr = 0; pr < 2; ++pr)
          for (int f = 0; f < 2; ++f)
            launch_gs_fused_batched<float>(fix(gsf_[0][pr].w[f]), s_, false, f == 1);
        launches = 2;
      } else if (kernel == 0) {
        for (int c = 0; c < 4; ++c)
          for (int f = 0; f < 2; ++f)
            launch_gs_batched<float>(fix(gs_[0][c].w[f]), s_, by_gs_[0], false, f == 1);
        launches = 4;
      } else {
        for (int f = 0; f < 2; ++f) launch_residual_batched<float>(fix(res_[0].w[f]), s_, by_res_[0], f == 1);
        launches = 1;
      }
    }
    MCW_HIP(hipEventRecord(e1, s_));
    MCW_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    MCW_HIP(hipEventElapsedTime(&ms, e0, e1));
    return {ms / reps, launches};
  }

 private:
  struct Slot {
    size_t jobs = 0, prefix = 0, member = 0;
    size_t bytes = 0;
  };

  template <class J>
  WorkList add(const std::vector<J>& jobs, const std::vector<int>& members) {
    std::vector<int> prefix(jobs.size() + 1, 0);
    for (size_t j = 0; j < jobs.size(); ++j) prefix[j + 1] = prefix[j] + nblocks_of(jobs[j]);
    WorkList W{};
    const size_t jo = add_raw(jobs.data(), jobs.size() * sizeof(J));
    const size_t po = add_raw(prefix.data(), prefix.size() * sizeof(int));
    const size_t mo = add_raw(members.data(), members.size() * sizeof(int));
    W.njobs = (int)jobs.size();
    W.total = prefix.back();
    // offsets are turned into device pointers once the blob exists
    W.jobs = reinterpret_cast<const void*>(jo);
    W.prefix = reinterpret_cast<const int*>(po);
    W.member = reinterpret_cast<const int*>(mo);
    return W;
  }

  // The work lists of one phase by stencil format (0: T values, 1: FP16), so
  // that each launch runs the kernel instance of its format.
  struct ByFormat {
    WorkList w[2]{};
    int njobs() const { return w[0].njobs + w[1].njobs; }
  };
  static int format_of(const ColJob& J) { return J.h16 ? 1 : 0; }
  static int format_of(const FusedJob& F) { return F.J0.h16 ? 1 : 0; }
  template <class J>
  ByFormat add_split(const std::vector<J>& jobs, const std::vector<int>& members) {
    std::vector<J> js[2];
    std::vector<int> ms[2];
    for (size_t k = 0; k < jobs.size(); ++k) {
      const int f = format_of(jobs[k]);
      js[f].push_back(jobs[k]);
      ms[f].push_back(members[k]);
    }
    ByFormat B;
    for (int f = 0; f < 2; ++f) B.w[f] = add(js[f], ms[f]);
    return B;
  }

  static int nblocks_of(const ColJob& J) { return J.nblocks; }
  static int nblocks_of(const FusedJob& F) { return F.nblocks; }
  static int nblocks_of(const XferJob& X) { return X.nblocks; }
  static int nblocks_of(const CoarseJob& C) { return C.nblocks; }
  static int nblocks_of(const VecJob& V) { return V.nblocks; }
  static int nblocks_of(const TileJob& A) { return A.gx * A.gy; }
  static int nblocks_of(const RecoverJob& R) { return R.gx * R.gy; }
  static int nblocks_of(const CgJob& C) { return C.nblocks; }

  size_t add_raw(const void* p, size_t bytes) {
    const size_t off = (host_.size() + 255) & ~size_t(255);
    host_.resize(off + bytes);
    if (p && bytes) std::memcpy(&host_[off], p, bytes);
    return off;
  }
  size_t alloc_host(size_t bytes) { return add_raw(nullptr, bytes); }

  template <class T> T* dev(size_t off) { return reinterpret_cast<T*>(base_ + off); }

  // device pointers of a work list built by add()
  WorkList fix(const WorkList& W) {
    WorkList R = W;
    R.jobs = base_ + reinterpret_cast<size_t>(W.jobs);
    R.prefix = reinterpret_cast<const int*>(base_ + reinterpret_cast<size_t>(W.prefix));
    R.member = reinterpret_cast<const int*>(base_ + reinterpret_cast<size_t>(W.member));
    R.active = reinterpret_cast<const int*>(base_ + active_off_);
    return R;
  }

  template <class J>
  void put(const WorkList& W, const std::vector<J>& jobs) {
    std::memcpy(&host_[reinterpret_cast<size_t>(W.jobs)], jobs.data(), jobs.size() * sizeof(J));
  }

  void set_active(const std::vector<int>& a) {
    std::memcpy(&host_[active_off_], a.data(), a.size() * sizeof(int));
  }
  void upload() {
    MCW_HIP(hipMemcpyAsync(base_, host_.data(), host_.size(), hipMemcpyHostToDevice, s_));
  }
  void upload_active() {
    MCW_HIP(hipMemcpyAsync(base_ + active_off_, &host_[active_off_], m_ * sizeof(int),
                           hipMemcpyHostToDevice, s_));
  }
  void fetch_sums() {
    MCW_HIP(hipMemcpyAsync(host_sums_, base_ + sums_slot_, (size_t)m_ * 4 * sizeof(double),
                           hipMemcpyDeviceToHost, s_));
    MCW_HIP(hipStreamSynchronize(s_));
  }

  // one batched FP32 V-cycle over all members (depth-first over levels)
  void vcycle_levels(int d) {
    const int nu_pre = hs_[0]->opt.nu_pre, nu_post = hs_[0]->opt.nu_post;
    launch_coarse_batched<float>(fix(coarse_[d]), std::max(max_coarse_, 1), s_);
    if (res_[d].njobs() == 0) return;
    for (int s = 0; s < nu_pre; ++s) {
      if (fused_[d]) {
        for (int pr = 0; pr < 2; ++pr) {
          const bool side = pr == 1 && s == nu_pre - 1;
          const ByFormat& g = side ? gsf3r_[d] : gsf_[d][pr];
          for (int f = 0; f < 2; ++f) launch_gs_fused_batched<float>(fix(g.w[f]), s_, false, f == 1, side);
        }
        continue;
      }
      const bool last = s == nu_pre - 1;
      for (int c = 0; c < 4; ++c) {
        const ByFormat& g = last && c == 2 ? gs2r_[d] : (last && c == 3 ? gs3r_[d] : gs_[d][c]);
        for (int f = 0; f < 2; ++f)
          launch_gs_batched<float>(fix(g.w[f]), s_, by_gs_[d], false, f == 1, last && c == 3);
      }
      if (last)
        for (int f = 0; f < 2; ++f)
          launch_side_residual_batched<float>(fix(gs2r_[d].w[f]), s_, by_gs_[d], f == 1);
    }
    // with pre-smoothing, the last colour's residual is already in place
    for (int f = 0; f < 2; ++f) launch_residual_batched<float>(fix(resv_[d].w[f]), s_, by_res_[d], f == 1);
    launch_restrict_batched<float>(fix(restr_[d]), s_);
    launch_fill_batched<float>(fix(fillx_[d]), s_);
    if (d + 1 < depth_) vcycle_levels(d + 1);
    launch_prolong_batched<float>(fix(prol_[d]), s_);
    // with CG the post-smoother is the reverse sweep, which keeps the cycle symmetric
    for (int s = 0; s < nu_post; ++s) {
      if (fused_[d]) {
        for (int pr = 0; pr < 2; ++pr) {
          const ByFormat& g = krylov_ ? gsfr_[d][pr] : gsf_[d][pr];
          for (int f = 0; f < 2; ++f) launch_gs_fused_batched<float>(fix(g.w[f]), s_, krylov_, f == 1);
        }
        continue;
      }
      for (int cc = 0; cc < 4; ++cc) {
        const int c = krylov_ ? 3 - cc : cc;
        for (int f = 0; f < 2; ++f) launch_gs_batched<float>(fix(gs_[d][c].w[f]), s_, by_gs_[d], krylov_, f == 1);
      }
    }
  }

  // One batched CG step for the members whose flag is on (the single-handle
  // step of pcg_step, member by member in one launch per phase).
  void cg_step_record() {
    const int* act = dev<int>(active_off_);
    const CgJob* tab = dev<CgJob>(cgtab_off_);
    launch_fill_batched<float>(fix(f0_), s_);  // z = 0
    vcycle_levels(0);
    launch_dot2_batched<float>(fix(cgvec_), s_);
    launch_cg_coeff_batched(tab, m_, 0, act, s_);
    launch_cg_direction_batched<float>(fix(cgvec_), s_);
    for (int f = 0; f < 2; ++f) launch_neg_apply_dot_batched<float>(fix(cgres_.w[f]), s_, by_res_[0], f == 1);
    launch_cg_coeff_batched(tab, m_, 1, act, s_);
    launch_cg_update_batched<float>(fix(cgvec_), s_);
    launch_cg_coeff_batched(tab, m_, 2, act, s_);
  }

  void cg_step() {
    if (!hs_[0]->opt.use_graph) {
      cg_step_record();
      return;
    }
    if (!cg_graph_) {
      hipGraph_t g = nullptr;
      MCW_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
      try {
        cg_step_record();
      } catch (...) {
        (void)hipStreamEndCapture(s_, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      MCW_HIP(hipStreamEndCapture(s_, &g));
      const hipError_t e = hipGraphInstantiate(&cg_graph_, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      MCW_HIP(e);
    }
    MCW_HIP(hipGraphLaunch(cg_graph_, s_));
  }

  // CG from e = 0 for the members in `act` until each one's recursive r.r
  // falls to its stop2 (0: never) or it has taken its mmax steps; returns the
  // steps of each member.  Leaves the flags of `act` set again.
  std::vector<int> cg_inner(const std::vector<int>& act, const std::vector<double>& stop2,
                            const std::vector<int>& mmax) {
    std::vector<int> a = act, steps(m_, 0);
    set_active(a);
    upload_active();
    launch_cg_reset_batched(dev<CgJob>(cgtab_off_), m_, dev<int>(active_off_), s_);
    launch_fill_batched<float>(fix(cgfill_), s_);
    for (int i = 0; i < m_; ++i)
      if (a[i] && mmax[i] <= 0) a[i] = 0;
    for (;;) {
      bool any = false;
      for (int i = 0; i < m_; ++i) any = any || a[i];
      if (!any) break;
      set_active(a);
      upload_active();
      cg_step();
      MCW_HIP(hipMemcpyAsync(host_cg_, base_ + cg_slot_, (size_t)m_ * 4 * sizeof(double),
                             hipMemcpyDeviceToHost, s_));
      MCW_HIP(hipStreamSynchronize(s_));
      for (int i = 0; i < m_; ++i) {
        if (!a[i]) continue;
        ++steps[i];
        const double rr = host_cg_[4 * i + 3];
        if (steps[i] >= mmax[i] || (stop2[i] > 0.0 && !(rr > stop2[i]))) a[i] = 0;
      }
    }
    set_active(act);
    upload_active();
    return steps;
  }

  void vcycle() {
    if (!hs_[0]->opt.use_graph) {
      vcycle_levels(0);
      return;
    }
    if (!graph_) {
      hipGraph_t g = nullptr;
      MCW_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
      try {
        vcycle_levels(0);
      } catch (...) {
        (void)hipStreamEndCapture(s_, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      MCW_HIP(hipStreamEndCapture(s_, &g));
      const hipError_t e = hipGraphInstantiate(&graph_, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      MCW_HIP(e);
    }
    MCW_HIP(hipGraphLaunch(graph_, s_));
  }

  std::vector<mcw_handle*> hs_;
  int m_;
  hipStream_t s_;
  bool krylov_ = false;
  hipGraphExec_t cg_graph_ = nullptr;
  double* host_cg_ = nullptr;
  std::vector<CgJob> cg_jobs_;
  WorkList cgvec_{}, cgfill_{};
  ByFormat cgres_{};
  size_t cg_slot_ = 0, cgtab_off_ = 0;
  int depth_ = 0, max_coarse_ = 0;
  std::vector<std::array<ByFormat, 4>> gs_;
  std::vector<ByFormat> gs2r_;  // colour (0,1) writing its part of r: the last pre-smoothing sweep
  std::vector<ByFormat> gs3r_;  // colour (1,1) writing r and the side sums: the last pre-smoothing pass
  // two-colour passes (forward pairs, reversed pairs, the last pre-smoothing
  // pair writing r), used at the depths where fused_ is set
  std::vector<std::array<ByFormat, 2>> gsf_, gsfr_;
  std::vector<ByFormat> gsf3r_;
  std::vector<char> fused_;
  std::vector<int> by_gs_, by_res_;
  std::vector<ByFormat> res_;   // the full residual (kernel timing)
  std::vector<ByFormat> resv_;  // the V-cycle's residual after pre-smoothing
  std::vector<WorkList> restr_, fillx_, prol_, coarse_;
  WorkList zf_{}, rhs_{}, res64_{}, div_{}, rec_{}, sc_{}, f0_{}, up_{};
  std::vector<VecJob> zf_jobs_, sc_jobs_, f0_jobs_, up_jobs_;
  std::vector<TileJob> rhs_jobs_, res_jobs_, div_jobs_;
  std::vector<RecoverJob> rec_jobs_;
  std::vector<SumJob> s1_jobs_, s2_jobs_;
  std::vector<int> all_;
  size_t s1_off_ = 0, s2_off_ = 0, active_off_ = 0, zero_slot_ = 0, scales_slot_ = 0, sums_slot_ = 0;
  std::vector<char> host_;
  DevBuf blob_;
  char* base_ = nullptr;
  double* host_sums_ = nullptr;
  hipGraphExec_t graph_ = nullptr;
};

void check_batch_handles(int m, mcw_handle* const* hs) {
  for (int i = 0; i < m; ++i) {
    if (!hs[i]) Fail::arg("batch member " + std::to_string(i) + " has a null handle");
    if (hs[i]->device != hs[0]->device) Fail::arg("batch members must share one device");
    if (hs[i]->opt.precision != hs[0]->opt.precision) Fail::arg("batch members must share one precision");
    if (hs[i]->opt.nu_pre != hs[0]->opt.nu_pre || hs[i]->opt.nu_post != hs[0]->opt.nu_post)
      Fail::arg("batch members must share nu_pre and nu_post");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) Fail::arg("a handle appears twice in the batch");
  }
}

mcw_status run_kernel_batch_impl(int m, mcw_handle* const* hs, int kernel, int reps,
                                 float* ms_per_rep, int32_t* launches_per_rep) {
  if (m < 1 || !hs) Fail::arg("need at least one member");
  if (kernel < 0 || kernel > 1 || reps < 1 || reps > 10000) Fail::arg("bad kernel or reps");
  check_batch_handles(m, hs);
  for (int i = 0; i < m; ++i)
    if (hs[i]->opt.precision != MCW_FP32_REFINE || hs[i]->opt.smoother != MCW_SMOOTH_POINT ||
        hs[i]->opt.krylov != hs[0]->opt.krylov)
      Fail::arg("batched kernels run FP32_REFINE point-smoother members of one kind");
  for (int i = 1; i < m; ++i) MCW_HIP(hipStreamSynchronize(hs[i]->stream));
  Batch b(std::vector<mcw_handle*>(hs, hs + m));
  b.build();
  const std::pair<float, int> t = b.run_fine(kernel, reps);
  if (ms_per_rep) *ms_per_rep = t.first;
  if (launches_per_rep) *launches_per_rep = t.second;
  return MCW_OK;
}

mcw_status solve_batch_impl(int m, mcw_handle* const* hs, const double* const* u0,
                            double* const* lambda, double* const* u, mcw_info* infos) {
  if (m == 0) return MCW_OK;
  for (int i = 0; i < m; ++i) {
    if (!hs[i] || !u0[i] || !lambda[i]) Fail::arg("batch member " + std::to_string(i) + " has a null argument");
    if (hs[i]->device != hs[0]->device) Fail::arg("batch members must share one device");
    if (hs[i]->opt.precision != hs[0]->opt.precision) Fail::arg("batch members must share one precision");
    if (hs[i]->opt.nu_pre != hs[0]->opt.nu_pre || hs[i]->opt.nu_post != hs[0]->opt.nu_post)
      Fail::arg("batch members must share nu_pre and nu_post");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) Fail::arg("a handle appears twice in the batch");
  }
  bool sequential = false;
  for (int i = 0; i < m; ++i)
    sequential = sequential || hs[i]->opt.krylov != hs[0]->opt.krylov ||
                 hs[i]->opt.smoother != MCW_SMOOTH_POINT;
  if (hs[0]->opt.precision != MCW_FP32_REFINE || sequential) {
    // plain FP64, line-smoother handles and batches mixing CG with the plain
    // iteration are solved one after another
    mcw_status first = MCW_OK;
    for (int i = 0; i < m; ++i) {
      const mcw_status s = solve_impl(*hs[i], u0[i], lambda[i], u ? u[i] : nullptr,
                                      infos ? &infos[i] : nullptr);
      if (s != MCW_OK && first == MCW_OK) first = s;
    }
    return first;
  }
  // members may run on their own streams: order them after the batch stream
  for (int i = 1; i < m; ++i) MCW_HIP(hipStreamSynchronize(hs[i]->stream));
  Batch b(std::vector<mcw_handle*>(hs, hs + m));
  b.build();
  return b.solve(u0, lambda, u, infos);
}

// ---------------------------------------------------------------- allocation-free divergence check

// Scratch of mcw_divergence_noalloc: two partial sums per element tile, the
// two reduced sums, and the flag of the grid-structure check.  Every block
// writes its own partials and the reduction writes the sums; the flag is
// cleared by a fill kernel before the check.  Each device holds its own copy
// until the process ends.
static constexpr size_t kNoAllocDoubles = MCW_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kNoAllocDoubles];

// Device address of `scratch` on the current device, looked up once per device.
// On the host the array's name is only a stand-in: kernels get this address.
static double* noalloc_scratch() {
  static std::mutex mu;
  static std::array<double*, 256> ptr{};
  int dev = 0;
  MCW_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= (int)ptr.size()) Fail::arg("device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    MCW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error{MCW_HIP_ERROR, "hipGetSymbolAddress returned no address for the scratch array"};
    ptr[dev] = static_cast<double*>(p);
  }
  return ptr[dev];
}

static mcw_status divergence_noalloc_impl(const mcw_grid_desc* g, const double* u0, const double* lam,
                                   double* D, double* rel, void* stream) {
  validate_grid(g);
  if (g->gamma_faces == 63u)
    throw Error{MCW_SINGULAR, "Gamma covers every face: lambda is only defined up to a constant"};
  if (!u0 || !lam || !D) Fail::arg("null vector");
  const Dims d{g->nx, g->ny, g->nz};
  const size_t tiles = tile_count(d);
  if (tiles > MCW_NOALLOC_MAX_TILES)
    Fail::arg("grid of " + std::to_string(tiles) + " element tiles exceeds the " +
              std::to_string(MCW_NOALLOC_MAX_TILES) + " the fixed scratch holds");
  double* sp = noalloc_scratch();
  hipStream_t s = static_cast<hipStream_t>(stream);
  // whether the grid is terrain-following is found on the device, so that the
  // call needs no wait: the divergence kernel reads the flag
  int* flag = reinterpret_cast<int*>(sp + 2 * tiles + 2);
  launch_fill<double>(sp + 2 * tiles + 2, 1, 0.0, s);
  launch_structure_check(g->X, g->Y, d, flag, s);
  GridRef G{g->X, g->Y, g->Z, d, {}, Faces{g->gamma_faces}, 0, flag};
  for (int k = 0; k < 3; ++k) G.c[k] = 1.0 / (g->a[k] * g->a[k]);
  launch_divergence_ref(G, u0, lam, D, sp, s);
  if (rel) {
    launch_sum_partials(sp, tiles, 2, sp + 2 * tiles, s);
    double out[2] = {0.0, 0.0};
    MCW_HIP(hipMemcpyAsync(out, sp + 2 * tiles, sizeof(out), hipMemcpyDeviceToHost, s));
    MCW_HIP(hipStreamSynchronize(s));
    *rel = out[1] > 0.0 ? std::sqrt(out[0] / out[1]) : std::sqrt(out[0]);
  }
  return MCW_OK;
}

// ================================================================ C ABI

extern "C" {

void mcw_default_options(mcw_options* o) {
  if (!o) return;
  o->precision = MCW_FP32_REFINE;
  o->rtol = 1e-8;
  o->max_cycles = 200;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->inner_cycles = 0;
  o->coarsen_rule = MCW_COARSEN_OPERATOR;
  o->coarse_direct_max = 1024;
  o->use_graph = 1;
  o->verbose = std::getenv("MCW_LOG") ? 1 : 0;
  o->autotune = 1;
  o->krylov = 0;
  o->smoother = MCW_SMOOTH_POINT;
  o->stencil_fp16 = 0;
  o->merge_spacing = MCW_MERGE_LEVEL_SPACING;
  o->tune_cache = nullptr;
}

mcw_status mcw_create(const mcw_grid_desc* g, const mcw_options* opts, void* stream,
                      mcw_handle** out) {
  if (!out) {
    g_error = "out must be non-null";
    return MCW_INVALID_ARG;
  }
  *out = nullptr;
  mcw_options o;
  if (opts) o = *opts;
  else mcw_default_options(&o);
  auto* h = new (std::nothrow) mcw_handle();
  if (!h) return MCW_OOM;
  const mcw_status st = guarded(nullptr, [&] {
    create_impl(g, o, stream, *h);
    return MCW_OK;
  });
  if (st != MCW_OK) {
    destroy_impl(h);
    return st;
  }
  *out = h;
  return MCW_OK;
}

void mcw_destroy(mcw_handle* h) { destroy_impl(h); }

mcw_status mcw_set_tolerance(mcw_handle* h, double rtol, int32_t max_cycles) {
  if (!h) return MCW_INVALID_ARG;
  if (!(rtol > 0.0) || !(rtol < 1.0) || max_cycles < 1) {
    h->last_error = "rtol must be in (0, 1) and max_cycles >= 1";
    return MCW_INVALID_ARG;
  }
  h->opt.rtol = rtol;
  h->opt.max_cycles = max_cycles;
  return MCW_OK;
}

mcw_status mcw_solve(mcw_handle* h, const double* u0, double* lambda, double* u, mcw_info* info) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] { return solve_impl(*h, u0, lambda, u, info); });
}

mcw_status mcw_solve_batch(int32_t m, mcw_handle* const* hs, const double* const* u0,
                           double* const* lambda, double* const* u, mcw_info* infos) {
  if (m < 0 || (m > 0 && (!hs || !u0 || !lambda))) {
    g_error = "bad batch arguments";
    return MCW_INVALID_ARG;
  }
  return guarded(nullptr, [&] { return solve_batch_impl(m, hs, u0, lambda, u, infos); });
}

mcw_status mcw_adjoint(mcw_handle* h, const double* lambda, const double* g_u, float* dL_du0,
                       double dL_da[3], mcw_info* info) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!lambda || !g_u || !dL_du0 || !dL_da) Fail::arg("adjoint arguments must be non-null");
    if (info) std::memset(info, 0, sizeof(*info));
    const size_t N = h->d.N();
    size_t np = 0;
    double gg = 0.0;
    // g_lambda = G_1^T diag(c) g_u on the free nodes (right-hand side of the transpose solve)
    launch_adjoint_scatter(*h, g_u, h->f64.as<double>(), h->partials.as<double>(), &np);
    reduce_to_host(*h, np, 1, &gg);
    const double gnorm = std::sqrt(gg);
    if (!std::isfinite(gnorm)) {
      h->last_error = "non-finite adjoint right-hand side";
      return MCW_NONFINITE;
    }
    double* mu = h->t64.as<double>();
    launch_fill<double>(mu, N, 0.0, h->stream);
    Progress pg;
    mcw_status st = MCW_OK;
    if (gnorm > 0.0) st = iterate(*h, mu, gnorm, pg);
    if (st != MCW_OK && st != MCW_NOT_CONVERGED) {
      if (info) {
        fill_info(*h, pg, info);
        info->status = st;
      }
      return st;
    }
    double dc[3] = {0.0, 0.0, 0.0};
    launch_adjoint_elements(*h, g_u, lambda, mu, dL_du0, h->partials.as<double>(), &np);
    reduce_to_host(*h, np, 3, dc);
    for (int d = 0; d < 3; ++d) dL_da[d] = -2.0 * dc[d] / (h->a[d] * h->a[d] * h->a[d]);
    if (info) {
      fill_info(*h, pg, info);
      info->f_norm = gnorm;
      info->status = st;
    }
    return st;
  });
}

mcw_status mcw_apply_K(mcw_handle* h, const double* x, double* y) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!x || !y) Fail::arg("null vector");
    launch_apply(*h, x, nullptr, y, 0, nullptr, nullptr);
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_rhs(mcw_handle* h, const double* u0, double* f) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!u0 || !f) Fail::arg("null vector");
    launch_rhs(*h, u0, f, nullptr, nullptr);
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_recover(mcw_handle* h, const double* u0, const double* lambda, double* u) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!u0 || !lambda || !u) Fail::arg("null vector");
    launch_recover(*h, u0, lambda, u);
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_divergence(mcw_handle* h, const double* u0, const double* lambda, double* D,
                          double* rel) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!u0 || !lambda || !D) Fail::arg("null vector");
    size_t np = 0;
    double s[2];
    launch_divergence(*h, u0, lambda, D, h->partials.as<double>(), &np);
    reduce_to_host(*h, np, 2, s);
    if (rel) *rel = s[1] > 0.0 ? std::sqrt(s[0] / s[1]) : std::sqrt(s[0]);
    return MCW_OK;
  });
}

mcw_status mcw_divergence_noalloc(const mcw_grid_desc* g, const double* u0, const double* lambda,
                                  double* D, double* rel, void* stream) {
  return guarded(nullptr, [&] { return divergence_noalloc_impl(g, u0, lambda, D, rel, stream); });
}

mcw_status mcw_interp_wind(mcw_handle* h, const mcw_coarse_wind* cw, double* u0) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!cw || !u0 || !cw->hagl || !cw->wind) Fail::arg("null coarse wind or output");
    if (cw->ncx < 2 || cw->ncy < 2 || cw->nl < 1) Fail::arg("need ncx, ncy >= 2 and nl >= 1");
    const double v[5] = {cw->x0, cw->y0, cw->dx, cw->dy, cw->z0};
    for (double x : v)
      if (!std::isfinite(x)) Fail::arg("coarse grid origin, spacing and z0 must be finite");
    if (!(cw->dx > 0.0) || !(cw->dy > 0.0) || !(cw->z0 > 0.0)) Fail::arg("dx, dy and z0 must be > 0");
    if (!launch_coarse_check(*h, *cw))
      Fail::arg("coarse level heights must be finite, increase up each column and start above z0");
    launch_interp_wind(*h, *cw, u0);
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_surface_wind(mcw_handle* h, const double* u, double height, double z0, double* uv) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!u || !uv) Fail::arg("null wind or output");
    if (!(height > 0.0) || !std::isfinite(height) || !(z0 > 0.0) || !std::isfinite(z0))
      Fail::arg("height and z0 must be finite and > 0");
    launch_surface_wind(*h, u, height, z0, uv);
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_tile_shape(const mcw_handle* hc, int32_t l, int32_t* rows_smooth, int32_t* rows_residual) {
  auto* h = const_cast<mcw_handle*>(hc);
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    const Level& L = level_at(h, l, false);
    if (rows_smooth) *rows_smooth = L.by_gs;
    if (rows_residual) *rows_residual = L.by_res;
    return MCW_OK;
  });
}

int32_t mcw_num_levels(const mcw_handle* h) { return h ? (int32_t)h->levels.size() : 0; }

mcw_status mcw_level_info(const mcw_handle* hc, int32_t l, int32_t dims[3], int32_t* coarsen_h,
                          int32_t* keep_z, int32_t* n_keep) {
  auto* h = const_cast<mcw_handle*>(hc);
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    const Level& L = level_at(h, l, false);
    if (dims) {
      dims[0] = L.d.nx;
      dims[1] = L.d.ny;
      dims[2] = L.d.nz;
    }
    if (coarsen_h) *coarsen_h = L.coarsen_h;
    if (n_keep) *n_keep = (int32_t)L.keep_z.size();
    if (keep_z)
      for (size_t q = 0; q < L.keep_z.size(); ++q) keep_z[q] = L.keep_z[q];
    return MCW_OK;
  });
}

mcw_status mcw_get_stencil(mcw_handle* h, int32_t l, int32_t prec, void* out) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!out) Fail::arg("null output");
    Level& L = level_at(h, l, false);
    if (prec == MCW_FP64) {
      if (L.st64.p) {
        launch_unsplit_stencil(L.d, L.st64.p, out, 1, h->stream);
      } else if (l == 0) {
        DevBuf tmp;
        tmp.alloc(SW * L.d.layout().nodes * sizeof(double));
        launch_fill<double>(tmp.as<double>(), SW * L.d.layout().nodes, 0.0, h->stream);
        launch_assemble_stencil(*h, tmp.as<double>());
        launch_unsplit_stencil(L.d, tmp.p, out, 1, h->stream);
        MCW_HIP(hipStreamSynchronize(h->stream));
      } else {
        Fail::arg("FP64 coarse stencils are kept only by FP64 handles");
      }
    } else if (prec == MCW_FP32_REFINE) {
      // the values the FP32 V-cycle computes with (FP16 ones times their level scale)
      if (L.st16.p) launch_unsplit_stencil(L.d, L.st16.p, out, 2, h->stream, L.st_scale);
      else if (L.st32.p) launch_unsplit_stencil(L.d, L.st32.p, out, 0, h->stream);
      else Fail::arg("FP32 stencils exist only in FP32_REFINE handles");
    } else {
      Fail::arg("bad precision");
    }
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_smooth(mcw_handle* h, int32_t l, void* x, const void* f, int32_t sweeps) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!x || !f || sweeps < -1000 || sweeps > 1000) Fail::arg("bad smoother arguments");
    if (is_f32(h)) smooth_t(*h, l, static_cast<float*>(x), static_cast<const float*>(f), sweeps);
    else smooth_t(*h, l, static_cast<double*>(x), static_cast<const double*>(f), sweeps);
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_residual(mcw_handle* h, int32_t l, const void* x, const void* f, void* r) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!x || !f || !r) Fail::arg("null vector");
    if (is_f32(h))
      residual_t(*h, l, static_cast<const float*>(x), static_cast<const float*>(f), static_cast<float*>(r));
    else
      residual_t(*h, l, static_cast<const double*>(x), static_cast<const double*>(f),
                 static_cast<double*>(r));
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_restrict(mcw_handle* h, int32_t l, const void* r, void* rc) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!r || !rc) Fail::arg("null vector");
    if (is_f32(h)) restrict_t(*h, l, static_cast<const float*>(r), static_cast<float*>(rc));
    else restrict_t(*h, l, static_cast<const double*>(r), static_cast<double*>(rc));
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_prolong(mcw_handle* h, int32_t l, const void* e, void* x) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!e || !x) Fail::arg("null vector");
    if (is_f32(h)) prolong_t(*h, l, static_cast<const float*>(e), static_cast<float*>(x));
    else prolong_t(*h, l, static_cast<const double*>(e), static_cast<double*>(x));
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_coarse_solve(mcw_handle* h, const void* r, void* e) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!r || !e) Fail::arg("null vector");
    if (is_f32(h)) coarse_t(*h, static_cast<const float*>(r), static_cast<float*>(e));
    else coarse_t(*h, static_cast<const double*>(r), static_cast<double*>(e));
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_vcycle(mcw_handle* h, void* x, const void* f) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (!x || !f) Fail::arg("null vector");
    if (is_f32(h)) vcycle_t(*h, static_cast<float*>(x), static_cast<const float*>(f));
    else vcycle_t(*h, static_cast<double*>(x), static_cast<const double*>(f));
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

mcw_status mcw_run_kernel_batch(int32_t m, mcw_handle* const* hs, int32_t kernel, int32_t reps,
                                float* ms_per_rep, int32_t* launches_per_rep) {
  return guarded(nullptr, [&] {
    return run_kernel_batch_impl(m, hs, kernel, reps, ms_per_rep, launches_per_rep);
  });
}

mcw_status mcw_run_kernel(mcw_handle* h, int32_t l, int32_t kernel, int32_t reps) {
  if (!h) return MCW_INVALID_ARG;
  return guarded(h, [&] {
    if (kernel < 0 || kernel > 4 || reps < 0) Fail::arg("bad kernel or repetition count");
    Level& L = level_at(h, l, kernel == 2 || kernel == 3);
    if (kernel == 4 && l != 0) Fail::arg("the matrix-free residual runs on level 0");
    for (int r = 0; r < reps; ++r) {
      if (kernel == 4) {
        launch_apply(*h, h->t64.as<double>(), h->f64.as<double>(), h->r64.as<double>(), 1, nullptr,
                     nullptr);
        continue;
      }
      if (is_f32(h)) {
        float *x = L.x.as<float>(), *f = L.f.as<float>(), *rr = L.r.as<float>();
        if (kernel == 0)
          launch_smooth_sweep<float>(L.d, h->faces, stencil_of<float>(L), f, x, h->stream, L.by_gs, false,
                                     line_buf<float>(*h, L));
        if (kernel == 1)
          launch_residual<float>(L.d, h->faces, stencil_of<float>(L), x, f, rr, nullptr, nullptr, h->stream,
                                 L.by_res);
        if (kernel == 2 || kernel == 3) {
          Level& C = h->levels[l + 1];
          if (kernel == 2)
            launch_restrict<float>(L.d, C.d, h->faces, L.dmx, L.dmy, L.dmz, rr, C.f.as<float>(), h->stream);
          else
            launch_prolong_dims<float>(L.d, C.d, h->faces, L.dmx, L.dmy, L.dmz, C.x.as<float>(), x,
                                       h->stream);
        }
      } else {
        double *x = L.x.as<double>(), *f = L.f.as<double>(), *rr = L.r.as<double>();
        if (kernel == 0)
          launch_smooth_sweep<double>(L.d, h->faces, L.st64.as<double>(), f, x, h->stream, L.by_gs, false,
                                      line_buf<double>(*h, L));
        if (kernel == 1)
          launch_residual<double>(L.d, h->faces, L.st64.as<double>(), x, f, rr, nullptr, nullptr, h->stream,
                                  L.by_res);
        if (kernel == 2 || kernel == 3) {
          Level& C = h->levels[l + 1];
          if (kernel == 2)
            launch_restrict<double>(L.d, C.d, h->faces, L.dmx, L.dmy, L.dmz, rr, C.f.as<double>(), h->stream);
          else
            launch_prolong_dims<double>(L.d, C.d, h->faces, L.dmx, L.dmy, L.dmz, C.x.as<double>(), x,
                                        h->stream);
        }
      }
    }
    MCW_HIP(hipStreamSynchronize(h->stream));
    return MCW_OK;
  });
}

const char* mcw_status_string(mcw_status s) {
  switch (s) {
    case MCW_OK: return "MCW_OK";
    case MCW_INVALID_ARG: return "MCW_INVALID_ARG";
    case MCW_BAD_GEOMETRY: return "MCW_BAD_GEOMETRY";
    case MCW_SINGULAR: return "MCW_SINGULAR";
    case MCW_NONFINITE: return "MCW_NONFINITE";
    case MCW_NOT_CONVERGED: return "MCW_NOT_CONVERGED";
    case MCW_OOM: return "MCW_OOM";
    case MCW_HIP_ERROR: return "MCW_HIP_ERROR";
  }
  return "unknown status";
}

const char* mcw_last_error(const mcw_handle* h) { return h ? h->last_error.c_str() : g_error.c_str(); }

}  // extern "C"
