// Internal declarations shared by the libmcwind sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/mcwind.h"

namespace mcw {

// ---------------------------------------------------------------- errors

struct Error {
  mcw_status status;
  std::string msg;
};

#define MCW_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::mcw::Error{e_ == hipErrorOutOfMemory ? MCW_OOM : MCW_HIP_ERROR,         \
                         std::string(#call) + ": " + hipGetErrorString(e_)};          \
  } while (0)

#define MCW_CHECK_LAUNCH() MCW_HIP(hipGetLastError())

// Every launch that writes per-block partial sums checks, before it launches,
// that its blocks times channels fit the buffer.
inline void need_partials(size_t entries, size_t cap) {
  if (entries > cap)
    throw Error{MCW_HIP_ERROR, "internal error: " + std::to_string(entries) +
                                   " partial sums exceed the buffer of " + std::to_string(cap)};
}

// ---------------------------------------------------------------- device buffers

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    MCW_HIP(hipMalloc(&p, n));
    bytes = n;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------- reductions

// Sum over the 64 lanes of a wave by a butterfly of lane exchanges (no LDS);
// lane 0's result has a fixed order of additions.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Block-wide sum of one double per thread into *out: each wave's sum, then
// thread 0 adds the waves' sums in wave order (deterministic).  s_red holds at
// least one slot per wave of the block.
__device__ __forceinline__ void block_sum_to(double v, double* s_red, double* out) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double s = s_red[0];
    for (int w = 1; w < nw; ++w) s += s_red[w];
    *out = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- stencil layout

// 27-point stencils are stored per node as SW = 28 values (27 coefficients
// and a zero pad), in 16-byte groups (4 floats or 2 doubles).  Nodes are
// numbered plane by plane and row by row, with the even x indices of a row
// first and then the odd ones, each half padded to a multiple of 64 nodes;
// for every run of 64 consecutive node numbers the layout stores group 0 of
// all 64 nodes, then group 1, and so on.  A wave of 64 lanes updating one
// colour class of a row thus reads each coefficient group as one contiguous
// 1 KB block, with a single address per lane and immediate offsets.
constexpr int SW = 28;

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so that neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, rem = n & 7, x = b & 7, s = b >> 3;
  return x * q + min(x, rem) + s;
}

struct StLayout {
  int NY = 0, NXeP = 0, rowlen = 0;
  size_t nodes = 0;  // padded node count
  __host__ __device__ size_t node(int i, int j, int k) const {
    return ((size_t)k * NY + j) * rowlen + ((i & 1) ? NXeP + (i >> 1) : (i >> 1));
  }
};

// FP64 stencils: SW slots per node (the 27 coefficients and a pad), in groups of
// two doubles interleaved over 64 consecutive nodes.
template <class T>
__host__ __device__ inline size_t st_entry(size_t p, int o);
template <>
__host__ __device__ inline size_t st_entry<double>(size_t p, int o) {
  constexpr int G = SW / 2;
  return ((p >> 6) * G + o / 2) * (size_t)128 + (p & 63) * 2 + (o % 2);
}

// FP32 stencils store 25 of the 26 off-diagonal coefficients.  The diagonal
// of the FP32 operator is minus the sum of the off-diagonals (stencil_diag),
// and the coupling to the node below in the same column (o = 4) is the
// coupling of that node to the one above it (its o = 22): the column coupling
// of the FP32 operator is symmetric by construction, and zero below the
// bottom plane.  Both are formed where they are used instead of being read; a
// thread marching up a column already holds the o = 22 value of the node
// below.  Per 64 consecutive nodes: six groups of four floats (slots 0-23)
// and one single float (slot 24), each interleaved over the 64 nodes; 100 B
// per node.
constexpr int SW32 = 25;
__host__ __device__ constexpr bool stored32(int o) { return o != 4 && o != 13; }
__host__ __device__ constexpr int slot32(int o) { return o < 4 ? o : (o < 13 ? o - 1 : o - 2); }
template <>
__host__ __device__ inline size_t st_entry<float>(size_t p, int o) {
  const int s = slot32(o);
  const size_t base = (p >> 6) * (size_t)(64 * SW32);
  return s < 24 ? base + (size_t)(s >> 2) * 256 + (p & 63) * 4 + (s & 3) : base + 1536 + (p & 63);
}

// FP16 stencils (option stencil_fp16): the same 25 stored coefficients,
// divided by a power of two s per level (the level's largest magnitude rounded
// up) and rounded once to FP16 (below 2^-14 to zero).  Per 64 consecutive nodes: three
// groups of eight halves (slots 0-23) and one single half (slot 24); 50 B per
// node.  The kernels compute with the scaled values and scale f and r by 1/s
// and s, both exact.
constexpr int SW16 = 25;
__host__ __device__ inline size_t st_entry16(size_t p, int o) {
  const int s = slot32(o);
  const size_t base = (p >> 6) * (size_t)(64 * SW16);
  return s < 24 ? base + (size_t)(s >> 3) * 512 + (p & 63) * 8 + (s & 7) : base + 1536 + (p & 63);
}

// A level's stencil as the kernels see it: the array, whether it holds FP16
// values, and the level scale s with its inverse (1 for FP32 and FP64).
struct StRef {
  const void* p = nullptr;
  int h16 = 0;
  float sc = 1.f, isc = 1.f;
  StRef() = default;
  StRef(const void* q) : p(q) {}  // NOLINT: an FP32 or FP64 array
};

// Diagonal of the FP32 operator from its off-diagonal coefficients a[o],
// o != 13: minus their sum, accumulated in FP64 in the order of o and rounded
// once, so that constants stay in the null space of the unconstrained FP32
// operator as they are for K.
__host__ __device__ inline float stencil_diag(const float* a) {
  double sum = 0.0;
  for (int o = 0; o < 27; ++o)
    if (o != 13) sum += (double)a[o];
  return (float)(-sum);
}

// ---------------------------------------------------------------- grid geometry

// Node-grid dimensions of one level: NX = nx+1 nodes in x, etc.
struct Dims {
  int nx, ny, nz;  // elements
  __host__ __device__ int NX() const { return nx + 1; }
  __host__ __device__ int NY() const { return ny + 1; }
  __host__ __device__ int NZ() const { return nz + 1; }
  __host__ __device__ size_t N() const { return (size_t)NX() * NY() * NZ(); }
  // number of even x indices (they come first in every stencil row)
  __host__ __device__ int NXe() const { return (NX() + 1) >> 1; }
  __host__ __device__ StLayout layout() const {
    StLayout L;
    L.NY = NY();
    L.NXeP = (NXe() + 63) & ~63;
    L.rowlen = L.NXeP + ((NX() - NXe() + 63) & ~63);
    L.nodes = (size_t)NZ() * NY() * L.rowlen;
    return L;
  }
};

// Free-node test: a node is fixed iff it lies on a face outside Gamma.
struct Faces {
  uint32_t gamma;
  __host__ __device__ bool x_fixed(int i, int NX) const {
    return (i == 0 && !(gamma & MCW_GAMMA_XLO)) || (i == NX - 1 && !(gamma & MCW_GAMMA_XHI));
  }
  __host__ __device__ bool y_fixed(int j, int NY) const {
    return (j == 0 && !(gamma & MCW_GAMMA_YLO)) || (j == NY - 1 && !(gamma & MCW_GAMMA_YHI));
  }
  __host__ __device__ int k_first() const { return (gamma & MCW_GAMMA_BOTTOM) ? 0 : 1; }
  __host__ __device__ int k_last(int NZ) const { return (gamma & MCW_GAMMA_TOP) ? NZ - 1 : NZ - 2; }
};

// Interpolation between a level and the next coarser one, per direction.
// Fine index p maps to coarse lo[p], hi[p] (equal when p is kept, weight 1;
// else weight 1/2 each).  Coarse index c has fine centre ctr[c] and support
// [slo[c], shi[c]] (the kept node and its dropped neighbours).
struct DirMap {
  int nf = 0, nc = 0;  // node counts
  std::vector<int> lo, hi, ctr, slo, shi;
};

struct DirMapDev {
  const int* lo;
  const int* hi;
  const int* ctr;
  const int* slo;
  const int* shi;
};

// ---------------------------------------------------------------- launch jobs

// Arguments of one member's share of a launch.  Single solves launch one job
// per kernel; a batch launches one persistent kernel per phase over the jobs
// of all members (a flattened list of (job, block) work items).
struct ColJob {  // smoother colour pass, residual
  const void* st;
  const void* f;
  void* x;
  void* r;
  int NX, NY, NZ;
  Faces fc;
  int ci, cj, ncx, ncy;  // colour class and its column counts (smoother)
  int by;                // rows of 64-column tiles per block (block = 64 * by threads)
  int tiles_x, nblocks;  // local grid of 64 x by column tiles
  double* part;          // per-block partial sums of a batched residual with a dot product
  int h16;               // the stencil holds FP16 values scaled by 1/sc (FP32 V-cycles only)
  float sc, isc;         // sc and 1/sc; 1 for FP32 and FP64 stencils
  void* rlast;           // forward pass ending a sweep: also write r of this colour's columns
  void* rside;           // forward (1,1) pass ending a sweep: side sums for the (0,1) columns
  int skip11;            // residual: 1, the (1,1) columns already hold r; 2, every odd row does
};

struct FusedJob {  // two colour passes of the same rows, one block per row (batched)
  ColJob J0, J1;
  int nblocks;  // rows: J0.ncy
};

struct XferJob {  // restriction rc = P^T r (src = r, dst = rc); prolongation x += P e (src = e, dst = x)
  const void* src;
  void* dst;
  int NXf, NYf, NZf, NXc, NYc, NZc;
  Faces fc;
  DirMapDev mx, my, mz;
  int tiles_x, nblocks;
};

struct CoarseJob {  // e = K_L^-1 r on the free coarsest nodes
  int n;
  const double* inv;
  const int* idx;
  const void* r;
  void* e;
  int nblocks;
};

struct VecJob {  // fills, casts, lambda updates, zeroing of fixed nodes
  void* p;          // output
  const void* q;    // input
  size_t n;
  const double* scale;  // device scalar (casts / updates)
  int NX, NY, NZ;       // zeroing of fixed nodes
  Faces fc;
  int nblocks;
};

struct SumJob {  // deterministic sum of `width` channels of n_part block partials
  const double* partials;
  size_t n_part;
  int width;
  double* out;
};

struct TileJob {  // element-tile kernels (matrix-free apply/residual, rhs, divergence, adjoint)
  const double* X;
  const double* Y;
  const double* Z;
  const double* v;   // nodal field (apply, residual, divergence)
  const double* f;   // right-hand side (residual)
  const double* ue;  // element 3-vectors (rhs, divergence, adjoint scatter)
  double* out;       // nodal output
  double* uout;      // divergence: when not null, the recovered wind (element 3-vectors)
  double* partials;  // [channel][block] sums of squares over the free nodes
  int nx, ny, nz;
  double c[3];
  Faces faces;
  int gx, gy;        // tile grid
  int tf;            // 1: terrain-following grid (x depends on i only, y on j only)
  const int* tf_flag;  // device flag (0 = terrain-following) for kernels told at run time
};

struct RecoverJob {  // u = u0 + diag(c) grad lambda at element centres
  const double* X;
  const double* Y;
  const double* Z;
  const double* lam;
  const double* u0;
  double* u;
  int nx, ny, nz;
  double c[3];
  int gx, gy;
};

// Work list of a batched launch: job j owns global blocks [prefix[j], prefix[j+1]);
// member[j] indexes the per-member active flags.
struct CgJob {  // conjugate-gradient vectors of one batch member (level 0, row-split order)
  void* e;           // correction
  void* p;           // direction
  const void* z;     // preconditioned residual
  void* r;           // residual
  const void* q;     // -K p
  double* sc;        // 4 device scalars {r.z, alpha, beta, r.r}
  double* partials;  // the member's partial-sum buffer
  size_t n;          // vector length
  int nblocks;       // blocks of the vector kernels, cg_blocks(n)
  int res_blocks;    // blocks of the member's q = -K p launch
  int member;
};

struct WorkList {
  const void* jobs;
  const int* prefix;
  const int* member;
  const int* active;
  int njobs;
  int total;
};

struct Level {
  Dims d;
  std::vector<int> keep_z;  // kept planes towards the next level (empty at the coarsest)
  int coarsen_h = 0;
  DevBuf st64;              // SW x N FP64 stencil (node-major, rows split even/odd in x)
  DevBuf st32;              // SW32 x N FP32 stencil (FP32_REFINE)
  DevBuf st16;              // SW16 x N FP16 stencil (FP32_REFINE with stencil_fp16), scaled by 1/st_scale
  float st_scale = 1.f;
  DevBuf x, f, r;           // level vectors in V-cycle precision, row-split order
  DirMap mx, my, mz;        // to the next coarser level
  DevBuf maps;              // device copies of the three DirMaps
  DirMapDev dmx{}, dmy{}, dmz{};
  // tuned tile shapes: rows of 64 columns per block of the colour pass (0: the
  // fused two-colour pass, one block per row) and of the residual
  int by_gs = 0, by_res = 4;
  double h1 = 0, h2 = 0;
  std::vector<double> h3;
};

}  // namespace mcw

struct mcw_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  mcw_options opt{};         // opt.tune_cache is cleared; the path is kept below
  std::string tune_cache;    // the autotuner's cache file (tune_cache_set: given in the options)
  bool tune_cache_set = false;
  mcw::Dims d{};
  mcw::Faces faces{};
  double a[3]{};
  double c[3]{};  // a_d^-2
  mcw::DevBuf X, Y, Z;
  std::vector<mcw::Level> levels;
  // coarsest level direct solve: inverse of K_L on its free nodes (FP64)
  int n_coarse = 0;
  mcw::DevBuf coarse_inv;   // n_coarse x n_coarse, symmetric
  mcw::DevBuf coarse_idx;   // n_coarse node numbers of the free coarsest nodes
  // FP64 outer-loop work vectors (fine level)
  mcw::DevBuf f64, r64, t64;
  // reductions
  mcw::DevBuf partials;     // per-block partial sums (double)
  mcw::DevBuf scalars;      // device results of reductions
  size_t n_partials = 0;
  double* host_scalars = nullptr;  // pinned
  mcw::DevBuf flag;         // geometry check result
  bool terrain = false;     // x of every node depends on i only and y on j only
  hipEvent_t ev[8]{};
  // hipGraph of one FP32 V-cycle (level vectors are fixed per handle)
  hipGraphExec_t vgraph = nullptr;
  bool vgraph_ready = false;
  // conjugate gradients (krylov = 1): level-0 vectors in the row-split order;
  // FP32 refinement keeps r and z in the level-0 f and x
  mcw::DevBuf kr, kz, kp, kq, ke;
  hipGraphExec_t kgraph = nullptr;  // one CG step
  bool kgraph_ready = false;
  // V-cycle rate measured at set-up (FP32 refinement with the plain iteration;
  // 0 = not measured): the first cycle count of every solve is chosen from it
  double rho_setup = 0.0;
  std::string last_error;
};

namespace mcw {

// ---------------------------------------------------------------- launchers (kernels.hip)

// Element geometry and element-tile kernels
void launch_geometry_check(const mcw_handle& h, long long* first_bad);
void launch_assemble_stencil(const mcw_handle& h, double* st64);
void launch_apply(const mcw_handle& h, const double* x, const double* f, double* out, int mode,
                  double* partials, size_t* n_part);
void launch_rhs(const mcw_handle& h, const double* u0, double* f, double* partials, size_t* n_part);
// With u not null the same launch also writes the recovered wind u = u0 +
// diag(c) grad lambda(centre), bit for bit what launch_recover writes.
void launch_divergence(const mcw_handle& h, const double* u0, const double* lam, double* D,
                       double* partials, size_t* n_part, double* u = nullptr);
// The geometry the element-tile kernels read, without a handle: node
// coordinates in place, dimensions, coefficients a_d^-2 and Gamma.
struct GridRef {
  const double *X, *Y, *Z;
  Dims d;
  double c[3];
  Faces faces;
  int tf;              // 1: terrain-following (x depends on i only, y on j only)
  const int* tf_flag;  // or, when not null, a device flag that says so (0 = terrain-following)
};
// Blocks of an element-tile launch on a grid (one partial sum per block and channel).
size_t tile_count(const Dims& d);
// *flag |= 1 if some node's x differs from that of its (i, 0, 0) node or its y
// from that of its (0, j, 0) node, i.e. the grid is not terrain-following.
void launch_structure_check(const double* X, const double* Y, const Dims& d, int* flag,
                            hipStream_t s);
// Weak divergence with 2 partial sums per block written to partials[0 .. 2 tile_count).
void launch_divergence_ref(const GridRef& G, const double* u0, const double* lam, double* D,
                           double* partials, hipStream_t s, double* u = nullptr);
void launch_recover(const mcw_handle& h, const double* u0, const double* lam, double* u);
// Steps around the solve (coupling_kernels.hip)
bool launch_coarse_check(const mcw_handle& h, const mcw_coarse_wind& cw);
void launch_interp_wind(const mcw_handle& h, const mcw_coarse_wind& cw, double* u0);
void launch_surface_wind(const mcw_handle& h, const double* u, double height, double z0, double* uv);
void launch_adjoint_scatter(const mcw_handle& h, const double* g_u, double* g_lam, double* partials,
                            size_t* n_part);
void launch_adjoint_elements(const mcw_handle& h, const double* g_u, const double* lam,
                             const double* mu, float* dL_du0, double* partials, size_t* n_part);
void launch_check_finite(const mcw_handle& h, const double* v, size_t n, double* partials,
                         size_t* n_part);

// element-tile modes and batched element launches
enum TileMode { M_APPLY = 0, M_RESID = 1, M_RHS = 2, M_DIV = 3, M_ADJ = 4 };
TileJob tile_job(const mcw_handle& h);
RecoverJob recover_job(const mcw_handle& h, const double* u0, const double* lam, double* u);
void launch_tile_batched(int mode, const WorkList& W, hipStream_t s);
void launch_recover_batched(const WorkList& W, hipStream_t s);

// Multigrid kernels (templated on the V-cycle precision)
// line_buf: null for the point smoother; for the vertical line smoother a
// level-sized scratch vector (the elimination coefficients)
// r_last: when given (forward sweeps only), the sweep also leaves r = f - K x
// on the columns whose residual it already knows: those of the last colour,
// (1,1), which no later pass changes (returns 1), and, where the odd rows run
// as one two-colour launch of the point smoother, those of (0,1) too, whose
// only later change is the (1,1) pass of the same launch (returns 2: every odd
// row holds r).  launch_residual given that value computes only the rest.
// Returns 0 without r_last.
template <class T>
int launch_smooth_sweep(const Dims& d, const Faces& fc, StRef st, const T* f, T* x,
                        hipStream_t s, int by = 0, bool reverse = false, T* line_buf = nullptr,
                        T* r_last = nullptr);
// preconditioned conjugate gradients; sc = device scalars {r.z, alpha, beta, r.r}
void launch_cg_reset(double* sc, hipStream_t s);
template <class T>
void launch_cg_beta(const T* z, const T* r, const T* q, size_t n, double* partials, size_t cap,
                    double* sc, hipStream_t s);
void launch_cg_alpha(size_t n_part, const double* partials, double* sc, hipStream_t s);
template <class T>
void launch_add(T* y, const T* x, size_t n, hipStream_t s);
template <class T>
void launch_cg_direction(T* p, const T* z, const double* sc, size_t n, hipStream_t s);
template <class T>
void launch_cg_update(T* e, const T* p, T* r, const T* q, double* sc, size_t n, double* partials,
                      size_t cap, hipStream_t s);
template <class T>
void launch_neg_apply_dot(const Dims& d, const Faces& fc, StRef st, const T* p, T* q,
                          double* partials, size_t cap, size_t* n_part, hipStream_t s, int by);
// A V-cycle residual job after a sweep that left r on some columns (mode 1:
// the (1,1) ones; 2: every odd row, and the job then covers the even rows only).
void residual_skip(ColJob& J, int mode);
template <class T>
void launch_residual(const Dims& d, const Faces& fc, StRef st, const T* x, const T* f, T* r,
                     double* partials, size_t* n_part, hipStream_t s, int by = 4, size_t cap = 0,
                     int last_colour_done = 0);
template <class T>
void launch_restrict(const Dims& df, const Dims& dc, const Faces& fc, const DirMapDev& mx,
                     const DirMapDev& my, const DirMapDev& mz, const T* r, T* rc, hipStream_t s);
template <class T>
void launch_prolong_dims(const Dims& df, const Dims& dc, const Faces& fc, const DirMapDev& mx,
                         const DirMapDev& my, const DirMapDev& mz, const T* e, T* x,
                         hipStream_t s);
template <class T>
void launch_coarse_solve(int n, const double* inv, const int* idx, const T* r, T* e, hipStream_t s);
template <class T>
void launch_fill(T* p, size_t n, T v, hipStream_t s);

void launch_rap(const Dims& df, const Dims& dc, const DirMapDev& mx, const DirMapDev& my,
                const DirMapDev& mz, const double* stf, double* stc, hipStream_t s);
void launch_round_stencil(const Dims& d, const double* st64, float* st32, hipStream_t s);
// largest |off-diagonal coefficient| of an FP64 stencil (device work, result on the host)
double stencil_absmax(const Dims& d, const double* st64, double* scratch, hipStream_t s);
// FP16 copy of an FP64 stencil's off-diagonals, each divided by scale (a power of two)
void launch_round_stencil16(const Dims& d, const double* st64, uint16_t* st16, double inv_scale,
                            hipStream_t s);
// natural-order (27, N) copy: kind 0 FP32, 1 FP64, 2 FP16 times scale (written as FP32)
void launch_unsplit_stencil(const Dims& d, const void* st, void* out, int kind, hipStream_t s,
                            float scale = 1.f);
// r32 (row-split) = (float)(r * *scale); lam += e (row-split) / *scale (device scalar)
void launch_scale_to_f32(const Dims& d, const double* r, const double* scale, float* r32,
                         hipStream_t s);
void launch_update_lambda(const Dims& d, const float* e, const double* scale, double* lam,
                          hipStream_t s);
// natural <-> row-split copies of level vectors
template <class T>
void launch_relayout(const Dims& d, const T* src, T* dst, bool to_split, hipStream_t s);
void launch_axpy64(size_t n, double alpha, const double* x, double* y, hipStream_t s);
void launch_zero_fixed(const Dims& d, const Faces& fc, double* v, hipStream_t s);
// p[i] = pseudo-random values in [-1, 1), a fixed function of i and seed.
void launch_hash_fill(double* p, size_t n, unsigned long long seed, hipStream_t s);
void launch_sum_partials(const double* partials, size_t n_part, int width, double* out,
                         hipStream_t s);

// Job builders (colour = -1: all columns)
ColJob col_job(const Dims& d, const Faces& fc, StRef st, const void* f, void* x, void* r,
               int colour, int by = 4);
XferJob xfer_job(const Dims& df, const Dims& dc, const Faces& fc, const DirMapDev& mx,
                 const DirMapDev& my, const DirMapDev& mz, const void* src, void* dst,
                 bool restriction);
CoarseJob coarse_job(int n, const double* inv, const int* idx, const void* r, void* e);
VecJob vec_job(void* p, const void* q, size_t n, const double* scale);

// Batched (persistent) launches over a work list of jobs
// h16: every job of W has FP16 stencils (else none has); the batched colour
// pass, residual and q = -K p run the kernel instance of that format
// side: the (1,1) pass of the sweep that ends the pre-smoothing, with the jobs'
// rlast and rside set; launch_side_residual_batched then finishes the (0,1)
// columns of the jobs of colour (0,1) (rlast set) that ran before it
template <class T> void launch_gs_batched(const WorkList& W, hipStream_t s, int by, bool reverse, bool h16,
                                          bool side = false);
template <class T> void launch_side_residual_batched(const WorkList& W, hipStream_t s, int by, bool h16);
// batched conjugate gradients (lists of CgJob; residual lists of ColJob with part set)
unsigned cg_blocks(size_t n);
template <class T> void launch_dot2_batched(const WorkList& W, hipStream_t s);
template <class T> void launch_cg_direction_batched(const WorkList& W, hipStream_t s);
template <class T> void launch_cg_update_batched(const WorkList& W, hipStream_t s);
template <class T> void launch_neg_apply_dot_batched(const WorkList& W, hipStream_t s, int by, bool h16);
void launch_cg_coeff_batched(const CgJob* jobs, int n, int mode, const int* active, hipStream_t s);
void launch_cg_reset_batched(const CgJob* jobs, int n, const int* active, hipStream_t s);
template <class T> void launch_residual_batched(const WorkList& W, hipStream_t s, int by, bool h16);
// FusedJob work items: colour J0 then J1 of one row per block (as gs_fused_kernel)
// side: the odd-row launch of the sweep that ends the pre-smoothing, with the
// jobs' rlast and rside set (gs_fused_kernel with SIDE)
template <class T> void launch_gs_fused_batched(const WorkList& W, hipStream_t s, bool reverse, bool h16,
                                                bool side = false);
template <class T> void launch_restrict_batched(const WorkList& W, hipStream_t s);
template <class T> void launch_prolong_batched(const WorkList& W, hipStream_t s);
template <class T> void launch_coarse_batched(const WorkList& W, int max_n, hipStream_t s);
template <class T> void launch_fill_batched(const WorkList& W, hipStream_t s);
void launch_scale_batched(const WorkList& W, hipStream_t s);
void launch_update_batched(const WorkList& W, hipStream_t s);
void launch_zero_fixed_batched(const WorkList& W, hipStream_t s);
void launch_sum_batched(const SumJob* jobs, int n, hipStream_t s);

}  // namespace mcw
