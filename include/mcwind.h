/*
 * mcwind -- mass-consistent wind downscaling on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libmcwind.so.  The library solves the finite element form of the
 * problem of Mandel, Farguell, Kochanski, Mallia and Hilburn, "Simple finite
 * elements and multigrid for efficient mass-consistent wind downscaling in a
 * coupled fire-atmosphere model":
 *
 *   find the wind u closest to u0 in the norm weighted by A = diag(a_d^2)
 *   subject to div u = 0 in the domain and u.n = 0 on the surface Gamma
 *   (Sec. 2, eq. (1)),
 *
 * through its Lagrange multiplier lambda, which solves the generalized
 * Poisson problem -div A^-1 grad lambda = div u0 with lambda = 0 on the
 * boundary outside Gamma (eq. (4)) in the variational form of eq. (5),
 * discretised by isoparametric trilinear hexahedra (2x2x2 Gauss stiffness,
 * one-point right-hand side), solved by multigrid with 4-colour vertical
 * Gauss-Seidel smoothing and variational coarse-grid correction with adaptive
 * semicoarsening (Sec. 3, eqs. (6)-(7)); the wind is recovered at element
 * centres as u = u0 + A^-1 grad lambda (eq. (3)).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Grid: nx x ny x nz hexahedral elements on a logically Cartesian grid of
 *   N = (nx+1)(ny+1)(nz+1) nodes.  Node arrays are x fastest: node (i,j,k) is
 *   entry i + (nx+1)*(j + (ny+1)*k).  Elements must be right-handed
 *   (i, j, k increasing along x, y, z), i.e. det J > 0 everywhere.
 * Element arrays (u0, u, gradients) are structure of arrays (3, nz, ny, nx):
 *   component d of element (i,j,k) is entry i + nx*(j + ny*(k + nz*d)).
 * Gamma: bit mask of grid faces where u.n = 0 is imposed (lambda free):
 *   bit 0 bottom k=0, bit 1 top k=nz, bit 2 x-low i=0, bit 3 x-high i=nx,
 *   bit 4 y-low j=0, bit 5 y-high j=ny.  lambda = 0 at every node on a face
 *   outside Gamma (edges shared with Gamma included).  The paper's setting is
 *   MCW_GAMMA_BOTTOM.
 * Memory: every array pointer is a DEVICE pointer on the device that was
 *   current at mcw_create, unless the parameter says "host".  The caller
 *   owns all arrays; the handle owns its hierarchy, operators and workspace.
 * Streams: the handle runs all work on the stream given to mcw_create (a
 *   hipStream_t passed as void*, NULL = default stream).  Entry points return
 *   after the work is complete unless stated otherwise.
 * Errors: every call returns an mcw_status; nothing throws across the ABI.
 *   mcw_last_error() gives a message for the last failing call on the handle
 *   (or for a failed mcw_create, mcw_last_error(NULL)).
 * Threads: one host thread at a time per handle.
 */
#ifndef MCWIND_H
#define MCWIND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MCW_OK = 0,
  MCW_INVALID_ARG = 1,    /* null pointer, nx/ny < 2, nz < 1, a_d <= 0 or non-finite, bad option */
  MCW_BAD_GEOMETRY = 2,   /* det J <= 0 at a Gauss point or centre; message names the element */
  MCW_SINGULAR = 3,       /* Gamma covers the whole boundary: lambda is defined up to a constant */
  MCW_NONFINITE = 4,      /* NaN or Inf in the right-hand side or the residual */
  MCW_NOT_CONVERGED = 5,  /* max_cycles reached; lambda holds the last iterate, info the residual */
  MCW_OOM = 6,            /* device allocation failed */
  MCW_HIP_ERROR = 7       /* a HIP runtime call failed; message has hipGetErrorString */
} mcw_status;

#define MCW_GAMMA_BOTTOM 1u
#define MCW_GAMMA_TOP 2u
#define MCW_GAMMA_XLO 4u
#define MCW_GAMMA_XHI 8u
#define MCW_GAMMA_YLO 16u
#define MCW_GAMMA_YHI 32u

typedef enum {
  MCW_FP64 = 0,        /* all multigrid work in FP64 */
  MCW_FP32_REFINE = 1  /* FP32 V-cycles inside FP64 iterative refinement */
} mcw_precision;

typedef enum {
  /* coupling ratio a3*h3 / (a_h*h_h) of the assembled operator (coefficient a_d^-2) */
  MCW_COARSEN_OPERATOR = 0,
  /* the ratio printed in Sec. 3: a_h*h3 / (h_h*a3) */
  MCW_COARSEN_LITERAL = 1,
  /* base method of Sec. 3: coarsen every direction by 2 */
  MCW_COARSEN_FULL = 2
} mcw_coarsen_rule;

typedef enum {
  /* the layer test of the semicoarsening rule (Sec. 3) compares each layer with
     the horizontal spacing of the level being coarsened, so that both thresholds
     bound the coupling anisotropy of the grid the smoother runs on by 9 */
  MCW_MERGE_LEVEL_SPACING = 0,
  /* it compares with the spacing after the horizontal step (twice the level's
     when the level coarsens horizontally), as printed in Sec. 3: merged pairs
     can then reach coupling anisotropy 36, and the cycle converges more slowly
     on stretched layers */
  MCW_MERGE_COARSENED_SPACING = 1
} mcw_merge_spacing;

typedef enum {
  /* Sec. 3: pointwise Gauss-Seidel, each column from the bottom up, colours
     (0,0),(1,0),(0,1),(1,1) */
  MCW_SMOOTH_POINT = 0,
  /* vertical line Gauss-Seidel: each column's free nodes solved together
     (tridiagonal in the column), the neighbour columns held fixed, same colours */
  MCW_SMOOTH_LINE = 1
} mcw_smoother;

/* Problem statement (Sec. 2): node coordinates, penalties, Gamma. */
typedef struct {
  int32_t nx, ny, nz;     /* elements per direction; nx, ny >= 2, nz >= 1; ny <= 262140,
                             nz <= 4096, (nx+1)(ny+1) <= 2^30 */
  const double* X;        /* device, N node x-coordinates (copied by mcw_create) */
  const double* Y;        /* device, N node y-coordinates */
  const double* Z;        /* device, N node z-coordinates */
  double a[3];            /* penalty constants a_1, a_2, a_3 > 0 (A = diag(a_d^2)) */
  uint32_t gamma_faces;   /* MCW_GAMMA_* mask; must not contain all six faces */
} mcw_grid_desc;

typedef struct {
  int32_t precision;          /* mcw_precision; default MCW_FP32_REFINE */
  double rtol;                /* stop when ||f - K lambda||_2 <= rtol ||f||_2 (free nodes); default 1e-8 */
  int32_t max_cycles;         /* V-cycles per solve before MCW_NOT_CONVERGED; default 200 */
  int32_t nu_pre, nu_post;    /* Gauss-Seidel sweeps before / after the coarse correction; default 2, 2 */
  int32_t inner_cycles;       /* FP32 V-cycles per refinement step; 0 = chosen from the V-cycle
                                 rate (measured at set-up from a fixed pseudo-random right-hand
                                 side, then from the solve's own refinement steps) */
  int32_t coarsen_rule;       /* mcw_coarsen_rule; default MCW_COARSEN_OPERATOR */
  int32_t coarse_direct_max;  /* largest coarsest-level unknown count (direct solve); default 1024, max 4096 */
  int32_t use_graph;          /* capture the FP32 V-cycle in a hipGraph and replay it; default 1 */
  int32_t verbose;            /* print setup and convergence lines to stderr; default 0 */
  int32_t autotune;           /* time tile shapes of the colour pass and residual per level at
                                 set-up and keep the fastest (cached in the file tune_cache
                                 names); before that,
                                 on every level of at least 2^22 nodes, time up to 6 physical
                                 placements of its stencil and vectors (fresh allocations) and
                                 keep the fastest: set-up then holds up to 5 extra copies of
                                 that level's stencil and vectors until the level is done, and
                                 stops early when free memory is short.  Results do not depend
                                 on either choice; default 1 */
  int32_t krylov;             /* 0: the multigrid iteration of Sec. 3 (default); 1: conjugate
                                 gradients preconditioned by one symmetric V-cycle (the
                                 post-smoothing sweeps run in reverse: colours 3..0, each
                                 column top-down), restarted at every refinement step;
                                 needs nu_pre == nu_post */
  int32_t smoother;           /* mcw_smoother; default MCW_SMOOTH_POINT */
  int32_t stencil_fp16;       /* FP32_REFINE only.  0 (default): the V-cycle's stencils are FP32.
                                 1: they are kept in FP16 (50 instead of 100 bytes per node), each
                                 level's off-diagonals divided by a power of two above their
                                 largest magnitude; the V-cycle still computes in FP32 and the
                                 refinement in FP64, so the solution meets rtol as before.  One
                                 refinement step then reduces the residual by at most about 1e-3
                                 (3e-5 with FP32 stencils).  Not part of the paper's method. */
  int32_t merge_spacing;      /* mcw_merge_spacing; default MCW_MERGE_LEVEL_SPACING */
  const char* tune_cache;     /* host string, the autotuner's JSON cache file; NULL = the file
                                 named by the environment variable MCW_TUNE_CACHE, else
                                 ~/.cache/mcwind/tune.json; "" = no cache.  Copied by mcw_create. */
} mcw_options;

#define MCW_MAX_LEVELS 24
#define MCW_HISTORY 64

typedef struct {
  int32_t outer_steps;            /* FP64 residual evaluations after the start */
  int32_t cycles;                 /* V-cycles performed (with krylov = 1: CG steps, one V-cycle each) */
  double rel_residual;            /* final ||f - K lambda|| / ||f|| (FP64, free nodes) */
  double rel_divergence;          /* ||D|| / ||D0||, D the weak divergence of u0 + A^-1 grad lambda */
  double rho;                     /* mean residual reduction per V-cycle */
  double f_norm;                  /* ||f||_2 over the free nodes */
  int32_t n_levels;
  int32_t level_dims[MCW_MAX_LEVELS][3];
  int32_t n_history;
  double history[MCW_HISTORY];    /* relative residual after each outer step (FP64) */
  float ms_total;                 /* device time of the whole solve */
  float ms_rhs;                   /* right-hand side assembly */
  float ms_cycles;                /* V-cycles (incl. casts/updates) */
  float ms_outer;                 /* FP64 matrix-free residuals */
  float ms_finish;                /* recovery and divergence check */
  int32_t status;                 /* mcw_status of this solve; for a batch, the member's own */
} mcw_info;

typedef struct mcw_handle mcw_handle;

/* Fill o with the defaults listed above. */
void mcw_default_options(mcw_options* o);

/* Set up a grid (Sec. 2, discretisation of eq. (5); Sec. 3, coarsening rule
 * and eq. (7) for the coarse operators): validates the
 * arguments, checks det J > 0 at every Gauss point and element centre,
 * assembles the 27-point fine stiffness stencil from 2x2x2 Gauss quadrature,
 * chooses the coarse grids by the coarsening rule, forms the Galerkin
 * operators K_c = P^T K P and factors the coarsest one.  A coarse level always
 * keeps a free node: where pairing layers between a fixed bottom and a fixed
 * top would leave none, every plane is kept.  A grid with no free node at all
 * (one layer with both z faces fixed, say) is accepted: its solves return
 * lambda = 0 and u = u0.  opts may be NULL (defaults).  stream is a hipStream_t or NULL.  On success *out owns all of
 * the handle's device memory until mcw_destroy. */
mcw_status mcw_create(const mcw_grid_desc* g, const mcw_options* opts, void* stream,
                      mcw_handle** out);

void mcw_destroy(mcw_handle* h);

/* Change the stopping tolerance and cycle limit of later solves on h
 * (rtol in (0,1), max_cycles >= 1); the hierarchy and operators are kept. */
mcw_status mcw_set_tolerance(mcw_handle* h, double rtol, int32_t max_cycles);

/* Solve for the multiplier and recover the wind (Sec. 2): lambda solves the
 * discrete eq. (5) with lambda = 0 on the boundary outside Gamma (eq. (4)),
 * by the multigrid iteration of Sec. 3 (eqs. (6)-(7)), and u follows from
 * eq. (3) at the element centres.
 * u0:     device, (3, nz, ny, nx) FP64 initial wind at element centres.
 * lambda: device, N FP64; on entry the starting guess (warm start from the
 *         previous time step; zeros = cold start; entries at fixed nodes are
 *         ignored), on exit the solution with zeros at fixed nodes.
 * u:      device, (3, nz, ny, nx) FP64 output wind; may be NULL (skips recovery).
 * info:   host, may be NULL.
 * Returns MCW_NOT_CONVERGED with lambda = last iterate if rtol is not reached
 * in max_cycles V-cycles, MCW_NONFINITE if u0 or the iteration is not finite. */
mcw_status mcw_solve(mcw_handle* h, const double* u0, double* lambda, double* u, mcw_info* info);

/* Solve m independent problems (an ensemble or several time steps), each as
 * in mcw_solve (Sec. 2, eqs. (3)-(5); Sec. 3, eqs. (6)-(7)) on its own
 * handle, advancing them together: every multigrid phase is one
 * launch over all members that still iterate.  Arrays as in mcw_solve, one
 * per member (host arrays of device pointers); u may be NULL, and so may u[i]
 * (that member's recovery is skipped); infos may be NULL or hold m entries,
 * each with the member's own status.  Each member stops on its own rtol and
 * runs at most its own max_cycles, as when solved alone.  All handles must
 * share one device, precision and smoothing counts; the stream of hs[0] is used.
 * FP32_REFINE members with krylov = 1 run batched CG, each member stopping
 * on its own residual; FP64 handles, line-smoother handles and batches that
 * mix CG with the plain iteration are solved one member after another.
 * Returns the first non-OK member status. */
mcw_status mcw_solve_batch(int32_t m, mcw_handle* const* hs, const double* const* u0,
                           double* const* lambda, double* const* u, mcw_info* infos);

/* Reverse mode through the solve: the chain rule through eq. (3) (recovery)
 * and the discrete eq. (5) (lambda from u0 and a).  With g_lambda = G^T
 * A^-1 g_u, the transpose problem K mu = g_lambda has the same symmetric
 * operator and is solved by the same multigrid iteration; then
 * dL/du0 = g_u - 8 detJ(0) B(0) mu and dL/da_d follows from the derivatives
 * of K and of A^-1 in eq. (3) (the coefficients are a_d^-2).
 * lambda: device N FP64, the solution of mcw_solve for this u0 and handle.
 * g_u:    device (3, nz, ny, nx) FP64, dL/du at element centres.
 * dL_du0: device (3, nz, ny, nx) FP32 output.
 * dL_da:  host double[3] output, dL/da_d.
 * info:   host, may be NULL (describes the transpose solve). */
mcw_status mcw_adjoint(mcw_handle* h, const double* lambda, const double* g_u, float* dL_du0,
                       double dL_da[3], mcw_info* info);

/* ---- single-step entry points (each runs one operation of the path) ---- */

/* y = K x, K the stiffness matrix of the left side of eq. (5) (Sec. 2:
 * 2x2x2 Gauss quadrature), by the matrix-free element-by-element apply, FP64,
 * full node vectors, no boundary conditions applied (rows of fixed nodes are
 * the unconstrained stiffness rows). */
mcw_status mcw_apply_K(mcw_handle* h, const double* x, double* y);

/* f = right-hand side of eq. (5) by one-point quadrature: f_a = -sum_e
 * 8 detJ_e(0) (B_e(0)^T u0_e)_a at free nodes, 0 at fixed nodes. */
mcw_status mcw_rhs(mcw_handle* h, const double* u0, double* f);

/* u = u0 + A^-1 grad lambda at element centres (eq. (3)). */
mcw_status mcw_recover(mcw_handle* h, const double* u0, const double* lambda, double* u);

/* Weak divergence D of u0 + A^-1 grad lambda: the constraint div u = 0 of
 * eq. (1) tested with every free hat function, i.e. eq. (5) moved to one side
 * (each term with its own quadrature, Sec. 2), at all nodes (0 at fixed
 * nodes), and rel = ||D|| / ||D0|| over the free nodes, D0 the u0 term (host
 * double, may be NULL).  D = -(f - K lambda), so rel equals the relative
 * residual of the solve. */
mcw_status mcw_divergence(mcw_handle* h, const double* u0, const double* lambda, double* D,
                          double* rel);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * divergence check of mcw_divergence without a handle and without any
 * allocation.  g describes the grid as for mcw_create, but X, Y, Z are read in
 * place (not copied) and det J is not checked.  u0, lambda, D and rel as in
 * mcw_divergence.  stream: a hipStream_t or NULL.  With rel non-NULL the call
 * returns when the work is complete; with rel NULL it only enqueues the work
 * on the stream (nothing waits, so the call can be captured).
 * The per-block partial sums live in one fixed device array of the library,
 * MCW_NOALLOC_SCRATCH_BYTES on every device it runs on, held until the process
 * ends: grids of more than MCW_NOALLOC_MAX_TILES element tiles (15 x 15 node
 * columns each, i.e. ceil((nx+1)/15) * ceil((ny+1)/15)) give MCW_INVALID_ARG.
 * Calls that overlap on one device share that array and race. */
#define MCW_NOALLOC_SCRATCH_BYTES (2u << 20)
#define MCW_NOALLOC_MAX_TILES ((MCW_NOALLOC_SCRATCH_BYTES / 8u - 3u) / 2u)
mcw_status mcw_divergence_noalloc(const mcw_grid_desc* g, const double* u0, const double* lambda,
                                  double* D, double* rel, void* stream);

/* ---- steps on either side of the solve (coupled fire-atmosphere model) ----
 * The solve takes the place of plainly interpolating the atmospheric model's
 * wind to the fire model's grid (Sec. 1).  These two calls are that
 * interpolation, giving the solve's u0, and the fire model's read-out of the
 * solved wind.  Heights are above the ground: an element centre (the mean of
 * its 8 corner nodes) minus the mean height of its column's 4 bottom nodes.
 * Vertically, values are linear in height between levels, equal to the top
 * level above it, and follow the neutral log law v(h1) ln(z/z0) / ln(h1/z0)
 * below the lowest level h1 (0 at z <= z0). */
typedef struct {
  int32_t ncx, ncy;      /* coarse columns along x and y, >= 2 each */
  int32_t nl;            /* levels per column, >= 1 */
  double x0, y0;         /* horizontal position of column (0, 0) */
  double dx, dy;         /* column spacing, > 0 */
  double z0;             /* roughness length of the log law, > 0 */
  const double* hagl;    /* device, (nl, ncy, ncx): level heights above ground, increasing
                            up each column, all > z0 */
  const double* wind;    /* device, (3, nl, ncy, ncx): wind components at the levels */
} mcw_coarse_wind;

/* The atmospheric model's wind brought to the fire grid, the input u0 of
 * eq. (1) (Sec. 1 places the solve after this step).
 * u0 (device, (3, nz, ny, nx)) at the element centres from the coarse wind:
 * at each centre, the wind of the four coarse columns around it (bilinear
 * weights; positions outside the column grid take its edge) at the centre's
 * height above ground.  MCW_INVALID_ARG if the level heights do not increase
 * or do not start above z0. */
mcw_status mcw_interp_wind(mcw_handle* h, const mcw_coarse_wind* cw, double* u0);

/* The fire model's read-out of the solved wind (Sec. 1).
 * uv (device, (2, ny, nx)): the horizontal wind u[0], u[1] (device,
 * (3, nz, ny, nx), element centres) at `height` > 0 above the ground over
 * each element column, by the vertical rule above on the column's centres. */
mcw_status mcw_surface_wind(mcw_handle* h, const double* u, double height, double z0, double* uv);

/* The hierarchy of Sec. 3 (coarsening rule of its last paragraph).
 * Number of levels, and the dimensions of level l (host int32[3]: nx, ny, nz),
 * whether it coarsens horizontally towards level l+1 (host int32, may be NULL)
 * and its kept node planes (host int32[nz+1], may be NULL; count written to
 * *n_keep). */
int32_t mcw_num_levels(const mcw_handle* h);
mcw_status mcw_level_info(const mcw_handle* h, int32_t l, int32_t dims[3], int32_t* coarsen_h,
                          int32_t* keep_z, int32_t* n_keep);

/* The operator of level l: K of eq. (5) on level 0, K_c = P^T K P of eq. (7)
 * on the coarse levels.
 * Copy the 27-point stencil of level l into out: device, 27 x N_l, entry
 * o*N_l + n holds K[n, n + offset(o)] with o = (di+1) + 3(dj+1) + 9(dk+1), in
 * natural node order.  prec = MCW_FP64 gives the FP64 operator (available in
 * FP64 handles; for FP32_REFINE handles only level 0, recomputed), MCW_FP32_REFINE the
 * FP32 operator of the V-cycles (out is then float*): off-diagonals rounded once
 * from FP64, except that the coupling to the node below (o = 4) is the node
 * below's rounded coupling to the node above (o = 22; zero on the bottom plane),
 * and the diagonal minus the off-diagonal sum; with stencil_fp16 the FP16 values
 * times the level's scale, defined the same way. */
mcw_status mcw_get_stencil(mcw_handle* h, int32_t l, int32_t prec, void* out);

/* The smoother of Sec. 3 (vertical Gauss-Seidel sweeps in four horizontal
 * red-black groups).
 * |sweeps| Gauss-Seidel sweeps on level l in the handle's precision of the
 * V-cycle (double* for MCW_FP64 handles, float* for MCW_FP32_REFINE): x in/out,
 * f in, level-sized node vectors.  sweeps > 0: the smoother of Sec. 3 (colours
 * (0,0),(1,0),(0,1),(1,1), each column bottom-up); sweeps < 0: the reverse
 * (adjoint) sweep, colours (1,1),(0,1),(1,0),(0,0), each column top-down.
 * |sweeps| <= 1000. */
mcw_status mcw_smooth(mcw_handle* h, int32_t l, void* x, const void* f, int32_t sweeps);

/* r = f - K_l x at free nodes, 0 at fixed nodes (V-cycle precision): the
 * residual whose restriction is the coarse right-hand side of eq. (7). */
mcw_status mcw_residual(mcw_handle* h, int32_t l, const void* x, const void* f, void* r);

/* rc = P_l^T r (level l+1 vector, 0 at fixed coarse nodes): f_c of eq. (7),
 * P the regular-grid linear interpolation of Sec. 3. */
mcw_status mcw_restrict(mcw_handle* h, int32_t l, const void* r, void* rc);

/* x += P_l e (x level l, e level l+1): the correction step of eq. (7). */
mcw_status mcw_prolong(mcw_handle* h, int32_t l, const void* e, void* x);

/* e = K_L^-1 r on the coarsest level (V-cycle precision, FP64 arithmetic):
 * K_c u_c = f_c of eq. (7) solved by a direct method (Sec. 3). */
mcw_status mcw_coarse_solve(mcw_handle* h, const void* r, void* e);

/* One V-cycle on level 0 with x in/out, f in (V-cycle precision): smoothing,
 * the coarse-grid correction of eqs. (6)-(7) applied recursively, smoothing
 * (Sec. 3).  The residual that is restricted is f - K x after the
 * pre-smoothing; where the last pre-smoothing sweep already knows it (the odd
 * rows with the point smoother, the (1,1) columns with the line smoother) it
 * is formed from that sweep's updates, which differs from computing f - K x
 * only by rounding. */
mcw_status mcw_vcycle(mcw_handle* h, void* x, const void* f);

/* Run `reps` launches of one multigrid kernel on level l's own buffers (their
 * current contents; no layout conversion, no allocation) and wait: kernel 0 =
 * one Gauss-Seidel sweep (4 colour passes, in 2 launches when the level uses
 * the fused two-colour pass), 1 = residual, 2 = restriction to
 * level l+1, 3 = prolongation from level l+1, 4 = FP64 matrix-free residual
 * f - K lambda on the fine grid (l must be 0).  For timing and profiling. */
mcw_status mcw_run_kernel(mcw_handle* h, int32_t l, int32_t kernel, int32_t reps);

/* Run `reps` launches of one batched phase over the finest level of m handles
 * (as mcw_solve_batch runs it; all members take part, on their own level
 * buffers and current contents) and wait: kernel 0 = one Gauss-Seidel sweep
 * (two batched two-colour launches where the largest member's fine level uses
 * the fused pass, else four batched colour passes), 1 = the residual.
 * FP32_REFINE point-smoother members with equal krylov and smoothing counts.
 * ms_per_rep (host, may be NULL) receives the device time per repetition,
 * taken with HIP events on the batch's stream around the launches only;
 * launches_per_rep (host, may be NULL) the launches of one repetition per
 * stencil format.  For timing and profiling. */
mcw_status mcw_run_kernel_batch(int32_t m, mcw_handle* const* hs, int32_t kernel, int32_t reps,
                                float* ms_per_rep, int32_t* launches_per_rep);

/* Tile shape used on level l by the Gauss-Seidel colour pass and by the
 * residual (host int32 outputs): rows of 64 columns per block, and for the
 * colour pass 0 when it runs fused, two colours per launch with one block per
 * row of the grid (the autotuner's choice; default 0 for the colour pass and
 * 4 for the residual). */
mcw_status mcw_tile_shape(const mcw_handle* h, int32_t l, int32_t* rows_smooth, int32_t* rows_residual);

/* ---- errors ---- */
const char* mcw_status_string(mcw_status s);
const char* mcw_last_error(const mcw_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* MCWIND_H */
