/*
 * fsimg — MI355X (gfx950) library for the linear solves inside one
 * approximate Newton step of a monolithic ALE fluid-structure solver
 * (Failer & Richter, "A parallel Newton multigrid framework for monolithic
 * fluid-structure interactions", arXiv:1904.02401).
 *
 * The reduced Jacobian of Sec. 4.2 (eq. REDUCEDMATRIX) splits into
 *   (1) the momentum system in (p, v), eq. problem:1,
 *   (2) the deformation update on interface/solid dofs, eq. problem:2,
 *   (3) the ALE extension, eq. problem:3.
 * (1) and (3) (and, optionally, (2) as a mass-matrix system) are solved by
 * flexible GMRES (Sec. 4.3 (I)) preconditioned with a geometric multigrid
 * V-cycle (Sec. 4.3 (II)) whose smoother is the additive Vanka iteration on
 * element patches (eq. vanka, Sec. 4.3 (III)); (2) is one vector addition
 * (Sec. 3.1, condensation of the deformation).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are block-CSR (BSR) with square b x b blocks stored row-major,
 *   the block layout of the paper's linear-algebra module (Sec. 4.3: block
 *   vectors and block matrices with n_c x n_c blocks).  Structure arrays are
 *   int32; value offsets are computed in 64 bit.
 * - Vectors are node-major block vectors: entry (node, component) at
 *   node * b + component.  Momentum components are (p, v_1, .., v_d).
 * - Node numbering is lexicographic on a tensor-product Q2 mesh with
 *   2*cells[a]+1 nodes per axis, x fastest; a Vanka patch holds all dofs of
 *   the 3^d nodes of one cell (Sec. 4.3), or, with FSIMG_PATCH_BLOCK, of the
 *   5^d nodes of a 2 x 2 (x 2) block of cells (Sec. 5.5.1).  Level l+1 is the
 *   uniform coarsening of level l.
 * - Identity ("dirichlet") rows: at those dofs the solution keeps the value
 *   that x carries in; b is ignored there.  Inhomogeneous data (such as the
 *   interface deformation of eq. problem:3) are passed in through x.
 * - Device pointers: every vector argument named *_dev is device memory of
 *   the context's GPU, owned by the caller; the library never frees caller
 *   memory.  Host arrays in descriptors are copied during the call and may
 *   be freed on return.
 * - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *   stream).  Work is ordered on it.  Entry points that return results to
 *   the host (fsimg_solve, fsimg_factor) synchronise the stream.
 * - Errors: every entry point returns an fsimg_status; nothing is thrown or
 *   aborted across the ABI.  fsimg_last_error() gives a thread-local message.
 * - Threading: a context and its hierarchies may be used from one host
 *   thread at a time.  Calls on different hierarchies that share a stream
 *   serialise on that stream.
 */
#ifndef FSIMG_H
#define FSIMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FSIMG_OK = 0,
  FSIMG_ERR_ARG = 1,       /* invalid argument (sizes, pointers, options) */
  FSIMG_ERR_OOM = 2,       /* device allocation failed */
  FSIMG_ERR_HIP = 3,       /* a HIP runtime call failed */
  FSIMG_ERR_SINGULAR = 4,  /* zero / tiny pivot in a patch or coarse matrix */
  FSIMG_ERR_NOCONV = 5,    /* iteration limit reached; x holds the last iterate */
  FSIMG_ERR_NONFINITE = 6, /* NaN / Inf in the right-hand side or the iteration */
  FSIMG_ERR_BUDGET = 7,    /* the allocation would exceed the context's HBM budget */
  FSIMG_ERR_STATE = 8      /* call out of order (e.g. solve before factor) */
} fsimg_status;

typedef enum { FSIMG_FP64 = 0, FSIMG_MIXED = 1 } fsimg_precision;

/* How the overlapping patch corrections of one Vanka step are summed.
   GATHER: every patch writes its local correction, then one pass adds, per
   dof, the contributions of its patches in patch order (no colours needed).
   PARITY / GREEDY: patches are coloured so that patches of one colour share
   no node (Sec. 5.5.3); colours are applied one after another and write the
   solution directly.  PARITY uses the 2^d cell-parity colours, GREEDY the
   paper's greedy colouring with fluid and solid patches kept apart. */
typedef enum { FSIMG_VANKA_GATHER = 0, FSIMG_VANKA_PARITY = 1, FSIMG_VANKA_GREEDY = 2 } fsimg_vanka_schedule;

/* Summation weight of overlapping patch corrections (reading of eq. vanka):
   PLAIN adds them as printed; MULT divides the sum at each dof by the number
   of element patches that contain it. */
typedef enum { FSIMG_WEIGHT_PLAIN = 0, FSIMG_WEIGHT_MULT = 1 } fsimg_weighting;
/* Vanka patch shapes (Sec. 5.5.1, the patch-size study).  ELEMENT: one patch
   per element (3^d nodes).  BLOCK: the 5^d nodes of a 2 x 2 (x 2) block of
   elements at even element coordinates form one patch -- in 2D every such
   block, in 3D only blocks whose eight elements all have a nonzero
   cell_class (solid); elements outside blocks keep one-element patches.
   With MULT weighting a dof's correction is divided by the number of
   patches containing it.  BLOCK needs the GATHER schedule. */
typedef enum { FSIMG_PATCH_ELEMENT = 0, FSIMG_PATCH_BLOCK = 1 } fsimg_patches;
/* Multigrid smoother.  VANKA: the additive Vanka iteration above (Sec. 4.3).
   ILU: the comparison smoother of Sec. 5.5, read as a block incomplete LU
   without fill-in on the matrix's block pattern (one b x b block per coupled
   node pair, the matrix's node order), x += omega_ilu (L U)^{-1} (b - A x)
   with identity rows kept.  The factors are computed in FP64 by fsimg_factor
   (level-scheduled: rows whose lower-triangle couplings are all factored go
   together) and applied by level-scheduled triangular solves.  ILU
   hierarchies are solved by fsimg_solve only: fsimg_solve_batch and the
   server reject them (ERR_ARG); the Vanka options are then ignored. */
typedef enum { FSIMG_SMOOTHER_VANKA = 0, FSIMG_SMOOTHER_ILU = 1 } fsimg_smoother;

/* One multigrid level; level 0 = finest.  Host arrays, copied. */
typedef struct {
  int dim;                  /* 2 or 3 */
  int block;                /* b: d+1 (momentum) or d (ALE / deformation); 1..4 */
  int cells[3];             /* cells per axis (unused axes: 1) */
  int64_t nrows;            /* block rows = prod(2*cells[a]+1) */
  int64_t nnzb;             /* nonzero blocks */
  const int32_t *rowptr;    /* [nrows+1] */
  const int32_t *colind;    /* [nnzb], sorted within each row, diagonal present */
  const double *vals;       /* [nnzb*b*b] row-major blocks */
  const uint8_t *dirichlet; /* [nrows*b], 1 = identity row (row must be e_i) */
  const uint8_t *cell_class; /* [prod(cells)] or NULL: patch class per cell (e.g. 0 fluid,
                                1 solid); GREEDY colouring never mixes classes in a colour */
} fsimg_level_desc;

typedef struct {
  double omega;        /* Vanka damping (Sec. 4.3: omega_V ~ 0.8) */
  double rtol;         /* stop when ||r||_2 <= rtol * ||r_0||_2 (FP64 residual) */
  int nu_pre, nu_post; /* Vanka steps before / after the coarse correction */
  int restart;         /* FGMRES restart length m, 1..32 */
  int max_iter;        /* total FGMRES iterations */
  int precision;       /* fsimg_precision */
  int vanka_schedule;  /* fsimg_vanka_schedule */
  int vanka_weighting; /* fsimg_weighting */
  int profile;         /* 1: time the finest-level smoother kernels and every level's patch
                          factorisation with events */
  int graphs;          /* 1: replay each FGMRES iteration (V-cycle, A z, Gram-Schmidt) as a
                          HIP graph captured once per batch composition; 0: launch eagerly.
                          Results are identical either way; profiling runs launch eagerly */
  int vanka_patches;   /* fsimg_patches */
  int smoother;        /* fsimg_smoother */
  double omega_ilu;    /* ILU damping (default 1: the undamped incomplete-LU step) */
  int krylov_lookahead; /* FGMRES iterations the host keeps in flight (1 or 2, default 2).
                           The Givens update and the stop test run on the device; the host
                           reads each iteration's stop flags only to stop launching.  With 2
                           it reads iteration j's flags while iteration j + 1 runs (no idle
                           GPU between iterations; after the last instance stops at most one
                           iteration runs with nothing to do); with 1 it waits for every
                           iteration before launching the next.  Results are identical */
  int small_level_kib;  /* GATHER / Vanka hierarchies: the levels below the finest whose patch
                           inverses and matrix values (in the V-cycle's precision) each take at
                           most this many KiB, down to the coarsest-but-one, run in one
                           workgroup per instance (one launch for their pre-smoothing,
                           residuals and restrictions, one for prolongations and
                           post-smoothing) instead of a launch per step and level; the same
                           per-row, per-patch and per-dof arithmetic, so results are
                           identical.  0 (default): never.  One workgroup walks a level's
                           rows and patches in rounds whose dependent loads it cannot hide,
                           so on this hardware it pays only for levels of a few hundred
                           unknowns (2D 32^2 with level 1 in it: 1.8x slower per step) */
} fsimg_opts;

#define FSIMG_HIST 64  /* residual-history entries in fsimg_stats */

typedef struct {
  int status;          /* fsimg_status of the solve */
  int iters;           /* FGMRES iterations (= V-cycles) */
  int restarts;        /* completed restart cycles */
  double rel_res;      /* ||b - A x||_2 / ||r_0||_2 recomputed in FP64 */
  double solve_ms;     /* host wall time of the solve */
  /* profile == 1: summed event times (ms) and launch counts of the finest
     level's Vanka patch kernel and residual SpMV kernel */
  double vanka_ms; int vanka_launches;
  double spmv_ms; int spmv_launches;
  /* profile == 1, GATHER schedule: the same for the restriction from and the
     prolongation to the finest level */
  double restrict_ms; int restrict_launches;
  double prolong_ms; int prolong_launches;
  double setup_ms;     /* host wall time of this hierarchy's fsimg_hier_create */
  double factor_ms;    /* host wall time of its last fsimg_factor (stream synchronised) */
  double bytes_moved;  /* algorithmic device-memory bytes of the solve's kernels: every matrix,
                          inverse, index and vector entry each kernel must read or write once
                          (SpMV, Vanka patch and gather, transfers, coarse GEMV, Krylov vector
                          operations), summed over the solve's iterations */
  int nhist;           /* entries of res_hist */
  double res_hist[FSIMG_HIST];  /* |g_{j+1}| / ||r_0||: the FGMRES residual estimate after
                                   iteration j + 1, for the first FSIMG_HIST iterations */
} fsimg_stats;

typedef struct {
  int64_t nrows, n;     /* block rows, scalar unknowns */
  int64_t nnzb;
  int64_t npatch;       /* active patches (at least one non-identity dof) */
  int np;               /* dofs per patch = 3^d * b */
  int ncolours;         /* colours of the selected schedule (1 for GATHER) */
  size_t bytes;         /* device bytes held by this level */
  double factor_ms;     /* profiling on: HIP-event time (ms) of this level's last patch
                           factorisation (every patch group), else 0 */
} fsimg_level_info;

typedef struct fsimg_ctx fsimg_ctx;
typedef struct fsimg_hier fsimg_hier;

/* Default options: omega 0.8, rtol 1e-8, nu 2/2, restart 20, max_iter 200,
   FP64, GATHER, MULT, no profiling. */
void fsimg_default_opts(fsimg_opts *opts);

/* Create a context on HIP device `device`; all allocations of hierarchies
   created in it are charged against hbm_budget_bytes (0 = no limit). */
fsimg_status fsimg_ctx_create(int device, size_t hbm_budget_bytes, fsimg_ctx **out);
void fsimg_ctx_destroy(fsimg_ctx *ctx);
size_t fsimg_ctx_bytes_in_use(const fsimg_ctx *ctx);

/* Device bytes a hierarchy with these levels and options will hold. */
fsimg_status fsimg_hier_footprint(const fsimg_level_desc *levels, int nlev, const fsimg_opts *opts,
                                  size_t *bytes);

/* Upload the level matrices (H1: structure, FP64 values, FP32 copies in
   mixed mode, masks), build patch lists, multiplicities, the chosen colouring
   and the transfer data.  ERR_BUDGET if the footprint exceeds the budget. */
fsimg_status fsimg_hier_create(fsimg_ctx *ctx, const fsimg_level_desc *levels, int nlev,
                               const fsimg_opts *opts, void *stream, fsimg_hier **out);
void fsimg_hier_destroy(fsimg_hier *h);
fsimg_status fsimg_hier_info(const fsimg_hier *h, int level, fsimg_level_info *out);

/* Switch the per-launch HIP-event timing of the finest level's Vanka patch
   kernel and residual SpMV on (1) or off (0) for the following solves (the
   `profile` option of fsimg_opts, changeable after creation).  Timing only. */
fsimg_status fsimg_hier_set_profile(fsimg_hier *h, int on);

/* Replace the values of one level (same structure); on_device != 0 means
   vals is a device pointer.  Invalidates the factorisation. */
fsimg_status fsimg_hier_update_values(fsimg_hier *h, int level, const double *vals, int on_device,
                                      void *stream);

/* Factor: every patch matrix A_i = R_i A R_i^T is inverted exactly (LU with
   partial pivoting in FP64, Sec. 4.3: local matrices inverted exactly) and
   stored (FP64, or FP32 in mixed mode); the coarsest matrix is inverted in
   FP64 (dense Gauss-Jordan with partial pivoting).  ERR_SINGULAR names the
   level and patch in fsimg_last_error(). */
fsimg_status fsimg_factor(fsimg_hier *h, void *stream);

/* Solve A x = b on level 0 by FGMRES(m) + V-cycle.  b_dev, x_dev: FP64
   device vectors of nrows*b; x_dev is the initial guess (and carries the
   identity-row data) on entry and the solution on return.  stats may be
   NULL.  Returns OK, NOCONV (x = last iterate) or NONFINITE. */
fsimg_status fsimg_solve(fsimg_hier *h, const double *b_dev, double *x_dev, fsimg_stats *stats,
                         void *stream);

/* Solve n independent systems A_i x_i = b_i at once (the same method as
   fsimg_solve, in lockstep): every multigrid operation runs as one launch per
   level for all instances, the Krylov iterations advance together and each
   instance stops at its own tolerance.  Each instance's arithmetic depends
   only on that instance, so its result is bitwise the one it gets alone.
   All hierarchies must belong to one context and share precision, block
   size, dimension and solver options; sizes and level counts may differ.
   stats: array of n (may be NULL).  Returns OK if every instance converged,
   else the first failing status (per-instance status in stats).
   fsimg_solve with the GATHER schedule is this call with n = 1.  ERR_ARG for
   hierarchies with the ILU smoother. */
fsimg_status fsimg_solve_batch(int n, fsimg_hier *const *hiers, const double *const *b_dev,
                               double *const *x_dev, fsimg_stats *stats, void *stream);

/* fsimg_solve for callers that cannot allocate: code under HIP graph capture
   of its own work, tight serving loops, harnesses that forbid hipMalloc.
   Same method, kernels and result as fsimg_solve (bitwise equal; launched
   eagerly, no HIP graphs, one FGMRES iteration in flight).  The solve's
   descriptor tables (level descriptors, work lists, Krylov descriptor,
   active flags, Hessenberg column, FGMRES control state; about 25 KB for
   five levels) are written into a fixed 64 KiB
   device array that every GPU the library runs on holds until the process
   ends (its address is looked up when a context is created on the GPU);
   host staging uses host memory.  The call makes no hipMalloc, hipFree,
   hipHostMalloc, stream or graph creation.  It needs a factored hierarchy
   (else ERR_STATE) with the GATHER schedule and the Vanka smoother (else
   ERR_ARG); ERR_ARG if its tables do not fit the array (more than about a
   dozen levels).  Every call on one GPU shares that GPU's array and rewrites
   all of it: calls that overlap on one GPU (other host threads, other
   streams) race, and the caller must serialise them.  Arguments and
   results otherwise as fsimg_solve. */
fsimg_status fsimg_solve_noalloc(fsimg_hier *h, const double *b_dev, double *x_dev,
                                 fsimg_stats *stats, void *stream);

/* Condensed deformation update (Sec. 3.1 and eq. problem:2):
     u_new = u_old + k theta v_new + k (1 - theta) v_old   at nodes with mask != 0,
     u_new = 0                                            elsewhere.
   v_new[node*v_stride + v_offset + c], u_old / v_old / u_new [nnodes*dim]
   (u_old, v_old may be NULL = 0).  All device pointers. */
fsimg_status fsimg_deform_update(int64_t nnodes, int dim, const uint8_t *mask_dev, double k,
                                 double theta, const double *v_new_dev, int v_stride, int v_offset,
                                 const double *u_old_dev, const double *v_old_dev,
                                 double *u_new_dev, void *stream);

/* ---- single steps of the path (the same kernels the solve uses) ----
   `precision` selects the buffers: FSIMG_FP64 -> double vectors and FP64
   matrices / inverses; FSIMG_MIXED -> float vectors and the FP32 copies. */

/* y = A_l x (no masking). */
fsimg_status fsimg_level_apply(fsimg_hier *h, int level, int precision, const void *x_dev,
                               void *y_dev, void *stream);
/* d = b - A_l x, zero at identity rows. */
fsimg_status fsimg_level_residual(fsimg_hier *h, int level, int precision, const void *b_dev,
                                  const void *x_dev, void *d_dev, void *stream);
/* One Vanka step on level l (requires fsimg_factor; ERR_STATE on an ILU
   hierarchy): d = b - A x; x += omega * W * sum_i R_i^T A_i^{-1} R_i d,
   identity dofs kept. */
fsimg_status fsimg_vanka_step(fsimg_hier *h, int level, int precision, const void *b_dev,
                              void *x_dev, void *stream);
/* One ILU step on level l of an ILU hierarchy (requires fsimg_factor; else
   ERR_STATE): d = b - A x; x += omega_ilu (L U)^{-1} d, identity dofs kept. */
fsimg_status fsimg_ilu_step(fsimg_hier *h, int level, int precision, const void *b_dev,
                            void *x_dev, void *stream);
/* The FP64 ILU factors of level l, copied to the host array out
   [nnzb * b * b], in the matrix's block-CSR layout: the blocks left of the
   diagonal hold L (unit diagonal implied), the others U.  ERR_STATE if the
   hierarchy is not an ILU one or not factored. */
fsimg_status fsimg_ilu_factors(fsimg_hier *h, int level, double *out);
/* r_c = R r_f from level l to l+1 (R = P^T), zero at coarse identity rows. */
fsimg_status fsimg_restrict(fsimg_hier *h, int level, int precision, const void *rf_dev,
                            void *rc_dev, void *stream);
/* x_f += P x_c from level l+1 to l, then zero at fine identity rows. */
fsimg_status fsimg_prolong_add(fsimg_hier *h, int level, int precision, const void *xc_dev,
                               void *xf_dev, void *stream);
/* x = A_{L-1}^{-1} r on the coarsest level (FP64), zero at identity rows. */
fsimg_status fsimg_coarse_solve(fsimg_hier *h, const double *r_dev, double *x_dev, void *stream);
/* z = V-cycle(r) on level 0 (the preconditioner), zero at identity rows. */
fsimg_status fsimg_vcycle(fsimg_hier *h, int precision, const void *r_dev, void *z_dev,
                          void *stream);
/* Copy the stored inverse of one active patch of level l to host memory as a
   dense row-major n_p x n_p FP64 matrix; *elem receives the patch's cell. */
fsimg_status fsimg_patch_inverse(fsimg_hier *h, int level, int64_t patch, double *out_host,
                                 int64_t *elem, void *stream);

/* ---- launch-shape tuning (no effect on any result bit) ----
   Two launch shapes of the bandwidth-bound kernels are free parameters
   that leave every result unchanged: the block rows each wavefront of the
   SpMV handles (1, 2 or 4) and the Vanka patches per workgroup (ppw, with
   ppw * n_p <= 1024).  A context keeps a table keyed by (kind, block size b
   for the SpMV or patch size n_p for Vanka, word bytes 4 / 8, size bucket
   floor(log2(rows or patches))); keys without an entry use built-in
   defaults.  Batch compositions cached before a change are dropped. */
typedef enum { FSIMG_TUNE_SPMV_ROWS = 0, FSIMG_TUNE_VANKA_PPW = 1 } fsimg_tune_kind;

/* Measure every candidate shape on the levels of h (its precision, plus the
   FP64 level-0 SpMV of the outer iteration) for keys the table lacks
   (force = 1: for all of them), and keep the fastest.  Uses h's work
   vectors: do not overlap with a solve of h.  Synchronises the stream. */
fsimg_status fsimg_hier_tune(fsimg_hier *h, int force, void *stream);
/* set / read one entry (read gives the value in use: the entry or the
   default).  ERR_ARG for an unknown kind or a value outside its range. */
fsimg_status fsimg_tune_set(fsimg_ctx *ctx, int kind, int key, int word, int64_t size, int value);
fsimg_status fsimg_tune_get(const fsimg_ctx *ctx, int kind, int key, int word, int64_t size,
                            int *value);
/* JSON file of the table: {"arch": "gfx950", "entries": [{"kind": k,
   "key": b_or_np, "word": w, "bucket": e, "value": v}, ...]}.  Loading a
   file written for another GPU architecture fails with ERR_ARG and leaves
   the table unchanged; loaded entries replace entries with the same key. */
fsimg_status fsimg_tune_save(const fsimg_ctx *ctx, const char *path);
fsimg_status fsimg_tune_load(fsimg_ctx *ctx, const char *path);

/* The Vanka schedule (fsimg_vanka_schedule: the patch-correction gather or
   one of the two colourings of the paper's coloured scatter) changes the
   summation order, so it is not a launch shape: it is fixed when a
   hierarchy is created.  This call measures it for the caller: for each of
   GATHER, PARITY and GREEDY it creates the hierarchy of `levels` with
   `opts` and that schedule, factors it, and times `reps` V-cycles (after one
   warm-up) with HIP events on `stream`; ms_out[0..2] receive the mean
   milliseconds per V-cycle in that order (-1 where the schedule does not
   apply, e.g. block patches, which need GATHER), *best the fastest
   schedule.  One hierarchy exists at a time (the context's budget
   applies); the call allocates two vectors of the finest level and frees
   everything before it returns.  Synchronises the stream. */
fsimg_status fsimg_tune_schedule(fsimg_ctx *ctx, const fsimg_level_desc *levels, int nlev,
                                 const fsimg_opts *opts, int reps, double *ms_out, int *best,
                                 void *stream);

/* ---- serving: many simulations sharing one GPU ----
   A request is one FSI simulation: time_steps time steps, newton_steps[t]
   Newton steps in step t; every Newton step is the linear solve of the
   reduced Jacobian (Sec. 4.2): momentum solve, condensed deformation update,
   ALE solve.  Time step t uses momentum state t % n_states (state 0: the
   values of `mom`; state s >= 1: state_vals[(s - 1) * nlev + l] for level
   l, same pattern); a time step with another state than the previous one
   uploads its values and refactors (the paper reassembles about once per
   time step, Sec. 5.5.2).  Newton step i of the request (counted over all
   time steps) solves the momentum system with right-hand side i % n_rhs
   (0: b_mom; j >= 1: rhs_mom[j - 1]).  The ALE matrix is fixed per request
   and factored once.  Requests wait in a queue until their
   hierarchies fit in the context's HBM budget (first fit in arrival order);
   admitted requests keep their hierarchies resident, and every server step
   solves the current Newton step of all admitted requests together (one
   batched solve per system and dimension), so requests join and leave
   between steps.  Each result equals the result of the request alone. */
typedef struct {
  int nlev;                         /* levels of both systems */
  const fsimg_level_desc *mom;      /* momentum levels, finest first */
  const fsimg_level_desc *ale;      /* ALE levels, finest first */
  const double *b_mom, *b_ale;      /* finest-level right-hand sides */
  const uint8_t *node_solid;        /* finest nodes on interface / in the solid */
  int time_steps;
  const int *newton_steps;          /* [time_steps] */
  double k, theta;                  /* time step and theta of the deformation update */
  double arrival;                   /* arrival time on the server clock (s) */
  int n_states;                     /* momentum states cycled over time steps (>= 1) */
  const double *const *state_vals;  /* [(n_states - 1) * nlev] or NULL */
  int n_rhs;                        /* momentum right-hand sides cycled over Newton steps (>= 1) */
  const double *const *rhs_mom;     /* [n_rhs - 1] or NULL */
} fsimg_request;

typedef struct fsimg_server fsimg_server;

/* opts: solver options of every hierarchy the server creates (the Vanka
   smoother: ERR_ARG for ILU); max_active: admitted requests at most (0 = no
   limit).  Host arrays of a submitted
   request are read at admission (the descriptors, right-hand sides, node
   mask) and, with n_states > 1, the momentum values of every state again at
   each change of state: the caller keeps them valid until the request
   completes (fsimg_server_poll reports completions). */
fsimg_status fsimg_server_create(fsimg_ctx *ctx, const fsimg_opts *opts, int max_active,
                                 fsimg_server **out);
void fsimg_server_destroy(fsimg_server *srv);
double fsimg_server_clock(const fsimg_server *srv);  /* seconds since creation */
fsimg_status fsimg_server_submit(fsimg_server *srv, const fsimg_request *req, int64_t *id);
/* Admission order of the queue: 0 (default) first fit in arrival order; 1
   first fit in order of least work (finest-level unknowns of both systems
   times the Newton steps the request asks for; a Newton request counts one
   step per time step), ties in arrival order.  Least work first lowers the
   median latency when requests of very different size compete for the
   budget; a large request may then wait while smaller ones keep arriving. */
fsimg_status fsimg_server_set_order(fsimg_server *srv, int order);
/* Admit what fits, then run one Newton step of every admitted request.
   Reports the number of admitted (running) and queued requests after the
   step.  ERR_BUDGET if the queue head can never fit an empty budget. */
fsimg_status fsimg_server_step(fsimg_server *srv, int *n_active, int *n_queued, void *stream);
/* Completed requests since the last call: ids, admission and finish times
   (server clock), at most max entries. */
fsimg_status fsimg_server_poll(fsimg_server *srv, int64_t *ids, double *admitted, double *finished,
                               int max, int *count);
/* Copy the last momentum and ALE solutions of a request (running or
   completed and not yet released) to host memory (either pointer may be NULL). */
fsimg_status fsimg_server_result(fsimg_server *srv, int64_t id, double *x_mom_host,
                                 double *x_ale_host);
/* Status of a request: FSIMG_OK while queued / running or after success,
   else the error that ended it (e.g. ERR_NOCONV of one of its solves,
   ERR_BUDGET if it can never fit).  ERR_ARG for an unknown id. */
fsimg_status fsimg_server_request_status(fsimg_server *srv, int64_t id, int *status);
/* Forget a completed request's stored solution. */
fsimg_status fsimg_server_release(fsimg_server *srv, int64_t id);

const char *fsimg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FSIMG_H */
