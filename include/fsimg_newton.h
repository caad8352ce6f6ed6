/*
 * fsimg_newton.h -- the approximate Newton loop around the linear solves of
 * fsimg.h: the condensed nonlinear residual of one theta time step of the
 * monolithic ALE fluid-structure model (Sec. 2, eq. aletime:2, with the solid
 * deformation condensed into the velocity, Sec. 3.1 eq. defgrad), its
 * approximate Jacobian (Sec. 4.2: every derivative with respect to the ALE
 * deformation dropped, the momentum block of eq. REDUCEDMATRIX = eq.
 * problem:1), assembled on the GPU on every multigrid level, and the Newton
 * iteration of eq. newton with the Jacobian-reuse rule of Sec. 5.5 and a
 * line search.
 *
 * Discretisation: equal-order Q2 elements on a tensor-product mesh (Sec.
 * 3.2), 3 Gauss points per axis, nodes numbered lexicographically with x
 * fastest, 2*cells[a]+1 nodes per axis; the pressure is stabilised by
 * s_h(p, xi) = sum_K delta_K (grad p, grad xi)_K,
 * delta_K = alpha0 k^2 h_K^2 / (rho_f (h_K^2 + k theta nu_f)), h_K the
 * longest cell side.  Inertia and convection carry rho_f; the pressure
 * enters the momentum rows as -k (J p F^-T, grad phi) and the divergence row
 * as +k (J tr(grad v F^-1), xi); the mesh-transport term uses
 * vbar = theta v_n + (1 - theta) v_{n-1}.
 *
 * Vectors (all FP64 device pointers, node-major):
 *   x      [nrows*(d+1)]  (p, v_1..v_d) per node: the momentum unknowns
 *   u      [nrows*d]      deformation; in fluid cells the ALE deformation,
 *                         in solid cells the residual uses the condensation
 *                         u_old + k theta v + k (1 - theta) v_old instead
 *   x_old, u_old          the same at t_{n-1} (the pressure of x_old is unused)
 * Errors are reported as in fsimg.h (status code, fsimg_last_error()).
 */
#ifndef FSIMG_NEWTON_H
#define FSIMG_NEWTON_H

#include "fsimg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Material and time-stepping parameters of eq. aletime:2. */
typedef struct {
  double rho_f, nu_f;        /* fluid density and kinematic viscosity */
  double rho_s, mu_s, lambda_s; /* solid density and Lame parameters (St. Venant-Kirchhoff) */
  double k, theta;           /* time step and theta of the theta scheme */
  double alpha0;             /* pressure stabilisation scale */
} fsimg_phys;

/* Geometry of one multigrid level (host arrays, copied).  A cell is the
   image of the reference cell under x(xi) = sum_i x_i N_i(xi) over its 3^d
   nodes (isoparametric Q2, Sec. 3.2 with the curved cylinder of Sec. 5);
   node positions come from node_coords, or, when it is NULL, from the
   tensor grid of coords (rectilinear cells).  The pressure stabilisation's
   h_K is the longest cell edge from the cell's first corner. */
typedef struct {
  const double *coords[3];   /* per-axis node coordinates, 2*cells[a]+1 each (unused axes:
                                NULL) */
  const uint8_t *cell_solid; /* [prod(cells)] 1 = solid cell, 0 = fluid cell */
  const double *node_coords; /* [nnodes * dim] node positions, node-major, or NULL */
} fsimg_fsi_level;

typedef struct fsimg_fsi fsimg_fsi;

/* Bind the Newton loop to a momentum hierarchy `mom` (block d+1, its level
   matrices carry the identity rows of the momentum system and the full Q2
   element pattern) and an ALE hierarchy `ale` (block d, the vector Laplacian
   of eq. problem:3 with identity rows at interface, solid and outer-boundary
   nodes; NULL: residual and Jacobian only, no Newton loop).  levels[l]
   describes level l of `mom` (cells taken from it).  Both hierarchies must
   use FP64 or mixed precision and stay alive while the object exists; the
   object allocates its work vectors from mom's context (budget-charged).
   ERR_ARG on inconsistent sizes. */
fsimg_status fsimg_fsi_create(fsimg_hier *mom, fsimg_hier *ale, const fsimg_fsi_level *levels,
                              const fsimg_phys *phys, fsimg_fsi **out);
void fsimg_fsi_destroy(fsimg_fsi *f);

/* res = B - A(U) of the momentum and divergence rows on the finest level
   (B = 0: no volume forces), zero at the identity rows.  ERR_SINGULAR if
   det F <= 0 at a Gauss point.  Synchronises the stream. */
fsimg_status fsimg_fsi_residual(fsimg_fsi *f, const double *x, const double *u, const double *x_old,
                                const double *u_old, double *res, void *stream);

/* Assemble the approximate Jacobian at U into the momentum hierarchy's FP64
   values on every level (the state injected to the coarse levels: coarse
   node g is fine node 2g per axis), with that hierarchy's identity rows
   (row and column eliminated, diagonal one), and its FP32 copies in mixed
   mode.  Invalidates the factorisation (call fsimg_factor).  ERR_SINGULAR as
   above; ERR_ARG if a level's block pattern lacks an element coupling.
   Synchronises the stream. */
fsimg_status fsimg_fsi_jacobian(fsimg_fsi *f, const double *x, const double *u, const double *x_old,
                                const double *u_old, void *stream);

typedef struct {
  double rtol;       /* stop when ||B - A(U)||_inf <= rtol * (its initial value) (default 1e-8) */
  double atol;       /* ... or <= atol (default 0) */
  int max_steps;     /* Newton steps (default 20) */
  double gamma;      /* reassemble the Jacobian when the rate rho_l > gamma (default 0.05) */
  int max_halvings;  /* line search: halve omega while the residual does not decrease, at
                        most this often (default 4) */
  double lin_rtol;   /* relative tolerance of each momentum solve inside the loop (Sec. 5.5
                        reduces the error by 1e-4 per Newton step); 0 (default): the momentum
                        hierarchy's own rtol. */
  double ale_rtol;   /* relative tolerance of each ALE solve inside the loop; 0 (default):
                        the ALE hierarchy's own rtol */
} fsimg_newton_opts;

typedef struct {
  int status;           /* fsimg_status of the loop */
  int steps;            /* Newton steps taken */
  int jacobians;        /* Jacobians assembled (and factored) in this call */
  int halvings;         /* line-search halvings in this call */
  int lin_iters_mom, lin_iters_ale;  /* FGMRES iterations of the momentum / ALE solves */
  double res0, res;     /* initial and final max-norm of B - A(U) (momentum, ALE and
                           condensation rows) */
  double res_hist[32];  /* the max-norm before step l (l < 32) */
  double omega_hist[32];/* the accepted line-search parameter of step l */
  double ms_total, ms_residual, ms_jacobian, ms_factor, ms_solve;  /* host wall times */
} fsimg_newton_stats;

void fsimg_default_newton_opts(fsimg_newton_opts *o);

/* One time step t_{n-1} -> t_n by the approximate Newton method, in place on
   (x, u) (the initial guess on entry; identity-row values of x are kept).
   Each step: the residual R = B - A(U) and the ALE residual b5 = -E u at the
   fluid rows; the Jacobian is assembled and factored if none is held yet or
   the last rate ||R_l|| / ||R_{l-1}|| exceeded gamma (a Jacobian is kept
   across calls, i.e. across time steps); the momentum system J W = R
   (eq. problem:1) is solved by FGMRES + multigrid; the interface and solid
   deformation increment is r_u + k theta W_v (eq. problem:2, one vector
   addition), r_u = u_old + k theta v + k (1 - theta) v_old - u the residual
   of the condensation relation at the nodes of solid cells (nonzero when a
   time step starts from u = u_old); the ALE system E du = b5 with that
   increment at its identity rows (eq. problem:3) is solved likewise; then
   U += omega (W, du) with omega = 1, halved while the max-norm of the
   residual (momentum, ALE and condensation rows) does not decrease.
   Requires an ALE hierarchy.  Returns OK, NOCONV (max_steps reached), a
   linear-solve failure, or ERR_SINGULAR (det F <= 0). */
fsimg_status fsimg_fsi_newton(fsimg_fsi *f, double *x, double *u, const double *x_old,
                              const double *u_old, const fsimg_newton_opts *opts,
                              fsimg_newton_stats *stats, void *stream);

/* Forget the Jacobian held by the object (the next Newton call assembles). */
fsimg_status fsimg_fsi_drop_jacobian(fsimg_fsi *f);

/* One step of a time-stepping run (Sec. 5: the benchmark's start-up from
   rest, with time-dependent inflow): copies the current state (x, u) into the
   old level (x_old, u_old: buffers of their own, sizes as for x and u), sets
   the held rows rows[i] of x to scale * vals[i] (the Dirichlet data of t_n,
   e.g. the inflow profile times the start-up factor), then runs
   fsimg_fsi_newton from the previous state.  rows and vals are device arrays
   of n_rows entries (n_rows may be 0); every row must be a held (identity)
   row of the momentum system, else ERR_ARG; the list is checked before
   anything is written, so a refused call leaves x, u, x_old and u_old as
   they were.
   The Jacobian held by the object carries over from the previous step. */
fsimg_status fsimg_fsi_time_step(fsimg_fsi *f, double *x, double *u, double *x_old, double *u_old,
                                 const int64_t *rows, const double *vals, int64_t n_rows, double scale,
                                 const fsimg_newton_opts *opts, fsimg_newton_stats *stats, void *stream);

/* Drag and lift in the residual form of Sec. 5 (quantities of interest): the
   step operator A(U) of the momentum rows (eq. aletime:2, no identity rows)
   tested with psi e_j, psi the nodal function equal to one at the listed
   nodes (device int64 array of n_nodes node numbers of the finest level,
   e.g. every node of a rigid obstacle) and zero elsewhere, divided by k and
   negated: the mean force on the obstacle over the step (positive drag for a
   flow past it).  force: host array of d doubles (x, y[, z]).  The sum runs
   in a fixed order (same result on every call).  Uses the object's residual
   work vector (not during a Newton call on the same object); synchronises
   the stream.  ERR_ARG for a node out of range, ERR_SINGULAR for an
   inverted element. */
fsimg_status fsimg_fsi_force(fsimg_fsi *f, const double *x, const double *u, const double *x_old,
                             const double *u_old, const int64_t *nodes, int64_t n_nodes, double *force,
                             void *stream);

/* Timing only: on != 0 records HIP events on the launch stream around every
   launch of the finest level's element kernels (one launch per parity colour)
   of the following residual and Jacobian assemblies and resets the sums;
   fsimg_fsi_profile returns the summed milliseconds and launch counts
   (any output pointer may be NULL). */
fsimg_status fsimg_fsi_set_profile(fsimg_fsi *f, int on);
fsimg_status fsimg_fsi_profile(const fsimg_fsi *f, double *jac_ms, int *jac_launches, double *res_ms,
                               int *res_launches);

/* A serving request that runs real Newton time steps (instead of the
   synthetic states and right-hand sides of fsimg_request): the server creates
   its momentum and ALE hierarchies and its Newton object at admission, and
   every server step advances each running Newton request by one Newton step
   of fsimg_fsi_newton, with the momentum and ALE solves of all of them
   batched (fsimg_solve_batch).  A time step ends when its residual meets the
   tolerance; the next starts from the converged state with the Jacobian
   carried over.  Each request's result is bitwise the one fsimg_fsi_newton
   gives it alone, time step after time step.  Host arrays are read at
   admission; the caller keeps them valid until the request completes. */
typedef struct {
  int nlev;                         /* levels of both systems */
  const fsimg_level_desc *mom;      /* momentum levels, finest first */
  const fsimg_level_desc *ale;      /* ALE levels, finest first */
  const fsimg_fsi_level *geom;      /* [nlev] geometry of the momentum levels */
  fsimg_phys phys;
  const double *x, *u;              /* initial state (host, finest level) */
  const double *x_old, *u_old;      /* the state at t_{n-1} of the first time step */
  int time_steps;
  fsimg_newton_opts newton;
  double arrival;                   /* arrival time on the server clock (s) */
} fsimg_newton_request;

fsimg_status fsimg_server_submit_newton(fsimg_server *srv, const fsimg_newton_request *req,
                                        int64_t *id);
/* Newton statistics of a Newton request summed over its finished time steps
   (steps, Jacobians, halvings, linear iterations, times; res0 / res /
   res_hist of the last one).  fsimg_server_result returns its state: x as the
   momentum vector, u as the ALE vector.  ERR_ARG for an unknown id or a
   request of the other kind. */
fsimg_status fsimg_server_newton_stats(fsimg_server *srv, int64_t id, fsimg_newton_stats *out);

#ifdef __cplusplus
}
#endif
#endif
