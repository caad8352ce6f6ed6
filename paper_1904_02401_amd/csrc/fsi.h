// The Newton-loop object and the stages of one Newton step.  fsimg_fsi_newton
// runs the stages with solo linear solves; the serving loop runs the same
// stages for many requests with batched solves in between, so a request's
// result does not depend on what it is served with.
#pragma once
#include <chrono>
#include <vector>

#include "fsimg_newton.h"
#include "hier.h"

namespace fsimg {

struct FsiLevel {
  AsmLevel dev{};          // device view (pattern and mask borrowed from the hierarchy)
  double *coord[3] = {nullptr, nullptr, nullptr};
  double *xyz = nullptr;   // node positions [nrows * d] (isoparametric cells) or null
  uint8_t *solid = nullptr;
  // the state injected to this level (coarse levels only)
  double *x = nullptr, *u = nullptr, *xo = nullptr, *uo = nullptr;
};

// one time step of the Newton loop in progress (the stages below advance it)
struct NewtonRun {
  fsimg_newton_opts o{};
  double *x = nullptr, *u = nullptr;
  const double *xo = nullptr, *uo = nullptr;
  double nrm = 0.0, nrm0 = 0.0, rate = -1.0;  // rate < 0: no step taken yet
  bool done = true;
  fsimg_status status = FSIMG_OK;
  fsimg_newton_stats st{};
  std::chrono::steady_clock::time_point t_start;
};

}  // namespace fsimg

struct fsimg_fsi {
  fsimg_hier *mom = nullptr, *ale = nullptr;
  fsimg_phys phys{};
  int dim = 0;
  std::vector<fsimg::FsiLevel> lev;
  std::vector<std::pair<void *, size_t>> allocs;
  uint8_t *node_solid = nullptr;     // [nrows] fine nodes of a solid cell
  // finest-level work vectors
  double *res = nullptr, *W = nullptr, *xt = nullptr;           // [n_mom]
  double *du = nullptr, *b5 = nullptr, *ut = nullptr;           // [n_ale]
  double *ru = nullptr;  // [nrows*d] residual of the condensation relation (eq. problem:2)
  int *dflag = nullptr;                                          // [2] assembly flags
  unsigned long long *dnorm = nullptr;                           // max-norm slot
  int *hflag = nullptr;                                          // pinned host mirror
  unsigned long long *hnorm = nullptr;
  bool have_jac = false;
  // the force evaluation (allocated on its first call): an all-zero row mask
  // (the residual without identity rows) and the summed force components
  uint8_t *zero_mask = nullptr;
  double *dforce = nullptr;
  fsimg::NewtonRun run;
  // profiling: events around the finest level's element launches (one pair
  // per parity colour) and the accumulated times
  bool profile = false;
  hipEvent_t ev_jac[16] = {}, ev_res[16] = {};
  double jac_ms = 0.0, res_ms = 0.0;
  int jac_launches = 0, res_launches = 0;
};

namespace fsimg {

// Start a time step at (x, u) with t_{n-1} = (xo, uo): factor the ALE matrix
// once, evaluate the residual; run.done if it already meets the tolerance or
// on an error (run.status).
void newton_begin(fsimg_fsi *f, double *x, double *u, const double *xo, const double *uo,
                  const fsimg_newton_opts &o, hipStream_t s);
// Before the momentum solve: stop at max_steps (NOCONV); assemble and factor
// the Jacobian when none is held or the last rate exceeded gamma; W = 0.  The
// momentum solve is then  mom: J W = res  (W the initial guess).
void newton_prepare(fsimg_fsi *f, hipStream_t s);
// After the momentum solve: the deformation increment into du, the initial
// guess and identity-row data of the ALE solve  ale: E du = b5.
void newton_lift(fsimg_fsi *f, hipStream_t s);
// After the ALE solve: line search, update of (x, u), convergence test.
void newton_finish_step(fsimg_fsi *f, hipStream_t s);
// End the time step with an error (e.g. a failed linear solve).
void newton_fail(fsimg_fsi *f, fsimg_status status);
// The time step's statistics (final norm, wall time) once run.done.
fsimg_newton_stats newton_end(fsimg_fsi *f, hipStream_t s);
// the Newton options in effect (defaults when opts is null); ERR_ARG if one
// is out of range (the one check of the solo and the served Newton loops)
fsimg_status check_newton_options(const fsimg_newton_opts *opts, fsimg_newton_opts *o);
// device bytes fsimg_fsi_create allocates for these momentum levels (geom:
// their geometry, for the node positions it uploads; may be null)
size_t fsi_bytes(const fsimg_level_desc *mom, int nlev, bool with_ale, const fsimg_fsi_level *geom);

}  // namespace fsimg
