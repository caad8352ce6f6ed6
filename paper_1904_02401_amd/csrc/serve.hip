// Serving loop: many FSI simulations share one GPU.  Requests queue until
// their hierarchies fit in the HBM budget, stay resident while they run, and
// every server step advances all running requests by one Newton step with
// batched solves (continuous batching: requests join and leave between
// steps).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "fsi.h"

using namespace fsimg;

namespace {

struct Req {
  int64_t id = 0;
  fsimg_request r{};
  std::vector<int> newton;
  int state = 0;  // 0 queued, 1 running, 2 finished
  int status = FSIMG_OK;
  fsimg_hier *hm = nullptr, *ha = nullptr;
  double *b_mom = nullptr, *x_mom = nullptr, *b_ale = nullptr, *x_ale = nullptr;
  uint8_t *mask = nullptr;
  size_t vec_bytes = 0;
  size_t reserve = 0;  // batch plan allowance held while running
  std::vector<const double *> states;  // [(n_states - 1) * nlev] host value arrays
  std::vector<const double *> rhs;     // [n_rhs] host right-hand sides (b_mom first)
  int mstate = 0;                      // momentum state held by hm
  int64_t newton_done = 0;             // Newton steps completed over all time steps
  int t = 0, nstep = 0, dim = 0, bm = 0, ba = 0;
  int64_t nnodes = 0, nm = 0, na = 0;
  double admitted = -1.0, finished = -1.0;
  double work = 0.0;  // unknowns x Newton steps asked for (the least-work-first key)
  std::vector<double> xm_host, xa_host;
  // Newton requests: x_mom holds the state x, x_ale the state u
  bool nt = false;
  fsimg_newton_request nreq{};
  fsimg_fsi *fsi = nullptr;
  double *xo = nullptr, *uo = nullptr;
  fsimg_newton_stats acc{};
};

}  // namespace

struct fsimg_server {
  fsimg_ctx *ctx = nullptr;
  fsimg_opts opts{};
  int max_active = 0;
  std::chrono::steady_clock::time_point t0;
  int64_t next_id = 1;
  size_t reserved = 0;  // plan allowance of the running requests
  std::deque<Req *> queue;
  int order = 0;  // fsimg_server_set_order
  std::vector<Req *> running;
  std::vector<Req *> finished_unpolled;
  std::map<int64_t, Req *> all;
};

namespace {

double now_s(const fsimg_server *s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

void release_device(fsimg_server *S, Req *q) {
  if (q->fsi) fsimg_fsi_destroy(q->fsi);
  q->fsi = nullptr;
  for (void *p : {(void *)q->xo, (void *)q->uo})
    if (p) (void)hipFree(p);
  q->xo = q->uo = nullptr;
  if (q->hm) fsimg_hier_destroy(q->hm);
  if (q->ha) fsimg_hier_destroy(q->ha);
  q->hm = q->ha = nullptr;
  for (void *p : {(void *)q->b_mom, (void *)q->x_mom, (void *)q->b_ale, (void *)q->x_ale,
                  (void *)q->mask})
    if (p) (void)hipFree(p);
  q->b_mom = q->x_mom = q->b_ale = q->x_ale = nullptr;
  q->mask = nullptr;
  S->ctx->in_use -= q->vec_bytes;
  q->vec_bytes = 0;
  S->reserved -= q->reserve;
  q->reserve = 0;
}

// batch descriptor tables: every cached plan may hold an instance of each
// running request, at the depth of the deepest hierarchy the library accepts.
// Admission keeps (hierarchies + vectors + these allowances) within the
// budget, so plan tables, which are charged to the budget when built, fit.
size_t plan_reserve() { return kPlanCache * plan_bytes_bound(16); }

// bytes held against the budget apart from the plan tables
size_t held(const fsimg_server *S) { return S->ctx->in_use - S->ctx->plan_bytes + S->reserved; }

size_t request_bytes(const fsimg_server *S, const Req *q, fsimg_status *st) {
  size_t fm = 0, fa = 0;
  *st = fsimg_hier_footprint(q->r.mom, q->r.nlev, &S->opts, &fm);
  if (*st == FSIMG_OK) *st = fsimg_hier_footprint(q->r.ale, q->r.nlev, &S->opts, &fa);
  if (q->nt)
    return fm + fa + fsi_bytes(q->r.mom, q->r.nlev, true, q->nreq.geom) + (size_t)(2 * q->nm + 2 * q->na) * 8 +
           plan_reserve();
  return fm + fa + (size_t)((q->rhs.size() + 1) * q->nm + 2 * q->na) * 8 + (size_t)q->nnodes +
         plan_reserve();
}

// a Newton request: hierarchies, Newton object, state vectors, first residual
fsimg_status admit_newton(fsimg_server *S, Req *q, hipStream_t s) {
  const fsimg_newton_request &N = q->nreq;
  fsimg_status st = fsimg_hier_create(S->ctx, N.mom, N.nlev, &S->opts, s, &q->hm);
  if (st == FSIMG_OK) st = fsimg_hier_create(S->ctx, N.ale, N.nlev, &S->opts, s, &q->ha);
  if (st == FSIMG_OK) st = fsimg_fsi_create(q->hm, q->ha, N.geom, &N.phys, &q->fsi);
  if (st != FSIMG_OK) {
    release_device(S, q);
    return st;
  }
  const size_t bytes = (size_t)(2 * q->nm + 2 * q->na) * 8;
  if (S->ctx->budget && S->ctx->in_use + bytes > S->ctx->budget) {
    release_device(S, q);
    return set_error(FSIMG_ERR_BUDGET, "request vectors exceed the budget");
  }
  bool ok = hipMalloc(&q->x_mom, q->nm * 8) == hipSuccess && hipMalloc(&q->xo, q->nm * 8) == hipSuccess &&
            hipMalloc(&q->x_ale, q->na * 8) == hipSuccess && hipMalloc(&q->uo, q->na * 8) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    release_device(S, q);
    return set_error(FSIMG_ERR_OOM, "request vector allocation failed");
  }
  q->vec_bytes = bytes;
  S->ctx->in_use += bytes;
  q->reserve = plan_reserve();
  S->reserved += q->reserve;
  ok = hipMemcpyAsync(q->x_mom, N.x, q->nm * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
       hipMemcpyAsync(q->xo, N.x_old, q->nm * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
       hipMemcpyAsync(q->x_ale, N.u, q->na * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
       hipMemcpyAsync(q->uo, N.u_old, q->na * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
       hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    release_device(S, q);
    return set_error(FSIMG_ERR_HIP, "request upload failed");
  }
  std::memset(&q->acc, 0, sizeof q->acc);
  newton_begin(q->fsi, q->x_mom, q->x_ale, q->xo, q->uo, N.newton, s);
  q->state = 1;
  q->admitted = now_s(S);
  return FSIMG_OK;
}

// create hierarchies, factor, upload vectors; false if it does not fit now
fsimg_status admit(fsimg_server *S, Req *q, hipStream_t s) {
  if (q->nt) return admit_newton(S, q, s);
  fsimg_status st = fsimg_hier_create(S->ctx, q->r.mom, q->r.nlev, &S->opts, s, &q->hm);
  if (st == FSIMG_OK) st = fsimg_hier_create(S->ctx, q->r.ale, q->r.nlev, &S->opts, s, &q->ha);
  if (st == FSIMG_OK) st = fsimg_factor(q->hm, s);
  if (st == FSIMG_OK) st = fsimg_factor(q->ha, s);
  if (st != FSIMG_OK) {
    release_device(S, q);
    return st;
  }
  const size_t nr = q->rhs.size();
  const size_t bytes = (size_t)((nr + 1) * q->nm + 2 * q->na) * 8 + (size_t)q->nnodes;
  if (S->ctx->budget && S->ctx->in_use + bytes > S->ctx->budget) {
    release_device(S, q);
    return set_error(FSIMG_ERR_BUDGET, "request vectors exceed the budget");
  }
  bool ok = hipMalloc(&q->b_mom, nr * q->nm * 8) == hipSuccess &&
            hipMalloc(&q->x_mom, q->nm * 8) == hipSuccess &&
            hipMalloc(&q->b_ale, q->na * 8) == hipSuccess &&
            hipMalloc(&q->x_ale, q->na * 8) == hipSuccess &&
            hipMalloc(&q->mask, q->nnodes) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    release_device(S, q);
    return set_error(FSIMG_ERR_OOM, "request vector allocation failed");
  }
  q->vec_bytes = bytes;
  S->ctx->in_use += bytes;
  q->reserve = plan_reserve();
  S->reserved += q->reserve;
  for (size_t j = 0; j < nr && ok; ++j)
    ok = hipMemcpyAsync(q->b_mom + j * q->nm, q->rhs[j], q->nm * 8, hipMemcpyHostToDevice, s) ==
         hipSuccess;
  ok = ok &&
       hipMemcpyAsync(q->b_ale, q->r.b_ale, q->na * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
       hipMemcpyAsync(q->mask, q->r.node_solid, q->nnodes, hipMemcpyHostToDevice, s) == hipSuccess &&
       hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    release_device(S, q);
    return set_error(FSIMG_ERR_HIP, "request upload failed");
  }
  q->state = 1;
  q->admitted = now_s(S);
  return FSIMG_OK;
}

void finish(fsimg_server *S, Req *q, hipStream_t s) {
  q->xm_host.resize(q->nm);
  q->xa_host.resize(q->na);
  (void)hipMemcpyAsync(q->xm_host.data(), q->x_mom, q->nm * 8, hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(q->xa_host.data(), q->x_ale, q->na * 8, hipMemcpyDeviceToHost, s);
  (void)hipStreamSynchronize(s);
  q->finished = now_s(S);
  q->state = 2;
  release_device(S, q);
  S->finished_unpolled.push_back(q);
}

// a Newton request whose time step has ended: add its statistics, then
// finish it (error or last time step) or start the next time step from the
// converged state; repeated while a new time step meets the tolerance at once
void advance_newton(fsimg_server *S, Req *q, hipStream_t s) {
  while (q->state == 1 && q->fsi->run.done) {
    const fsimg_newton_stats st = newton_end(q->fsi, s);
    fsimg_newton_stats &a = q->acc;
    a.steps += st.steps;
    a.jacobians += st.jacobians;
    a.halvings += st.halvings;
    a.lin_iters_mom += st.lin_iters_mom;
    a.lin_iters_ale += st.lin_iters_ale;
    a.ms_total += st.ms_total;
    a.ms_residual += st.ms_residual;
    a.ms_jacobian += st.ms_jacobian;
    a.ms_factor += st.ms_factor;
    a.ms_solve += st.ms_solve;
    a.res0 = st.res0;
    a.res = st.res;
    std::memcpy(a.res_hist, st.res_hist, sizeof a.res_hist);
    std::memcpy(a.omega_hist, st.omega_hist, sizeof a.omega_hist);
    a.status = st.status;
    if (st.status != FSIMG_OK) {
      q->status = st.status;
      finish(S, q, s);
      return;
    }
    if (++q->t == q->nreq.time_steps) {
      finish(S, q, s);
      return;
    }
    // t_{n-1} <- the converged state, which is also the next initial guess
    if (hipMemcpyAsync(q->xo, q->x_mom, q->nm * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(q->uo, q->x_ale, q->na * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) {
      q->status = set_error(FSIMG_ERR_HIP, "state copy failed");
      finish(S, q, s);
      return;
    }
    newton_begin(q->fsi, q->x_mom, q->x_ale, q->xo, q->uo, q->nreq.newton, s);
  }
}

// one Newton step of every running Newton request of one dimension, the
// linear solves batched
fsimg_status newton_group_step(fsimg_server *S, int dim, hipStream_t s) {
  std::vector<Req *> group;
  for (Req *q : S->running)
    if (q->nt && q->dim == dim && q->state == 1) {
      advance_newton(S, q, s);
      if (q->state != 1) continue;
      newton_prepare(q->fsi, s);
      if (q->fsi->run.done) {
        advance_newton(S, q, s);
        continue;
      }
      group.push_back(q);
    }
  if (group.empty()) return FSIMG_OK;
  const auto t0 = std::chrono::steady_clock::now();
  // one batched solve per distinct tolerance (a batch shares its solver options):
  // the request's Newton option when set, else the hierarchy's own rtol; done(q, st)
  // takes each request's result
  auto solve_grouped = [&](const std::vector<Req *> &reqs, bool ale, auto &&done) -> fsimg_status {
    auto hier = [ale](Req *q) { return ale ? q->ha : q->hm; };
    auto tol_of = [&](Req *q) {
      const double t = ale ? q->nreq.newton.ale_rtol : q->nreq.newton.lin_rtol;
      return t > 0.0 ? t : hier(q)->opts.rtol;
    };
    std::vector<Req *> pending = reqs;
    while (!pending.empty()) {
      const double tol = tol_of(pending[0]);
      std::vector<Req *> part, rest;
      for (Req *q : pending) (tol_of(q) == tol ? part : rest).push_back(q);
      std::vector<fsimg_hier *> hs;
      std::vector<const double *> bs;
      std::vector<double *> xs;
      std::vector<double> keep;
      for (Req *q : part) {
        keep.push_back(hier(q)->opts.rtol);
        hier(q)->opts.rtol = tol;
        hs.push_back(hier(q));
        bs.push_back(ale ? q->fsi->b5 : q->fsi->res);
        xs.push_back(ale ? q->fsi->du : q->fsi->W);
      }
      std::vector<fsimg_stats> st(part.size(), fsimg_stats{});
      const fsimg_status r = solve_batch(S->ctx, (int)part.size(), hs.data(), bs.data(), xs.data(), st.data(), s);
      for (size_t g = 0; g < part.size(); ++g) hier(part[g])->opts.rtol = keep[g];
      if (r != FSIMG_OK && r != FSIMG_ERR_NOCONV && r != FSIMG_ERR_NONFINITE) return r;
      for (size_t g = 0; g < part.size(); ++g) done(part[g], st[g]);
      pending.swap(rest);
    }
    return FSIMG_OK;
  };
  std::vector<Req *> alive;
  fsimg_status r1 = solve_grouped(group, false, [&](Req *q, const fsimg_stats &st) {
    q->fsi->run.st.lin_iters_mom += st.iters;
    if (st.status != FSIMG_OK) {
      newton_fail(q->fsi, (fsimg_status)st.status);
      return;
    }
    newton_lift(q->fsi, s);
    alive.push_back(q);
  });
  if (r1 != FSIMG_OK) return r1;
  fsimg_status r2 = solve_grouped(alive, true, [&](Req *q, const fsimg_stats &st) {
    q->fsi->run.st.lin_iters_ale += st.iters;
    if (st.status != FSIMG_OK) newton_fail(q->fsi, (fsimg_status)st.status);
  });
  if (r2 != FSIMG_OK) return r2;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (Req *q : group) {
    q->fsi->run.st.ms_solve += ms;
    newton_finish_step(q->fsi, s);
    advance_newton(S, q, s);
  }
  return FSIMG_OK;
}

}  // namespace

extern "C" {

fsimg_status fsimg_server_create(fsimg_ctx *ctx, const fsimg_opts *opts, int max_active,
                                 fsimg_server **out) {
  if (!ctx || !opts || !out || max_active < 0) return set_error(FSIMG_ERR_ARG, "bad server arguments");
  if (opts->smoother != FSIMG_SMOOTHER_VANKA)
    return set_error(FSIMG_ERR_ARG, "the server batches Vanka hierarchies only");
  auto *S = new fsimg_server;
  S->ctx = ctx;
  S->opts = *opts;
  S->max_active = max_active;
  S->t0 = std::chrono::steady_clock::now();
  *out = S;
  return FSIMG_OK;
}

void fsimg_server_destroy(fsimg_server *S) {
  if (!S) return;
  for (auto &kv : S->all) {
    release_device(S, kv.second);
    delete kv.second;
  }
  delete S;
}

double fsimg_server_clock(const fsimg_server *S) { return S ? now_s(S) : 0.0; }

fsimg_status fsimg_server_submit(fsimg_server *S, const fsimg_request *r, int64_t *id) {
  if (!S || !r || !r->mom || !r->ale || !r->b_mom || !r->b_ale || !r->node_solid ||
      !r->newton_steps || r->time_steps < 1 || r->nlev < 1)
    return set_error(FSIMG_ERR_ARG, "incomplete request");
  const fsimg_level_desc &m0 = r->mom[0], &a0 = r->ale[0];
  if (m0.dim != a0.dim || m0.block != m0.dim + 1 || a0.block != a0.dim || m0.nrows != a0.nrows)
    return set_error(FSIMG_ERR_ARG, "request systems must be momentum (b = d+1) and ALE (b = d) "
                                    "on the same mesh");
  auto *q = new Req;
  q->id = S->next_id++;
  q->r = *r;
  q->newton.assign(r->newton_steps, r->newton_steps + r->time_steps);
  for (int v : q->newton)
    if (v < 1) {
      delete q;
      return set_error(FSIMG_ERR_ARG, "every time step needs at least one Newton step");
    }
  q->r.newton_steps = q->newton.data();
  if (r->n_states < 1 || r->n_rhs < 1 || (r->n_states > 1 && !r->state_vals) ||
      (r->n_rhs > 1 && !r->rhs_mom)) {
    delete q;
    return set_error(FSIMG_ERR_ARG, "n_states and n_rhs must be >= 1, with their arrays");
  }
  if (r->n_states > 1)
    q->states.assign(r->state_vals, r->state_vals + (size_t)(r->n_states - 1) * r->nlev);
  q->rhs.push_back(r->b_mom);
  for (int j = 1; j < r->n_rhs; ++j) q->rhs.push_back(r->rhs_mom[j - 1]);
  for (const double *p : q->states)
    if (!p) {
      delete q;
      return set_error(FSIMG_ERR_ARG, "null state values");
    }
  for (const double *p : q->rhs)
    if (!p) {
      delete q;
      return set_error(FSIMG_ERR_ARG, "null right-hand side");
    }
  q->dim = m0.dim;
  q->bm = m0.block;
  q->ba = a0.block;
  q->nnodes = m0.nrows;
  q->nm = m0.nrows * m0.block;
  q->na = a0.nrows * a0.block;
  int64_t nsteps = 0;
  for (int t = 0; t < r->time_steps; ++t) nsteps += r->newton_steps[t];
  q->work = (double)(q->nm + q->na) * (double)std::max<int64_t>(nsteps, 1);
  S->queue.push_back(q);
  S->all[q->id] = q;
  if (id) *id = q->id;
  return FSIMG_OK;
}

fsimg_status fsimg_server_submit_newton(fsimg_server *S, const fsimg_newton_request *r, int64_t *id) {
  if (!S || !r || !r->mom || !r->ale || !r->geom || !r->x || !r->u || !r->x_old || !r->u_old ||
      r->time_steps < 1 || r->nlev < 1)
    return set_error(FSIMG_ERR_ARG, "incomplete Newton request");
  const fsimg_level_desc &m0 = r->mom[0], &a0 = r->ale[0];
  if (m0.dim < 2 || m0.dim != a0.dim || m0.block != m0.dim + 1 || a0.block != a0.dim ||
      m0.nrows != a0.nrows)
    return set_error(FSIMG_ERR_ARG, "request systems must be momentum (b = d+1) and ALE (b = d) "
                                    "on the same mesh");
  fsimg_newton_opts o;
  {
    const fsimg_status st = check_newton_options(&r->newton, &o);
    if (st != FSIMG_OK) return st;
  }
  auto *q = new Req;
  q->id = S->next_id++;
  q->nt = true;
  q->nreq = *r;
  q->nreq.newton = o;
  q->r.nlev = r->nlev;
  q->r.mom = r->mom;
  q->r.ale = r->ale;
  q->r.arrival = r->arrival;
  q->r.time_steps = r->time_steps;
  q->dim = m0.dim;
  q->bm = m0.block;
  q->ba = a0.block;
  q->nnodes = m0.nrows;
  q->nm = m0.nrows * m0.block;
  q->na = a0.nrows * a0.block;
  q->work = (double)(q->nm + q->na) * r->time_steps;  // Newton steps not known in advance
  S->queue.push_back(q);
  S->all[q->id] = q;
  if (id) *id = q->id;
  return FSIMG_OK;
}

fsimg_status fsimg_server_set_order(fsimg_server *S, int order) {
  if (!S || order < 0 || order > 1) return set_error(FSIMG_ERR_ARG, "order must be 0 or 1");
  S->order = order;
  return FSIMG_OK;
}

fsimg_status fsimg_server_newton_stats(fsimg_server *S, int64_t id, fsimg_newton_stats *out) {
  if (!S || !out) return set_error(FSIMG_ERR_ARG, "null argument");
  auto it = S->all.find(id);
  if (it == S->all.end() || !it->second->nt) return set_error(FSIMG_ERR_ARG, "no Newton request with this id");
  *out = it->second->acc;
  return FSIMG_OK;
}

fsimg_status fsimg_server_step(fsimg_server *S, int *n_active, int *n_queued, void *stream) {
  if (!S) return set_error(FSIMG_ERR_ARG, "null server");
  hipStream_t s = static_cast<hipStream_t>(stream);
  fsimg_status ret = FSIMG_OK;
  // admission: first fit in arrival order, or in order of least work (ties
  // in arrival order)
  if (S->order == 1)
    std::stable_sort(S->queue.begin(), S->queue.end(), [](const Req *a, const Req *b) { return a->work < b->work; });
  for (auto it = S->queue.begin(); it != S->queue.end();) {
    Req *q = *it;
    if (S->max_active && (int)S->running.size() >= S->max_active) break;
    fsimg_status st;
    const size_t need = request_bytes(S, q, &st);
    if (st != FSIMG_OK) {  // invalid descriptors: the request fails
      q->status = st;
      q->state = 2;
      S->finished_unpolled.push_back(q);
      it = S->queue.erase(it);
      continue;
    }
    if (S->ctx->budget && need > S->ctx->budget) {  // can never fit
      q->status = FSIMG_ERR_BUDGET;
      q->state = 2;
      S->finished_unpolled.push_back(q);
      it = S->queue.erase(it);
      ret = set_error(FSIMG_ERR_BUDGET, "a request needs more than the whole HBM budget");
      continue;
    }
    if (S->ctx->budget && held(S) + need > S->ctx->budget) {
      ++it;
      continue;
    }
    st = admit(S, q, s);
    if (st == FSIMG_OK) {
      S->running.push_back(q);
      it = S->queue.erase(it);
    } else if (st == FSIMG_ERR_BUDGET || st == FSIMG_ERR_OOM) {
      ++it;
    } else {
      q->status = st;
      q->state = 2;
      S->finished_unpolled.push_back(q);
      it = S->queue.erase(it);
    }
  }
  if (!S->running.empty()) {
    // Newton requests: one Newton step each, linear solves batched per dimension
    for (int dim = 2; dim <= 3; ++dim) {
      const fsimg_status r = newton_group_step(S, dim, s);
      if (r != FSIMG_OK) return r;
    }
    {  // those that finished leave the running list
      std::vector<Req *> still;
      for (Req *q : S->running)
        if (q->state == 1) still.push_back(q);
      S->running.swap(still);
    }
    // one Newton step of every running synthetic request: batched per system
    // and dimension
    for (int dim = 2; dim <= 3; ++dim) {
      std::vector<fsimg_hier *> hs;
      std::vector<const double *> bs;
      std::vector<double *> xs;
      std::vector<Req *> group;
      for (Req *q : S->running)
        if (q->dim == dim && !q->nt) group.push_back(q);
      if (group.empty()) continue;
      for (Req *q : group) {
        launch_fill<double>(q->x_mom, q->nm, 0.0, s);
        hs.push_back(q->hm);
        bs.push_back(q->b_mom + (size_t)(q->newton_done % (int64_t)q->rhs.size()) * q->nm);
        xs.push_back(q->x_mom);
      }
      std::vector<fsimg_stats> st(group.size());
      fsimg_status r1 = solve_batch(S->ctx, (int)group.size(), hs.data(), bs.data(), xs.data(),
                                    st.data(), s);
      if (r1 != FSIMG_OK && r1 != FSIMG_ERR_NOCONV && r1 != FSIMG_ERR_NONFINITE) return r1;
      for (size_t g = 0; g < group.size(); ++g) {
        Req *q = group[g];
        if (st[g].status != FSIMG_OK && q->status == FSIMG_OK) q->status = st[g].status;
        launch_deform(q->nnodes, dim, q->mask, q->r.k, q->r.theta, q->x_mom, dim + 1, 1, nullptr,
                      nullptr, q->x_ale, s);
        hs[g] = q->ha;
        bs[g] = q->b_ale;
        xs[g] = q->x_ale;
      }
      fsimg_status r2 = solve_batch(S->ctx, (int)group.size(), hs.data(), bs.data(), xs.data(),
                                    st.data(), s);
      if (r2 != FSIMG_OK && r2 != FSIMG_ERR_NOCONV && r2 != FSIMG_ERR_NONFINITE) return r2;
      for (size_t g = 0; g < group.size(); ++g)
        if (st[g].status != FSIMG_OK && group[g]->status == FSIMG_OK) group[g]->status = st[g].status;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return set_error(FSIMG_ERR_HIP, "server step sync failed");
    std::vector<Req *> still;
    for (Req *q : S->running) {
      if (q->nt) {
        still.push_back(q);
        continue;
      }
      ++q->newton_done;
      if (++q->nstep == q->newton[q->t]) {
        q->nstep = 0;
        if (++q->t == q->r.time_steps) {
          finish(S, q, s);
          continue;
        }
        // a new time step: its Jacobian (another state: upload its values), refactored
        fsimg_status st = FSIMG_OK;
        const int want = q->t % q->r.n_states;
        if (want != q->mstate) {
          for (int l = 0; l < q->r.nlev && st == FSIMG_OK; ++l) {
            const double *v = want == 0 ? q->r.mom[l].vals
                                        : q->states[(size_t)(want - 1) * q->r.nlev + l];
            st = fsimg_hier_update_values(q->hm, l, v, 0, s);
          }
          q->mstate = want;
        }
        if (st == FSIMG_OK) st = fsimg_factor(q->hm, s);
        if (st != FSIMG_OK) {
          q->status = st;
          finish(S, q, s);
          continue;
        }
      }
      still.push_back(q);
    }
    S->running.swap(still);
  }
  if (n_active) *n_active = (int)S->running.size();
  if (n_queued) *n_queued = (int)S->queue.size();
  return ret;
}

fsimg_status fsimg_server_poll(fsimg_server *S, int64_t *ids, double *admitted, double *finished,
                               int max, int *count) {
  if (!S || !count || max < 0) return set_error(FSIMG_ERR_ARG, "bad poll arguments");
  int c = 0;
  while (c < max && !S->finished_unpolled.empty()) {
    Req *q = S->finished_unpolled.front();
    S->finished_unpolled.erase(S->finished_unpolled.begin());
    if (ids) ids[c] = q->status == FSIMG_OK ? q->id : -q->id;
    if (admitted) admitted[c] = q->admitted;
    if (finished) finished[c] = q->finished;
    ++c;
  }
  *count = c;
  return FSIMG_OK;
}

fsimg_status fsimg_server_result(fsimg_server *S, int64_t id, double *xm, double *xa) {
  if (!S) return set_error(FSIMG_ERR_ARG, "null server");
  auto it = S->all.find(id);
  if (it == S->all.end()) return set_error(FSIMG_ERR_ARG, "unknown request id");
  Req *q = it->second;
  if (q->state == 2) {
    if (xm && !q->xm_host.empty()) std::copy(q->xm_host.begin(), q->xm_host.end(), xm);
    if (xa && !q->xa_host.empty()) std::copy(q->xa_host.begin(), q->xa_host.end(), xa);
    return FSIMG_OK;
  }
  if (q->state == 1) {
    if (xm && hipMemcpy(xm, q->x_mom, q->nm * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return set_error(FSIMG_ERR_HIP, "result copy failed");
    if (xa && hipMemcpy(xa, q->x_ale, q->na * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return set_error(FSIMG_ERR_HIP, "result copy failed");
    return FSIMG_OK;
  }
  return set_error(FSIMG_ERR_STATE, "request not started");
}

fsimg_status fsimg_server_request_status(fsimg_server *S, int64_t id, int *status) {
  if (!S || !status) return set_error(FSIMG_ERR_ARG, "null server or status");
  auto it = S->all.find(id);
  if (it == S->all.end()) return set_error(FSIMG_ERR_ARG, "unknown request id");
  *status = it->second->status;
  return FSIMG_OK;
}

fsimg_status fsimg_server_release(fsimg_server *S, int64_t id) {
  if (!S) return set_error(FSIMG_ERR_ARG, "null server");
  auto it = S->all.find(id);
  if (it == S->all.end()) return set_error(FSIMG_ERR_ARG, "unknown request id");
  if (it->second->state != 2) return set_error(FSIMG_ERR_STATE, "request still queued or running");
  for (auto &f : S->finished_unpolled)
    if (f == it->second) return set_error(FSIMG_ERR_STATE, "poll the request before releasing it");
  delete it->second;
  S->all.erase(it);
  return FSIMG_OK;
}

}  // extern "C"
