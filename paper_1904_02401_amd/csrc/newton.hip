// The approximate Newton loop of one theta time step (eq. newton) around the
// linear solves of the library: residual and Jacobian assembly on the GPU
// (kernels_asm.hip) on every level of the momentum hierarchy, Jacobian reuse
// by the rate rule of Sec. 5.5, the reduced splitting of eq. REDUCEDMATRIX
// into the momentum solve (eq. problem:1), the deformation update (eq.
// problem:2) and the ALE solve (eq. problem:3), and a halving line search.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fsi.h"

using namespace fsimg;

namespace {

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

fsimg_status nfail(fsimg_status s, const std::string &m) { return set_error(s, m); }

#define NW_HIP(expr)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return nfail(FSIMG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));           \
  } while (0)
#define NW_TRY(expr)                 \
  do {                               \
    fsimg_status st_ = (expr);       \
    if (st_ != FSIMG_OK) return st_; \
  } while (0)

template <typename T>
fsimg_status falloc(fsimg_fsi *f, T **p, size_t count) {
  *p = nullptr;
  const size_t bytes = count * sizeof(T);
  if (bytes == 0) return FSIMG_OK;
  fsimg_ctx *ctx = f->mom->ctx;
  if (ctx->budget && ctx->in_use + bytes > ctx->budget)
    return nfail(FSIMG_ERR_BUDGET, "Newton work vectors exceed the context's HBM budget");
  void *q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nfail(FSIMG_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  ctx->in_use += bytes;
  f->allocs.push_back({q, bytes});
  *p = static_cast<T *>(q);
  return FSIMG_OK;
}

AsmPhys asm_phys(const fsimg_phys &p) {
  return AsmPhys{p.rho_f, p.nu_f, p.rho_s, p.mu_s, p.lambda_s, p.k, p.theta, p.alpha0};
}

// copy the assembly flags and the max-norm slot to the host and wait
fsimg_status read_flags(fsimg_fsi *f, hipStream_t s, int *flags, double *norm) {
  NW_HIP(hipMemcpyAsync(f->hflag, f->dflag, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  NW_HIP(hipMemcpyAsync(f->hnorm, f->dnorm, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  NW_HIP(hipStreamSynchronize(s));
  flags[0] = f->hflag[0];
  flags[1] = f->hflag[1];
  if (norm) {
    double v;
    std::memcpy(&v, f->hnorm, sizeof v);
    *norm = v;
  }
  return FSIMG_OK;
}

fsimg_status clear_flags(fsimg_fsi *f, hipStream_t s) {
  NW_HIP(hipMemsetAsync(f->dflag, 0, 2 * sizeof(int), s));
  NW_HIP(hipMemsetAsync(f->dnorm, 0, sizeof(unsigned long long), s));
  return FSIMG_OK;
}

// after a synchronisation: add the colour launches' event times
void add_event_times(const hipEvent_t *ev, int ncolour, double *ms, int *count) {
  for (int c = 0; c < ncolour; ++c) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ev[2 * c], ev[2 * c + 1]) == hipSuccess) {
      *ms += t;
      ++*count;
    }
  }
}

// the options in effect (defaults when opts is null), refused if out of range
fsimg_status newton_options(const fsimg_newton_opts *opts, fsimg_newton_opts *o) {
  fsimg_default_newton_opts(o);
  if (opts) *o = *opts;
  if (o->max_steps < 0 || o->max_halvings < 0 || !(o->rtol >= 0.0) || !(o->atol >= 0.0) ||
      !(o->gamma >= 0.0) || !(o->lin_rtol >= 0.0 && o->lin_rtol < 1.0) ||
      !(o->ale_rtol >= 0.0 && o->ale_rtol < 1.0))
    return nfail(FSIMG_ERR_ARG, "bad Newton options");
  return FSIMG_OK;
}

fsimg_status flags_status(const int *flags) {
  if (flags[1]) return nfail(FSIMG_ERR_ARG, "the momentum block pattern lacks an element coupling");
  if (flags[0]) return nfail(FSIMG_ERR_SINGULAR, "det F <= 0 at a Gauss point (inverted element)");
  return FSIMG_OK;
}

// residual R = -A(U) on the finest level into f->res; with the ALE system
// also its residual b5 = -E u at the fluid rows and the residual of the
// condensation relation on interface and solid nodes (f->ru); *norm = the
// max-norm over all of them
fsimg_status eval_residual(fsimg_fsi *f, const double *x, const double *u, const double *xo,
                           const double *uo, hipStream_t s, double *norm, bool with_ale) {
  const DevLevel &L = f->mom->lev[0];
  NW_TRY(clear_flags(f, s));
  launch_asm_residual(f->lev[0].dev, f->dim, asm_phys(f->phys), AsmState{x, u, xo, uo}, f->res,
                      L.nrows, f->dflag, s, f->profile ? f->ev_res : nullptr);
  launch_absmax_u64(f->res, L.n, f->dnorm, s);
  if (with_ale) {
    DevLevel &A = f->ale->lev[0];
    NW_TRY(fsimg_level_apply(f->ale, 0, FSIMG_FP64, u, f->b5, s));
    launch_neg_free(f->b5, A.mask, A.n, s);
    launch_absmax_u64(f->b5, A.n, f->dnorm, s);
    launch_cond_residual(L.nrows, f->dim, f->node_solid, f->phys.k, f->phys.theta, x, xo, u, uo, f->ru, s);
    launch_absmax_u64(f->ru, A.n, f->dnorm, s);
  }
  NW_HIP(hipGetLastError());
  int flags[2];
  NW_TRY(read_flags(f, s, flags, norm));
  if (f->profile) add_event_times(f->ev_res, 1 << f->dim, &f->res_ms, &f->res_launches);
  return flags_status(flags);
}

fsimg_status assemble_jacobian(fsimg_fsi *f, const double *x, const double *u, const double *xo,
                               const double *uo, hipStream_t s) {
  fsimg_hier *h = f->mom;
  const int nlev = (int)h->lev.size();
  const AsmPhys P = asm_phys(f->phys);
  NW_TRY(clear_flags(f, s));
  for (int l = 0; l < nlev; ++l) {
    DevLevel &L = h->lev[l];
    FsiLevel &F = f->lev[l];
    AsmState S{x, u, xo, uo};
    if (l > 0) {
      const DevLevel &Lf = h->lev[l - 1];
      const FsiLevel &Ff = f->lev[l - 1];
      const double *src[4] = {l == 1 ? x : Ff.x, l == 1 ? u : Ff.u, l == 1 ? xo : Ff.xo,
                              l == 1 ? uo : Ff.uo};
      double *dst[4] = {F.x, F.u, F.xo, F.uo};
      const int comps[4] = {f->dim + 1, f->dim, f->dim + 1, f->dim};
      for (int q = 0; q < 4; ++q) launch_inject(src[q], dst[q], Lf.nnode, L.nnode, comps[q], s);
      S = AsmState{F.x, F.u, F.xo, F.uo};
    }
    launch_asm_jacobian(F.dev, f->dim, P, S, L.vals64, L.nrows, L.nnzb, f->dflag, s,
                        (f->profile && l == 0) ? f->ev_jac : nullptr);
    if (L.vals32) launch_cast_d2f(L.vals64, L.vals32, L.nnzb * L.b * L.b, s);
  }
  NW_HIP(hipGetLastError());
  h->factored = false;
  int flags[2];
  NW_TRY(read_flags(f, s, flags, nullptr));
  if (f->profile) add_event_times(f->ev_jac, 1 << f->dim, &f->jac_ms, &f->jac_launches);
  return flags_status(flags);
}

// held rows of x take scale * vals (a time step's Dirichlet data); a row out
// of range or not held in the momentum system sets bad[0] and is skipped.
// write = 0 only checks the list (nothing of x is written)
__global__ __launch_bounds__(256) void k_set_held_rows(double *__restrict__ x, const int64_t *__restrict__ rows,
                                                       const double *__restrict__ vals, int64_t n, int64_t nx,
                                                       const uint8_t *__restrict__ mask, double scale,
                                                       int write, int *__restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t r = rows[i];
  if (r < 0 || r >= nx || !mask[r]) {
    bad[0] = 1;
    return;
  }
  if (write) x[r] = scale * vals[i];
}

// out[j] = sum over the listed nodes of res[node * B + 1 + j] / k, j < D: one
// workgroup, each thread a strided partial sum, then a fixed-order tree in
// LDS (the same order on every call); a node out of range sets bad[0]
constexpr int kForceThreads = 256;
__global__ __launch_bounds__(kForceThreads) void k_force_sum(const double *__restrict__ res,
                                                             const int64_t *__restrict__ nodes, int64_t n,
                                                             int64_t nrows, int D, double inv_k,
                                                             double *__restrict__ out, int *__restrict__ bad) {
  __shared__ double part[3][kForceThreads];
  const int t = threadIdx.x, B = D + 1;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = t; i < n; i += kForceThreads) {
    const int64_t g = nodes[i];
    if (g < 0 || g >= nrows) {
      bad[0] = 1;
      continue;
    }
    for (int j = 0; j < D; ++j) acc[j] += res[g * B + 1 + j];
  }
  for (int j = 0; j < 3; ++j) part[j][t] = acc[j];
  __syncthreads();
  for (int w = kForceThreads / 2; w > 0; w >>= 1) {
    if (t < w)
      for (int j = 0; j < 3; ++j) part[j][t] += part[j][t + w];
    __syncthreads();
  }
  if (t < D) out[t] = part[t][0] * inv_k;
}

}  // namespace

extern "C" {

void fsimg_default_newton_opts(fsimg_newton_opts *o) {
  if (!o) return;
  o->rtol = 1e-8;
  o->atol = 0.0;
  o->max_steps = 20;
  o->gamma = 0.05;
  o->max_halvings = 4;
  o->lin_rtol = 0.0;
  o->ale_rtol = 0.0;
}

void fsimg_fsi_destroy(fsimg_fsi *f) {
  if (!f) return;
  (void)hipSetDevice(f->mom->ctx->device);
  for (auto &a : f->allocs) {
    (void)hipFree(a.first);
    f->mom->ctx->in_use -= a.second;
  }
  if (f->hflag) (void)hipHostFree(f->hflag);
  if (f->hnorm) (void)hipHostFree(f->hnorm);
  for (int i = 0; i < 16; ++i) {
    if (f->ev_jac[i]) (void)hipEventDestroy(f->ev_jac[i]);
    if (f->ev_res[i]) (void)hipEventDestroy(f->ev_res[i]);
  }
  delete f;
}

fsimg_status fsimg_fsi_set_profile(fsimg_fsi *f, int on) {
  if (!f) return nfail(FSIMG_ERR_ARG, "null object");
  NW_HIP(hipSetDevice(f->mom->ctx->device));
  if (on && !f->ev_jac[0])
    for (int i = 0; i < 16; ++i) {
      NW_HIP(hipEventCreate(&f->ev_jac[i]));
      NW_HIP(hipEventCreate(&f->ev_res[i]));
    }
  f->profile = on != 0;
  f->jac_ms = f->res_ms = 0.0;
  f->jac_launches = f->res_launches = 0;
  return FSIMG_OK;
}

fsimg_status fsimg_fsi_profile(const fsimg_fsi *f, double *jac_ms, int *jac_launches, double *res_ms,
                               int *res_launches) {
  if (!f) return nfail(FSIMG_ERR_ARG, "null object");
  if (jac_ms) *jac_ms = f->jac_ms;
  if (jac_launches) *jac_launches = f->jac_launches;
  if (res_ms) *res_ms = f->res_ms;
  if (res_launches) *res_launches = f->res_launches;
  return FSIMG_OK;
}

fsimg_status fsimg_fsi_create(fsimg_hier *mom, fsimg_hier *ale, const fsimg_fsi_level *levels,
                              const fsimg_phys *phys, fsimg_fsi **out) {
  if (!out) return nfail(FSIMG_ERR_ARG, "null output");
  *out = nullptr;
  if (!mom || !levels || !phys) return nfail(FSIMG_ERR_ARG, "null hierarchy, levels or parameters");
  const DevLevel &L0 = mom->lev[0];
  const int d = L0.dim;
  if (d < 2 || d > 3 || L0.b != d + 1)
    return nfail(FSIMG_ERR_ARG, "the momentum hierarchy needs dimension 2 or 3 and block d+1");
  if (!(phys->k > 0.0) || !(phys->theta > 0.0) || phys->theta > 1.0 || !(phys->rho_f > 0.0))
    return nfail(FSIMG_ERR_ARG, "bad physical parameters");
  if (ale) {
    const DevLevel &A0 = ale->lev[0];
    if (ale->ctx != mom->ctx || A0.dim != d || A0.b != d || A0.nrows != L0.nrows)
      return nfail(FSIMG_ERR_ARG, "the ALE hierarchy must share context, mesh and dimension (block d)");
  }
  for (size_t l = 0; l < mom->lev.size(); ++l) {
    const DevLevel &L = mom->lev[l];
    for (int a = 0; a < d; ++a)
      if (L.cells[a] < 1 || L.nnode[a] != 2 * L.cells[a] + 1 || !levels[l].coords[a])
        return nfail(FSIMG_ERR_ARG, "level " + std::to_string(l) + ": coordinates / cells missing");
    if (!levels[l].cell_solid) return nfail(FSIMG_ERR_ARG, "null cell_solid");
    if (l > 0) {
      const DevLevel &Lf = mom->lev[l - 1];
      for (int a = 0; a < d; ++a)
        if (Lf.cells[a] != 2 * L.cells[a])
          return nfail(FSIMG_ERR_ARG, "levels must be nested (cells halved per axis)");
    }
  }
  if (hipSetDevice(mom->ctx->device) != hipSuccess) return nfail(FSIMG_ERR_HIP, "hipSetDevice");
  auto *f = new fsimg_fsi;
  f->mom = mom;
  f->ale = ale;
  f->phys = *phys;
  f->dim = d;
  f->lev.resize(mom->lev.size());
  auto bail = [&](fsimg_status st) {
    fsimg_fsi_destroy(f);
    return st;
  };
#define NW_CHK(expr)                          \
  do {                                        \
    fsimg_status st__ = (expr);               \
    if (st__ != FSIMG_OK) return bail(st__);  \
  } while (0)
  for (size_t l = 0; l < mom->lev.size(); ++l) {
    const DevLevel &L = mom->lev[l];
    FsiLevel &F = f->lev[l];
    int64_t ncell = 1;
    for (int a = 0; a < d; ++a) ncell *= L.cells[a];
    for (int a = 0; a < d; ++a) {
      NW_CHK(falloc(f, &F.coord[a], (size_t)L.nnode[a]));
      if (hipMemcpy(F.coord[a], levels[l].coords[a], L.nnode[a] * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess)
        return bail(nfail(FSIMG_ERR_HIP, "coordinate upload failed"));
    }
    if (levels[l].node_coords) {
      NW_CHK(falloc(f, &F.xyz, (size_t)(L.nrows * d)));
      if (hipMemcpy(F.xyz, levels[l].node_coords, L.nrows * d * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess)
        return bail(nfail(FSIMG_ERR_HIP, "node position upload failed"));
    }
    NW_CHK(falloc(f, &F.solid, (size_t)ncell));
    if (hipMemcpy(F.solid, levels[l].cell_solid, ncell, hipMemcpyHostToDevice) != hipSuccess)
      return bail(nfail(FSIMG_ERR_HIP, "cell flag upload failed"));
    if (l > 0) {
      NW_CHK(falloc(f, &F.x, (size_t)(L.nrows * (d + 1))));
      NW_CHK(falloc(f, &F.xo, (size_t)(L.nrows * (d + 1))));
      NW_CHK(falloc(f, &F.u, (size_t)(L.nrows * d)));
      NW_CHK(falloc(f, &F.uo, (size_t)(L.nrows * d)));
    }
    AsmLevel &A = F.dev;
    for (int a = 0; a < 3; ++a) {
      A.coord[a] = a < d ? F.coord[a] : nullptr;
      A.cells[a] = L.cells[a];
      A.nnode[a] = L.nnode[a];
    }
    A.xyz = F.xyz;
    A.solid = F.solid;
    A.rowptr = L.rowptr;
    A.colind = L.colind;
    A.mask = L.mask;
  }
  // fine nodes of a solid cell (interface and solid: the support of eq. problem:2)
  {
    const DevLevel &L = mom->lev[0];
    std::vector<uint8_t> ns(L.nrows, 0);
    int64_t ncell = 1;
    for (int a = 0; a < d; ++a) ncell *= L.cells[a];
    for (int64_t e = 0; e < ncell; ++e) {
      if (!levels[0].cell_solid[e]) continue;
      int ea[3] = {0, 0, 0};
      int64_t r = e;
      for (int a = 0; a < d; ++a) {
        ea[a] = (int)(r % L.cells[a]);
        r /= L.cells[a];
      }
      for (int i = 0; i < (d == 3 ? 27 : 9); ++i) {
        int64_t g = 0, st = 1;
        for (int a = 0; a < d; ++a) {
          const int la = (i / (a == 0 ? 1 : (a == 1 ? 3 : 9))) % 3;
          g += st * (2 * ea[a] + la);
          st *= L.nnode[a];
        }
        ns[g] = 1;
      }
    }
    NW_CHK(falloc(f, &f->node_solid, (size_t)L.nrows));
    if (hipMemcpy(f->node_solid, ns.data(), L.nrows, hipMemcpyHostToDevice) != hipSuccess)
      return bail(nfail(FSIMG_ERR_HIP, "node flag upload failed"));
    NW_CHK(falloc(f, &f->res, (size_t)L.n));
    NW_CHK(falloc(f, &f->W, (size_t)L.n));
    NW_CHK(falloc(f, &f->xt, (size_t)L.n));
    if (ale) {
      const int64_t na = ale->lev[0].n;
      NW_CHK(falloc(f, &f->du, (size_t)na));
      NW_CHK(falloc(f, &f->b5, (size_t)na));
      NW_CHK(falloc(f, &f->ut, (size_t)na));
      NW_CHK(falloc(f, &f->ru, (size_t)na));
    }
    NW_CHK(falloc(f, &f->dflag, 2));
    NW_CHK(falloc(f, &f->dnorm, 1));
  }
  if (hipHostMalloc((void **)&f->hflag, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&f->hnorm, sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
    return bail(nfail(FSIMG_ERR_OOM, "pinned host memory"));
  // levels whose pattern is exactly the Q2 stencil find block positions by
  // arithmetic instead of a search in the row
  for (size_t l = 0; l < mom->lev.size(); ++l) {
    FsiLevel &F = f->lev[l];
    if (hipMemsetAsync(f->dflag, 0, sizeof(int), nullptr) != hipSuccess)
      return bail(nfail(FSIMG_ERR_HIP, "hipMemsetAsync failed"));
    launch_check_structured(F.dev, d, mom->lev[l].nrows, f->dflag, nullptr);
    if (hipMemcpy(f->hflag, f->dflag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
      return bail(nfail(FSIMG_ERR_HIP, "pattern check failed"));
    F.dev.structured = f->hflag[0] == 0 ? 1 : 0;
  }
#undef NW_CHK
  *out = f;
  return FSIMG_OK;
}

fsimg_status fsimg_fsi_residual(fsimg_fsi *f, const double *x, const double *u, const double *x_old,
                                const double *u_old, double *res, void *stream) {
  if (!f || !x || !u || !x_old || !u_old || !res) return nfail(FSIMG_ERR_ARG, "null argument");
  NW_HIP(hipSetDevice(f->mom->ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  double nrm;
  NW_TRY(eval_residual(f, x, u, x_old, u_old, s, &nrm, false));
  NW_HIP(hipMemcpyAsync(res, f->res, f->mom->lev[0].n * sizeof(double), hipMemcpyDeviceToDevice, s));
  NW_HIP(hipStreamSynchronize(s));
  return FSIMG_OK;
}

fsimg_status fsimg_fsi_jacobian(fsimg_fsi *f, const double *x, const double *u, const double *x_old,
                                const double *u_old, void *stream) {
  if (!f || !x || !u || !x_old || !u_old) return nfail(FSIMG_ERR_ARG, "null argument");
  NW_HIP(hipSetDevice(f->mom->ctx->device));
  f->have_jac = false;
  NW_TRY(assemble_jacobian(f, x, u, x_old, u_old, static_cast<hipStream_t>(stream)));
  return FSIMG_OK;
}

fsimg_status fsimg_fsi_drop_jacobian(fsimg_fsi *f) {
  if (!f) return nfail(FSIMG_ERR_ARG, "null object");
  f->have_jac = false;
  return FSIMG_OK;
}

fsimg_status fsimg_fsi_newton(fsimg_fsi *f, double *x, double *u, const double *x_old,
                              const double *u_old, const fsimg_newton_opts *opts,
                              fsimg_newton_stats *stats, void *stream) {
  if (!f || !x || !u || !x_old || !u_old) return nfail(FSIMG_ERR_ARG, "null argument");
  if (!f->ale) return nfail(FSIMG_ERR_ARG, "the Newton loop needs an ALE hierarchy");
  fsimg_newton_opts o;
  NW_TRY(newton_options(opts, &o));
  NW_HIP(hipSetDevice(f->mom->ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  NewtonRun &R = f->run;
  newton_begin(f, x, u, x_old, u_old, o, s);
  while (!R.done) {
    newton_prepare(f, s);
    if (R.done) break;
    // momentum: J W = R (eq. problem:1)
    auto t0 = std::chrono::steady_clock::now();
    fsimg_stats ls;
    const double keep = f->mom->opts.rtol;
    if (o.lin_rtol > 0.0) f->mom->opts.rtol = o.lin_rtol;
    fsimg_status ss = fsimg_solve(f->mom, f->res, f->W, &ls, s);
    f->mom->opts.rtol = keep;
    R.st.lin_iters_mom += ls.iters;
    if (ss != FSIMG_OK) {
      R.st.ms_solve += ms_since(t0);
      newton_fail(f, ss);
      break;
    }
    newton_lift(f, s);
    // ALE extension (eq. problem:3)
    const double keep_ale = f->ale->opts.rtol;
    if (o.ale_rtol > 0.0) f->ale->opts.rtol = o.ale_rtol;
    ss = fsimg_solve(f->ale, f->b5, f->du, &ls, s);
    f->ale->opts.rtol = keep_ale;
    R.st.lin_iters_ale += ls.iters;
    R.st.ms_solve += ms_since(t0);
    if (ss != FSIMG_OK) {
      newton_fail(f, ss);
      break;
    }
    newton_finish_step(f, s);
  }
  const fsimg_newton_stats st = newton_end(f, s);
  if (stats) *stats = st;
  return static_cast<fsimg_status>(st.status);
}

fsimg_status fsimg_fsi_time_step(fsimg_fsi *f, double *x, double *u, double *x_old, double *u_old,
                                 const int64_t *rows, const double *vals, int64_t n_rows, double scale,
                                 const fsimg_newton_opts *opts, fsimg_newton_stats *stats, void *stream) {
  if (!f || !x || !u || !x_old || !u_old) return nfail(FSIMG_ERR_ARG, "null argument");
  if (n_rows < 0 || (n_rows > 0 && (!rows || !vals))) return nfail(FSIMG_ERR_ARG, "bad held-row list");
  if (!f->ale) return nfail(FSIMG_ERR_ARG, "the Newton loop needs an ALE hierarchy");
  if (x == x_old || u == u_old) return nfail(FSIMG_ERR_ARG, "the old level needs buffers of its own");
  fsimg_newton_opts o;
  NW_TRY(newton_options(opts, &o));  // before anything is written
  NW_HIP(hipSetDevice(f->mom->ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevLevel &L = f->mom->lev[0];
  const int64_t na = L.nrows * f->dim;
  const dim3 grid((unsigned)((n_rows + 255) / 256));
  if (n_rows > 0) {  // check the list first: a refused call writes none of x, u, x_old, u_old
    NW_TRY(clear_flags(f, s));
    hipLaunchKernelGGL(k_set_held_rows, grid, dim3(256), 0, s, x, rows, vals, n_rows, L.n, L.mask, scale, 0,
                       f->dflag);
    NW_HIP(hipGetLastError());
    int flags[2];
    NW_TRY(read_flags(f, s, flags, nullptr));
    if (flags[0]) return nfail(FSIMG_ERR_ARG, "a held-row index is out of range or not a held row");
  }
  NW_HIP(hipMemcpyAsync(x_old, x, L.n * sizeof(double), hipMemcpyDeviceToDevice, s));
  NW_HIP(hipMemcpyAsync(u_old, u, na * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (n_rows > 0) {
    hipLaunchKernelGGL(k_set_held_rows, grid, dim3(256), 0, s, x, rows, vals, n_rows, L.n, L.mask, scale, 1,
                       f->dflag);
    NW_HIP(hipGetLastError());
  }
  return fsimg_fsi_newton(f, x, u, x_old, u_old, opts, stats, stream);
}

fsimg_status fsimg_fsi_force(fsimg_fsi *f, const double *x, const double *u, const double *x_old,
                             const double *u_old, const int64_t *nodes, int64_t n_nodes, double *force,
                             void *stream) {
  if (!f || !x || !u || !x_old || !u_old || !force) return nfail(FSIMG_ERR_ARG, "null argument");
  if (n_nodes < 0 || (n_nodes > 0 && !nodes)) return nfail(FSIMG_ERR_ARG, "bad node list");
  NW_HIP(hipSetDevice(f->mom->ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevLevel &L = f->mom->lev[0];
  if (!f->zero_mask) {
    NW_TRY(falloc(f, &f->zero_mask, (size_t)L.n));
    NW_TRY(falloc(f, &f->dforce, 3));
    NW_HIP(hipMemsetAsync(f->zero_mask, 0, (size_t)L.n, s));
  }
  AsmLevel all = f->lev[0].dev;
  all.mask = f->zero_mask;
  NW_TRY(clear_flags(f, s));
  launch_asm_residual(all, f->dim, asm_phys(f->phys), AsmState{x, u, x_old, u_old}, f->res, L.nrows,
                      f->dflag, s, nullptr);
  hipLaunchKernelGGL(k_force_sum, dim3(1), dim3(kForceThreads), 0, s, f->res, nodes, n_nodes, L.nrows, f->dim,
                     1.0 / f->phys.k, f->dforce, f->dflag + 1);
  NW_HIP(hipGetLastError());
  double h[3];
  NW_HIP(hipMemcpyAsync(h, f->dforce, f->dim * sizeof(double), hipMemcpyDeviceToHost, s));
  int flags[2];
  NW_TRY(read_flags(f, s, flags, nullptr));
  if (flags[1]) return nfail(FSIMG_ERR_ARG, "a force node index is out of range");
  if (flags[0]) return nfail(FSIMG_ERR_SINGULAR, "det F <= 0 at a Gauss point (inverted element)");
  for (int j = 0; j < f->dim; ++j) force[j] = h[j];
  return FSIMG_OK;
}

}  // extern "C"

// ------------------------------------------------------------ Newton stages
namespace fsimg {

fsimg_status check_newton_options(const fsimg_newton_opts *opts, fsimg_newton_opts *o) {
  return newton_options(opts, o);
}

void newton_fail(fsimg_fsi *f, fsimg_status status) {
  f->run.done = true;
  f->run.status = status;
}

void newton_begin(fsimg_fsi *f, double *x, double *u, const double *xo, const double *uo,
                  const fsimg_newton_opts &o, hipStream_t s) {
  NewtonRun &R = f->run;
  R = NewtonRun{};
  R.o = o;
  R.x = x;
  R.u = u;
  R.xo = xo;
  R.uo = uo;
  R.done = false;
  R.status = FSIMG_OK;
  std::memset(&R.st, 0, sizeof R.st);
  R.t_start = std::chrono::steady_clock::now();
  // the ALE matrix never changes: factor it once
  if (!f->ale->factored) {
    const fsimg_status fs = fsimg_factor(f->ale, s);
    if (fs != FSIMG_OK) return newton_fail(f, fs);
  }
  const auto t0 = std::chrono::steady_clock::now();
  const fsimg_status rs = eval_residual(f, x, u, xo, uo, s, &R.nrm, true);
  R.st.ms_residual += ms_since(t0);
  if (rs != FSIMG_OK) return newton_fail(f, rs);
  R.nrm0 = R.nrm;
  R.st.res0 = R.nrm;
  R.st.res_hist[0] = R.nrm;
  R.rate = -1.0;
  if (R.nrm <= std::max(o.rtol * R.nrm0, o.atol)) R.done = true;
}

void newton_prepare(fsimg_fsi *f, hipStream_t s) {
  NewtonRun &R = f->run;
  if (R.done) return;
  if (R.st.steps >= R.o.max_steps)
    return newton_fail(f, nfail(FSIMG_ERR_NOCONV, "the Newton loop reached max_steps"));
  if (!f->have_jac || R.rate > R.o.gamma) {
    auto t0 = std::chrono::steady_clock::now();
    fsimg_status js = assemble_jacobian(f, R.x, R.u, R.xo, R.uo, s);
    R.st.ms_jacobian += ms_since(t0);
    if (js != FSIMG_OK) return newton_fail(f, js);
    t0 = std::chrono::steady_clock::now();
    f->have_jac = false;
    js = fsimg_factor(f->mom, s);
    if (js == FSIMG_OK && hipStreamSynchronize(s) != hipSuccess)
      js = nfail(FSIMG_ERR_HIP, "synchronisation after the factorisation failed");
    R.st.ms_factor += ms_since(t0);
    if (js != FSIMG_OK) return newton_fail(f, js);
    f->have_jac = true;
    ++R.st.jacobians;
  }
  launch_fill<double>(f->W, f->mom->lev[0].n, 0.0, s);
}

void newton_lift(fsimg_fsi *f, hipStream_t s) {
  // interface / solid deformation increment (eq. problem:2 with its
  // right-hand side): the condensation residual plus k theta W_v
  const DevLevel &Lm = f->mom->lev[0];
  launch_deform(Lm.nrows, f->dim, f->node_solid, f->phys.k, f->phys.theta, f->W, f->dim + 1, 1, f->ru,
                nullptr, f->du, s);
}

void newton_finish_step(fsimg_fsi *f, hipStream_t s) {
  NewtonRun &R = f->run;
  if (R.done) return;
  const DevLevel &Lm = f->mom->lev[0];
  const DevLevel &La = f->ale->lev[0];
  // line search: a trial state with an inverted element (det F <= 0) counts
  // as no decrease
  double omega = 1.0, nt = 0.0;
  for (int hv = 0;; ++hv) {
    launch_axpy_to(R.x, f->W, omega, f->xt, Lm.n, s);
    launch_axpy_to(R.u, f->du, omega, f->ut, La.n, s);
    const auto t0 = std::chrono::steady_clock::now();
    const fsimg_status rs = eval_residual(f, f->xt, f->ut, R.xo, R.uo, s, &nt, true);
    R.st.ms_residual += ms_since(t0);
    const bool inverted = rs == FSIMG_ERR_SINGULAR;
    if (rs != FSIMG_OK && !inverted) return newton_fail(f, rs);
    if (inverted && hv >= R.o.max_halvings) return newton_fail(f, rs);
    if (!inverted && (nt < R.nrm || hv >= R.o.max_halvings)) break;
    omega *= 0.5;
    ++R.st.halvings;
  }
  if (hipMemcpyAsync(R.x, f->xt, Lm.n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(R.u, f->ut, La.n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return newton_fail(f, nfail(FSIMG_ERR_HIP, "state update failed"));
  if (R.st.steps < 32) R.st.omega_hist[R.st.steps] = omega;
  R.rate = nt / R.nrm;
  R.nrm = nt;
  ++R.st.steps;
  if (R.st.steps < 32) R.st.res_hist[R.st.steps] = R.nrm;
  if (R.nrm <= std::max(R.o.rtol * R.nrm0, R.o.atol)) R.done = true;
}

fsimg_newton_stats newton_end(fsimg_fsi *f, hipStream_t s) {
  NewtonRun &R = f->run;
  if (hipStreamSynchronize(s) != hipSuccess && R.status == FSIMG_OK)
    R.status = nfail(FSIMG_ERR_HIP, "synchronisation at the end of the time step failed");
  R.st.res = R.nrm;
  R.st.status = R.status;
  R.st.ms_total = ms_since(R.t_start);
  R.done = true;
  return R.st;
}

size_t fsi_bytes(const fsimg_level_desc *mom, int nlev, bool with_ale, const fsimg_fsi_level *geom) {
  size_t b = 0;
  const int d = mom[0].dim;
  for (int l = 0; l < nlev; ++l) {
    if (geom && geom[l].node_coords) b += (size_t)mom[l].nrows * d * sizeof(double);
    int64_t ncell = 1;
    for (int a = 0; a < d; ++a) {
      b += (size_t)(2 * mom[l].cells[a] + 1) * sizeof(double);
      ncell *= mom[l].cells[a];
    }
    b += (size_t)ncell;
    if (l > 0) b += (size_t)mom[l].nrows * (2 * (d + 1) + 2 * d) * sizeof(double);
  }
  const int64_t n = mom[0].nrows;
  b += (size_t)n + 3 * (size_t)n * (d + 1) * sizeof(double);
  if (with_ale) b += 4 * (size_t)n * d * sizeof(double);
  return b + 2 * sizeof(int) + sizeof(unsigned long long);
}

}  // namespace fsimg
