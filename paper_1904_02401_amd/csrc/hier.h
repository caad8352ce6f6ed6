// Host-side structures of contexts and hierarchies, shared by the C-ABI
// implementation and the batched solve driver.
#pragma once
#include <array>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "fsimg_internal.h"

struct BatchPlan;
using fsimg::DevLevel;

namespace fsimg {
struct TuneTable {
  // (fsimg_tune_kind, block size or patch size, word bytes, floor(log2 size)) -> value
  std::map<std::array<int, 4>, int> entries;
};
}  // namespace fsimg

struct fsimg_ctx {
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;
  size_t plan_bytes = 0;  // part of in_use held by cached batch plans
  std::vector<BatchPlan *> plans;  // descriptor tables of recent batch compositions (LRU)
  fsimg::TuneTable tune;           // launch shapes of this context's kernels
  // the patch factorisations' stream while a coarse inverse runs beside
  // them: all CUs but kReservedCus, so that the coarse chain's one-workgroup
  // panel launches find a free CU at once.  One per context: a CU-masked
  // stream holds a hardware queue of its own, and one per hierarchy
  // oversubscribes the queues (every kernel of the process slows down).
  // nullptr: not created yet, or the runtime refused the mask
  hipStream_t pstream = nullptr;
  bool pstream_tried = false;
};

struct EventTimer {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  void begin_solve() { used = 0; }
  hipEvent_t next() {
    if (used == ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev.push_back(e);
    }
    return ev[used++];
  }
  double total_ms(int *count) const {
    double t = 0.0;
    int c = 0;
    for (size_t i = 0; i + 1 < used; i += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) { t += ms; ++c; }
    }
    *count = c;
    return t;
  }
  ~EventTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

struct fsimg_hier {
  uint64_t uid = 0;  // unique per created hierarchy (batch plan cache key)
  fsimg_ctx *ctx = nullptr;
  fsimg_opts opts{};
  std::vector<DevLevel> lev;
  std::vector<std::pair<void *, size_t>> allocs;
  std::vector<std::vector<uint8_t>> host_mask;
  std::vector<std::vector<uint8_t>> host_class;
  bool factored = false;
  double setup_ms = 0.0, factor_ms = 0.0;  // host wall time of create / the last factor
  int m = 20;
  // FGMRES workspace (FP64)
  double *V = nullptr, *Z = nullptr, *w = nullptr, *partial = nullptr, *small = nullptr;
  double *hpin = nullptr;
  int *dstatus = nullptr;
  int *hstatus = nullptr;
  EventTimer tv, ts;
  bool profiling = false;
  hipStream_t ilu_cap = nullptr;  // capture stream of the ILU sweep graphs
  // the coarse inverse runs on this stream while the patch factorisations of
  // the finer levels run on the caller's (fork / join events)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};


namespace fsimg {
fsimg_status set_error(fsimg_status s, const std::string &msg);
void destroy_plan(BatchPlan *p);
constexpr size_t kPlanCache = 8;  // batch compositions whose descriptor tables stay cached
// device bytes one instance adds to a batch plan whose deepest hierarchy has
// nlev levels, plus the plan's fixed part (an upper bound)
size_t plan_bytes_bound(int nlev);
bool plan_covers(const BatchPlan *p, uint64_t uid);
void drop_plans(fsimg_ctx *ctx);  // destroy every cached batch plan (e.g. after a shape change)
// batched FGMRES over n hierarchies (shared options / precision / block size)
fsimg_status solve_batch(fsimg_ctx *ctx, int n, fsimg_hier *const *hs, const double *const *b,
                         double *const *x, fsimg_stats *stats, hipStream_t s);
// One step of the multigrid path of one hierarchy through the batched kernels
// (the launches its solve makes, with one instance), on the caller's vectors
// of the hierarchy's V-cycle precision: the inputs are copied into the
// level's work vectors and the result is copied out.  GATHER / Vanka
// hierarchies only; `level` < the coarsest except for ONE_COARSE (the
// coarsest, FP64 hierarchies) and ONE_VCYCLE (0).
//   ONE_RESIDUAL  out = a - A_l b, 0 at identity rows
//   ONE_VANKA     out += Vanka correction of a - A_l out (one smoothing step)
//   ONE_RESTRICT  out = R a (level l -> l + 1), 0 at coarse identity rows
//   ONE_PROLONG   out += P a (level l + 1 -> l), then 0 at fine identity rows
//   ONE_COARSE    out = A_{L-1}^{-1} a on the free dofs, 0 at identity rows
//   ONE_VCYCLE    out = V-cycle(a)
enum SingleOp { ONE_RESIDUAL = 0, ONE_VANKA, ONE_RESTRICT, ONE_PROLONG, ONE_COARSE, ONE_VCYCLE };
// The no-allocation solve: noalloc_init looks up the calling device's copy of
// the fixed scratch array (device current; once per device, at context
// creation); solve_noalloc is fsimg_solve of one GATHER / Vanka hierarchy
// with its tables in that array, launched eagerly.
fsimg_status noalloc_init(int device);
size_t noalloc_scratch_bytes();
fsimg_status solve_noalloc(fsimg_hier *h, const double *b, double *x, fsimg_stats *stats,
                           hipStream_t s);
fsimg_status single_step(fsimg_hier *h, int op, int level, const void *a, const void *b, void *out,
                         hipStream_t s);
}  // namespace fsimg
