// Batched solve driver: FGMRES(m) + V-cycle over many independent
// hierarchies at once, one launch per operation and level for all of them.
//
// Levels are aligned from the top (level 0 = finest of every instance).  At
// level l an instance either smooths (l < L_i - 1), solves its coarse problem
// (l = L_i - 1) or has nothing to do, so each instance runs exactly the
// V-cycle it would run alone.  The Krylov iterations advance in lockstep: one
// device-to-host copy per iteration returns every instance's new Hessenberg
// column, the Givens rotations and stop tests run per instance on the host,
// and instances that stop are masked out of the following launches.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "hier.h"

using namespace fsimg;

struct BatchPlan {
  fsimg_ctx *ctx = nullptr;  // the budget the descriptor tables are charged to
  std::vector<uint64_t> key;
  int n = 0, Lmax = 0, b = 0, dim = 0, np = 0, nl = 0, npc = 0;
  bool mixed = false;
  std::vector<int> rpw, ppw;  // per level: SpMV rows per wave, Vanka patches per workgroup
  std::vector<int> ppw2;      // per level: block patches per workgroup
  int np2 = 0, nl2 = 0, npc2 = 0;  // block patches (0: none in any instance)
  int rpw0 = 1;               // FP64 level-0 SpMV (A z, true residual)
  void *dbuf = nullptr;
  size_t dbytes = 0;
  size_t kry_off = 0;
  DLev *dlev = nullptr;  // [Lmax][n]
  DKry *dkry = nullptr;  // [n]
  int *active = nullptr, *kcnt = nullptr, *flags = nullptr, *cyc = nullptr;
  int *cnt = nullptr;  // per instance: workgroups done in the current reduction pass
  double *hs = nullptr;  // [n * kHS]
  DGiv *gv = nullptr;    // [n] FGMRES control state
  std::vector<WorkSet> ws_spmv, ws_patch, ws_patch2, ws_gather, ws_restrict, ws_prolong, ws_cn, ws_cf;
  // the V-cycle's work sets without the levels an instance runs in its
  // small-level kernel (the same as ws_* where no instance has such levels)
  std::vector<WorkSet> vs_spmv, vs_patch, vs_patch2, vs_gather, vs_restrict, vs_prolong;
  // per level c: the instances whose coarsest level is c and that run the
  // levels tfrom[i] .. c - 1 in kb_vcycle_tail
  std::vector<const int32_t *> tail_inst;
  std::vector<int> tail_n;
  const int32_t *tfrom = nullptr;
  bool tails = false;
  bool zfuse = false;  // every instance has >= 2 levels: z_j can come from the last gather
  WorkSet ws_row0{}, ws_vec0{}, ws_kry{}, ws_inst{};
  std::vector<DKry> hkry;
  // pinned host staging: the active flags after each iteration j of a cycle
  // (ring[j * n + i]), cyc | kcnt after a cycle, the control states at the end
  int *ring_host = nullptr;
  int *int_host = nullptr;
  DGiv *gv_host = nullptr;
  hipEvent_t ev[kMaxVec] = {};  // recorded after iteration j's flags are copied
  EventTimer tv, ts, tr, tp;  // finest level: Vanka, SpMV, restriction, prolongation
  // FGMRES iteration j (copy-in, V-cycle, copy-out, A z_j, CGS2, norm, scale,
  // Givens update and stop test, active flags to the host) captured once per j
  hipStream_t cap = nullptr;
  std::vector<hipGraphExec_t> iter_graph;
  fsimg_opts graph_opts{};
  // tables placed in a buffer the plan does not own (the no-allocation
  // solve): never freed here, staging in the host arrays below
  bool fixed = false;
  int ring_one[kMaxVec] = {};
  int int_one[2] = {};
  DGiv gv_one{};
};

namespace fsimg {

void destroy_plan(BatchPlan *p) {
  if (!p) return;
  for (hipGraphExec_t g : p->iter_graph)
    if (g) (void)hipGraphExecDestroy(g);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->fixed) {
    delete p;
    return;
  }
  if (p->dbuf) {
    (void)hipFree(p->dbuf);
    if (p->ctx) {
      p->ctx->in_use -= p->dbytes;
      p->ctx->plan_bytes -= p->dbytes;
    }
  }
  for (hipEvent_t e : p->ev)
    if (e) (void)hipEventDestroy(e);
  if (p->ring_host) (void)hipHostFree(p->ring_host);
  if (p->int_host) (void)hipHostFree(p->int_host);
  if (p->gv_host) (void)hipHostFree(p->gv_host);
  delete p;
}

size_t plan_bytes_bound(int nlev) {
  // per instance: level descriptors, Krylov descriptor, five flags, its
  // first small level and tail-list entry, the Hessenberg slot, the FGMRES
  // control state and one (instance, prefix) entry in each work set (level
  // sets twice: all levels, and the V-cycle's without the small levels); per
  // plan: one prefix entry and 64-byte alignment of every table
  const size_t nset = 14 * (size_t)nlev + 4, ntab = 10 + 2 * nset + nlev;
  return (size_t)nlev * sizeof(DLev) + sizeof(DKry) + 7 * sizeof(int) + kHS * sizeof(double) +
         sizeof(DGiv) + nset * (sizeof(int32_t) + 2 * sizeof(int64_t)) + ntab * 64;
}

void drop_plans(fsimg_ctx *ctx) {
  for (BatchPlan *p : ctx->plans) destroy_plan(p);
  ctx->plans.clear();
}

bool plan_covers(const BatchPlan *p, uint64_t uid) {
  if (!p) return false;
  for (uint64_t k : p->key)
    if (k == uid) return true;
  return false;
}

namespace {

struct Blob {
  std::vector<unsigned char> data;
  size_t add(const void *src, size_t bytes) {
    const size_t off = (data.size() + 63) & ~size_t(63);
    data.resize(off + bytes);
    if (src && bytes) std::memcpy(data.data() + off, src, bytes);
    return off;
  }
};

struct WsHost {
  std::vector<int32_t> inst;
  std::vector<int64_t> pre{0};
  void push(int i, int64_t blocks) {
    if (blocks <= 0) return;
    inst.push_back(i);
    pre.push_back(pre.back() + blocks);
  }
};

struct WsRef {
  size_t inst_off, pre_off;
  int nset;
  int64_t nblocks;
};

WsRef stage(Blob &blob, const WsHost &w) {
  WsRef r;
  r.nset = (int)w.inst.size();
  r.nblocks = w.pre.back();
  r.inst_off = blob.add(w.inst.data(), w.inst.size() * sizeof(int32_t));
  r.pre_off = blob.add(w.pre.data(), w.pre.size() * sizeof(int64_t));
  return r;
}

WorkSet resolve(void *base, const WsRef &r) {
  WorkSet w;
  w.inst = reinterpret_cast<const int32_t *>(static_cast<unsigned char *>(base) + r.inst_off);
  w.pre = reinterpret_cast<const int64_t *>(static_cast<unsigned char *>(base) + r.pre_off);
  w.nset = r.nset;
  w.nblocks = r.nblocks;
  return w;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

DLev to_dlev(const DevLevel &L) {
  DLev d{};
  d.rowptr = L.rowptr; d.colind = L.colind; d.v64 = L.vals64; d.v32 = L.vals32; d.mask = L.mask;
  d.nrows = L.nrows; d.n = L.n;
  for (int a = 0; a < 3; ++a) d.cells[a] = L.cells[a];
  d.npatch = L.npatch; d.pnodes = L.pnodes; d.inv64 = L.inv64; d.inv32 = L.inv32;
  d.npatch2 = L.blk.npatch; d.yofs2 = L.blk.yofs; d.pnodes2 = L.blk.pnodes;
  d.inv64_2 = L.blk.inv64; d.inv32_2 = L.blk.inv32;
  d.gptr = L.gptr; d.gidx = L.gidx; d.sc64 = L.scale64; d.sc32 = L.scale32;
  d.r64 = L.r64; d.x64 = L.x64; d.d64 = L.d64; d.Y64 = L.Y64;
  d.r32 = L.r32; d.x32 = L.x32; d.d32 = L.d32; d.Y32 = L.Y32;
  d.nfree = L.nfree; d.cfree = L.cfree; d.cinv = L.cinv; d.ct0 = L.ct0; d.ct1 = L.ct1;
  return d;
}

// the first level of hierarchy h that the small-level kernel runs: the
// levels from there to the coarsest-but-one each hold at most
// opts.small_level_kib KiB of patch inverses and matrix values in the
// V-cycle's precision (L - 1: none)
int tail_from(const fsimg_hier *h) {
  const int L = (int)h->lev.size();
  const double limit = 1024.0 * h->opts.small_level_kib;
  if (limit <= 0.0 || h->opts.smoother != FSIMG_SMOOTHER_VANKA ||
      h->opts.vanka_schedule != FSIMG_VANKA_GATHER)
    return L - 1;
  const bool f32 = h->opts.precision == FSIMG_MIXED;
  const double w = f32 ? 4.0 : 8.0;
  int from = L - 1;
  for (int l = L - 2; l >= 0; --l) {
    const DevLevel &D = h->lev[l];
    const double bytes = (double)D.npatch * D.np * (f32 ? D.npc32 : D.npc64) * w +
                         (double)D.blk.npatch * D.blk.np * (f32 ? D.blk.npc32 : D.blk.npc64) * w +
                         (double)D.nnzb * D.b * D.b * w;
    if (bytes > limit) break;
    from = l;
  }
  return from;
}

// fixed != nullptr: place the tables in that device buffer of fixed_bytes
// (uploaded on stream s) instead of allocating, and stage through the plan's
// own host arrays (one instance only)
fsimg_status build_plan(fsimg_ctx *ctx, int n, fsimg_hier *const *hs, BatchPlan **out,
                        void *fixed = nullptr, size_t fixed_bytes = 0, hipStream_t s = nullptr) {
  auto *P = new BatchPlan;
  P->n = n;
  P->b = hs[0]->lev[0].b;
  P->dim = hs[0]->lev[0].dim;
  P->nl = hs[0]->lev[0].nl;
  P->np = hs[0]->lev[0].np;
  P->mixed = hs[0]->opts.precision == FSIMG_MIXED;
  P->npc = P->mixed ? hs[0]->lev[0].npc32 : hs[0]->lev[0].npc64;
  for (int i = 0; i < n; ++i) {
    P->key.push_back(hs[i]->uid);
    P->Lmax = std::max(P->Lmax, (int)hs[i]->lev.size());
  }
  const int Lmax = P->Lmax;
  // launch shapes per level, from the largest instance at that level
  const int word = P->mixed ? 4 : 8;
  P->rpw.assign(Lmax, 1);
  P->ppw.assign(Lmax, 1);
  P->ppw2.assign(Lmax, 1);
  for (int i = 0; i < n; ++i)
    for (const DevLevel &L : hs[i]->lev)
      if (L.blk.npatch > 0) {
        P->np2 = L.blk.np;
        P->nl2 = L.blk.nl;
        P->npc2 = P->mixed ? L.blk.npc32 : L.blk.npc64;
      }
  for (int l = 0; l < Lmax; ++l) {
    int64_t rows = 0, patches = 0, blocks = 0;
    for (int i = 0; i < n; ++i)
      if (l < (int)hs[i]->lev.size()) {
        rows = std::max(rows, hs[i]->lev[l].nrows);
        patches = std::max(patches, hs[i]->lev[l].npatch);
        blocks = std::max(blocks, hs[i]->lev[l].blk.npatch);
      }
    const TuneTable *tt = hs[0]->lev[0].tune;
    P->rpw[l] = spmv_rows_per_wave(tt, P->b, word, rows);
    P->ppw[l] = vanka_patches_per_wg(tt, P->np, word, patches);
    if (blocks > 0) P->ppw2[l] = vanka_patches_per_wg(tt, P->np2, word, blocks);
  }
  {
    int64_t rows = 0;
    for (int i = 0; i < n; ++i) rows = std::max(rows, hs[i]->lev[0].nrows);
    P->rpw0 = spmv_rows_per_wave(hs[0]->lev[0].tune, P->b, 8, rows);
  }
  Blob blob;
  std::vector<DLev> dl((size_t)Lmax * n);
  for (int l = 0; l < Lmax; ++l)
    for (int i = 0; i < n; ++i)
      if (l < (int)hs[i]->lev.size()) dl[(size_t)l * n + i] = to_dlev(hs[i]->lev[l]);
  const size_t lev_off = blob.add(dl.data(), dl.size() * sizeof(DLev));
  P->hkry.resize(n);
  P->kry_off = blob.add(nullptr, n * sizeof(DKry));
  const size_t act_off = blob.add(nullptr, n * sizeof(int));
  const size_t k_off = blob.add(nullptr, n * sizeof(int));
  const size_t fl_off = blob.add(nullptr, n * sizeof(int));
  const size_t cyc_off = blob.add(nullptr, n * sizeof(int));
  const size_t cnt_off = blob.add(nullptr, n * sizeof(int));
  const size_t hs_off = blob.add(nullptr, (size_t)n * kHS * sizeof(double));
  const size_t gv_off = blob.add(nullptr, (size_t)n * sizeof(DGiv));
  std::vector<WsRef> r_spmv, r_patch, r_patch2, r_gather, r_restrict, r_prolong, r_cn, r_cf;
  std::vector<WsRef> v_spmv, v_patch, v_patch2, v_gather, v_restrict, v_prolong;
  std::vector<int> from(n);
  P->zfuse = true;
  for (int i = 0; i < n; ++i) {
    from[i] = tail_from(hs[i]);
    P->tails = P->tails || from[i] < (int)hs[i]->lev.size() - 1;
    P->zfuse = P->zfuse && hs[i]->lev.size() >= 2;
  }
  const size_t tfrom_off = blob.add(from.data(), n * sizeof(int32_t));
  std::vector<size_t> tail_off(Lmax, 0);
  P->tail_n.assign(Lmax, 0);
  for (int l = 0; l < Lmax; ++l) {
    std::vector<int32_t> tl;
    for (int i = 0; i < n; ++i)
      if ((int)hs[i]->lev.size() - 1 == l && from[i] < l) tl.push_back(i);
    P->tail_n[l] = (int)tl.size();
    if (!tl.empty()) tail_off[l] = blob.add(tl.data(), tl.size() * sizeof(int32_t));
  }
  for (int l = 0; l < Lmax; ++l) {
    WsHost sp, pa, pa2, ga, re, pr, cn, cf;
    WsHost vsp, vpa, vpa2, vga, vre, vpr;
    for (int i = 0; i < n; ++i) {
      const int Li = (int)hs[i]->lev.size();
      if (l < from[i]) {
        const DevLevel &L = hs[i]->lev[l];
        vsp.push(i, cdiv(L.nrows, 4 * P->rpw[l] * spmv_group_rows(P->b, word)));
        vpa.push(i, cdiv(L.npatch, P->ppw[l]));
        vpa2.push(i, cdiv(L.blk.npatch, P->ppw2[l]));
        vga.push(i, cdiv(L.n, 256));
        const DevLevel &Cl = hs[i]->lev[l + 1];
        vre.push(i, P->dim == 3 ? restrict3_blocks(Cl.cells[0], Cl.cells[1], Cl.cells[2])
                                : cdiv(Cl.nrows, 256));
        vpr.push(i, cdiv(L.nrows, 256));
      }
      if (l < Li - 1) {
        const DevLevel &L = hs[i]->lev[l];
        sp.push(i, cdiv(L.nrows, 4 * P->rpw[l] * spmv_group_rows(P->b, word)));
        pa.push(i, cdiv(L.npatch, P->ppw[l]));
        pa2.push(i, cdiv(L.blk.npatch, P->ppw2[l]));
        ga.push(i, cdiv(L.n, 256));
        const DevLevel &Cl = hs[i]->lev[l + 1];
        re.push(i, P->dim == 3 ? restrict3_blocks(Cl.cells[0], Cl.cells[1], Cl.cells[2])
                               : cdiv(Cl.nrows, 256));
        pr.push(i, cdiv(L.nrows, 256));
      } else if (l == Li - 1) {
        const DevLevel &L = hs[i]->lev[l];
        cn.push(i, cdiv(L.n, 256));
        cf.push(i, cdiv(L.nfree, 4) + cdiv(L.n, 256));
      }
    }
    r_spmv.push_back(stage(blob, sp));
    r_patch.push_back(stage(blob, pa));
    r_patch2.push_back(stage(blob, pa2));
    r_gather.push_back(stage(blob, ga));
    r_restrict.push_back(stage(blob, re));
    r_prolong.push_back(stage(blob, pr));
    r_cn.push_back(stage(blob, cn));
    r_cf.push_back(stage(blob, cf));
    if (P->tails) {
      v_spmv.push_back(stage(blob, vsp));
      v_patch.push_back(stage(blob, vpa));
      v_patch2.push_back(stage(blob, vpa2));
      v_gather.push_back(stage(blob, vga));
      v_restrict.push_back(stage(blob, vre));
      v_prolong.push_back(stage(blob, vpr));
    }
  }
  WsHost row0, vec0, kr, ins;
  for (int i = 0; i < n; ++i) {
    const DevLevel &L = hs[i]->lev[0];
    row0.push(i, cdiv(L.nrows, 4 * P->rpw0 * spmv_group_rows(P->b, 8)));
    vec0.push(i, cdiv(L.n, 256));
    kr.push(i, krylov_blocks(L.n));
    ins.push(i, 1);
  }
  const WsRef r_row0 = stage(blob, row0), r_vec0 = stage(blob, vec0), r_kry = stage(blob, kr),
              r_ins = stage(blob, ins);
  P->dbytes = blob.data.size();
  if (fixed) {
    if (n != 1 || P->dbytes > fixed_bytes) {
      delete P;
      return set_error(FSIMG_ERR_ARG, "the hierarchy's solve tables (" + std::to_string(blob.data.size()) +
                                          " bytes) exceed the fixed scratch array (" +
                                          std::to_string(fixed_bytes) + " bytes)");
    }
    P->fixed = true;
    P->dbuf = fixed;
    // every table (flags, Hessenberg column, descriptors) is rewritten here
    if (hipMemcpyAsync(P->dbuf, blob.data.data(), P->dbytes, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      delete P;
      return set_error(FSIMG_ERR_HIP, "descriptor upload to the scratch array failed");
    }
  } else {
    if (ctx->budget && ctx->in_use + P->dbytes > ctx->budget) {
      delete P;
      return set_error(FSIMG_ERR_BUDGET, "batch descriptor tables exceed the HBM budget");
    }
    if (hipMalloc(&P->dbuf, P->dbytes) != hipSuccess) {
      (void)hipGetLastError();
      delete P;
      return set_error(FSIMG_ERR_OOM, "batch descriptor allocation failed");
    }
    P->ctx = ctx;
    ctx->in_use += P->dbytes;
    ctx->plan_bytes += P->dbytes;
    if (hipMemcpy(P->dbuf, blob.data.data(), P->dbytes, hipMemcpyHostToDevice) != hipSuccess) {
      destroy_plan(P);
      return set_error(FSIMG_ERR_HIP, "batch descriptor upload failed");
    }
  }
  unsigned char *base = static_cast<unsigned char *>(P->dbuf);
  P->dlev = reinterpret_cast<DLev *>(base + lev_off);
  P->dkry = reinterpret_cast<DKry *>(base + P->kry_off);
  P->active = reinterpret_cast<int *>(base + act_off);
  P->kcnt = reinterpret_cast<int *>(base + k_off);
  P->flags = reinterpret_cast<int *>(base + fl_off);
  P->cyc = reinterpret_cast<int *>(base + cyc_off);
  P->cnt = reinterpret_cast<int *>(base + cnt_off);
  P->hs = reinterpret_cast<double *>(base + hs_off);
  P->gv = reinterpret_cast<DGiv *>(base + gv_off);
  for (int l = 0; l < Lmax; ++l) {
    P->ws_spmv.push_back(resolve(base, r_spmv[l]));
    P->ws_patch.push_back(resolve(base, r_patch[l]));
    P->ws_patch2.push_back(resolve(base, r_patch2[l]));
    P->ws_gather.push_back(resolve(base, r_gather[l]));
    P->ws_restrict.push_back(resolve(base, r_restrict[l]));
    P->ws_prolong.push_back(resolve(base, r_prolong[l]));
    P->ws_cn.push_back(resolve(base, r_cn[l]));
    P->ws_cf.push_back(resolve(base, r_cf[l]));
  }
  if (P->tails) {
    for (int l = 0; l < Lmax; ++l) {
      P->vs_spmv.push_back(resolve(base, v_spmv[l]));
      P->vs_patch.push_back(resolve(base, v_patch[l]));
      P->vs_patch2.push_back(resolve(base, v_patch2[l]));
      P->vs_gather.push_back(resolve(base, v_gather[l]));
      P->vs_restrict.push_back(resolve(base, v_restrict[l]));
      P->vs_prolong.push_back(resolve(base, v_prolong[l]));
    }
  } else {
    P->vs_spmv = P->ws_spmv;
    P->vs_patch = P->ws_patch;
    P->vs_patch2 = P->ws_patch2;
    P->vs_gather = P->ws_gather;
    P->vs_restrict = P->ws_restrict;
    P->vs_prolong = P->ws_prolong;
  }
  P->tfrom = reinterpret_cast<const int32_t *>(base + tfrom_off);
  P->tail_inst.assign(Lmax, nullptr);
  for (int l = 0; l < Lmax; ++l)
    if (P->tail_n[l] > 0) P->tail_inst[l] = reinterpret_cast<const int32_t *>(base + tail_off[l]);
  P->ws_row0 = resolve(base, r_row0);
  P->ws_vec0 = resolve(base, r_vec0);
  P->ws_kry = resolve(base, r_kry);
  P->ws_inst = resolve(base, r_ins);
  if (P->fixed) {
    P->ring_host = P->ring_one;
    P->int_host = P->int_one;
    P->gv_host = &P->gv_one;
    *out = P;
    return FSIMG_OK;
  }
  bool ev_ok = true;
  for (hipEvent_t &e : P->ev) ev_ok = ev_ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  if (!ev_ok ||
      hipHostMalloc((void **)&P->ring_host, (size_t)kMaxVec * n * sizeof(int), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void **)&P->int_host, (size_t)2 * n * sizeof(int), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void **)&P->gv_host, (size_t)n * sizeof(DGiv), hipHostMallocDefault) != hipSuccess) {
    destroy_plan(P);
    return set_error(FSIMG_ERR_HIP, "event or pinned host staging creation failed");
  }
  *out = P;
  return FSIMG_OK;
}

// zj >= 0: an FGMRES iteration's V-cycle; when every instance smooths the
// finest level, its last gather also writes z_zj (returns true; else the
// caller copies x to z_zj)
template <typename T>
bool vcycle_batch(BatchPlan &P, const fsimg_opts &o, hipStream_t s, bool prof, int zj = -1) {
  const int n = P.n;
  const T omega = (T)o.omega;
  const int *act = P.active;
  // profiling times the finest level's level-wide kernels: no small-level kernel then
  const bool tail = P.tails && !prof;
  const std::vector<WorkSet> &Wsp = tail ? P.vs_spmv : P.ws_spmv, &Wpa = tail ? P.vs_patch : P.ws_patch,
                             &Wpa2 = tail ? P.vs_patch2 : P.ws_patch2,
                             &Wga = tail ? P.vs_gather : P.ws_gather,
                             &Wre = tail ? P.vs_restrict : P.ws_restrict,
                             &Wpr = tail ? P.vs_prolong : P.ws_prolong;
  const bool zf = zj >= 0 && !tail && P.zfuse && o.nu_post > 0;
  for (int l = 0; l < P.Lmax; ++l) {
    const DLev *L = P.dlev + (size_t)l * n;
    if (Wpa[l].nset > 0 || Wpa2[l].nset > 0 || Wsp[l].nset > 0) {
      const bool p0 = prof && l == 0;
      if (o.nu_pre == 0) launch_b_fill_x<T>(L, act, Wga[l], s);
      for (int k = 0; k < o.nu_pre; ++k) {
        if (k > 0) {
          hipEvent_t a = p0 ? P.ts.next() : nullptr;
          hipEvent_t b2 = p0 ? P.ts.next() : nullptr;
          if (a) (void)hipEventRecord(a, s);
          launch_b_spmv<T>(P.b, BS_VCYCLE, P.rpw[l], L, P.dkry, act, Wsp[l], 0, s);
          if (b2) (void)hipEventRecord(b2, s);
        }
        hipEvent_t v0 = p0 ? P.tv.next() : nullptr;
        hipEvent_t v1 = p0 ? P.tv.next() : nullptr;
        launch_b_vanka_blocks<T>(P.np2, P.b, P.nl2, P.npc2, P.ppw2[l], k == 0, L, act, Wpa2[l], s);
        launch_b_vanka<T>(P.np, P.b, P.nl, P.npc, P.ppw[l], omega, k == 0, k == 0, L, act, Wpa[l],
                          Wga[l], s, v0, v1);
      }
      hipEvent_t a = p0 ? P.ts.next() : nullptr;
      hipEvent_t b2 = p0 ? P.ts.next() : nullptr;
      if (a) (void)hipEventRecord(a, s);
      launch_b_spmv<T>(P.b, BS_VCYCLE, P.rpw[l], L, P.dkry, act, Wsp[l], 0, s);
      if (b2) (void)hipEventRecord(b2, s);
      hipEvent_t r0 = p0 ? P.tr.next() : nullptr;
      hipEvent_t r1 = p0 ? P.tr.next() : nullptr;
      if (r0) (void)hipEventRecord(r0, s);
      launch_b_restrict<T>(P.b, P.dim, L, L + n, act, Wre[l], s);
      if (r1) (void)hipEventRecord(r1, s);
    }
    const bool tl = tail && P.tail_n[l] > 0;
    if (tl)
      launch_b_tail<T>(P.b, P.dim, P.dlev, n, act, P.tail_inst[l], P.tail_n[l], P.tfrom, l, false, P.np,
                       P.npc, P.nl, P.np2, P.npc2, P.nl2, omega, o.nu_pre, o.nu_post, s);
    if (P.ws_cn[l].nset > 0) launch_b_coarse<T>(L, act, P.ws_cn[l], P.ws_cf[l], s);
    if (tl)
      launch_b_tail<T>(P.b, P.dim, P.dlev, n, act, P.tail_inst[l], P.tail_n[l], P.tfrom, l, true, P.np,
                       P.npc, P.nl, P.np2, P.npc2, P.nl2, omega, o.nu_pre, o.nu_post, s);
  }
  for (int l = P.Lmax - 2; l >= 0; --l) {
    if (Wpr[l].nset == 0) continue;
    const DLev *L = P.dlev + (size_t)l * n;
    const bool p0 = prof && l == 0;
    hipEvent_t q0 = p0 ? P.tp.next() : nullptr;
    hipEvent_t q1 = p0 ? P.tp.next() : nullptr;
    if (q0) (void)hipEventRecord(q0, s);
    launch_b_prolong<T>(P.b, P.dim, L, L + n, act, Wpr[l], s);
    if (q1) (void)hipEventRecord(q1, s);
    for (int k = 0; k < o.nu_post; ++k) {
      hipEvent_t a = p0 ? P.ts.next() : nullptr;
      hipEvent_t b2 = p0 ? P.ts.next() : nullptr;
      if (a) (void)hipEventRecord(a, s);
      launch_b_spmv<T>(P.b, BS_VCYCLE, P.rpw[l], L, P.dkry, act, Wsp[l], 0, s);
      if (b2) (void)hipEventRecord(b2, s);
      hipEvent_t v0 = p0 ? P.tv.next() : nullptr;
      hipEvent_t v1 = p0 ? P.tv.next() : nullptr;
      launch_b_vanka_blocks<T>(P.np2, P.b, P.nl2, P.npc2, P.ppw2[l], false, L, act, Wpa2[l], s);
      const bool zl = zf && l == 0 && k == o.nu_post - 1;
      launch_b_vanka<T>(P.np, P.b, P.nl, P.npc, P.ppw[l], omega, false, false, L, act, Wpa[l], Wga[l],
                        s, v0, v1, zl ? P.dkry : nullptr, zl ? zj : -1);
    }
  }
  return zf;
}

// the launches of FGMRES iteration j for every active instance: z_j = M^-1 v_j
// (V-cycle in the plan's precision), w = A z_j, two Gram-Schmidt passes, the
// norm of w and v_{j+1} = w / ||w|| (Hessenberg column left in P.hs), then
// the device-side Givens update and stop test, and the copy of the active
// flags to the host ring (slot j)
void issue_iteration(BatchPlan &P, const fsimg_opts &o, int j, hipStream_t s, bool prof) {
  // v_j is already in the finest level's r (written with v_j itself)
  if (P.mixed) {
    if (!vcycle_batch<float>(P, o, s, prof, j))
      launch_b_copy_out<float>(P.dlev, P.dkry, P.active, P.ws_vec0, j, s);
  } else {
    if (!vcycle_batch<double>(P, o, s, prof, j))
      launch_b_copy_out<double>(P.dlev, P.dkry, P.active, P.ws_vec0, j, s);
  }
  launch_b_spmv<double>(P.b, BS_AZ, P.rpw0, P.dlev, P.dkry, P.active, P.ws_row0, j, s);
  // classical Gram-Schmidt, two passes; the w.w pass ends with the Givens step
  launch_b_multidot(P.dkry, P.active, P.ws_kry, j + 1, false, P.hs, kOffH1, P.cnt, s);
  launch_b_axpy_red(P.dkry, P.active, P.ws_kry, j + 1, false, P.hs, kOffH1, kOffH2, P.cnt, nullptr, j, s);
  launch_b_axpy_red(P.dkry, P.active, P.ws_kry, j + 1, true, P.hs, kOffH2, kOffSS, P.cnt, P.gv, j, s);
  if (P.mixed)
    launch_b_scale<float>(P.dkry, P.active, P.ws_vec0, P.hs, j + 1, P.dlev, s);
  else
    launch_b_scale<double>(P.dkry, P.active, P.ws_vec0, P.hs, j + 1, P.dlev, s);
  (void)hipMemcpyAsync(P.ring_host + (size_t)j * P.n, P.active, P.n * sizeof(int), hipMemcpyDeviceToHost,
                       s);
}

bool same_solver_opts(const fsimg_opts &a, const fsimg_opts &b) {
  return a.omega == b.omega && a.nu_pre == b.nu_pre && a.nu_post == b.nu_post &&
         a.precision == b.precision && a.restart == b.restart;
}

// the executable graph of iteration j, captured on the plan's own stream the
// first time it is needed (kernel and copy nodes only; the instances' active
// flags and control states are read from device memory, so one graph serves
// every iteration j of every later solve of this batch composition)
hipError_t iteration_graph(BatchPlan &P, const fsimg_opts &o, int j) {
  if (!P.iter_graph.empty() && !same_solver_opts(P.graph_opts, o)) {
    for (hipGraphExec_t g : P.iter_graph)
      if (g) (void)hipGraphExecDestroy(g);
    P.iter_graph.clear();
  }
  if ((int)P.iter_graph.size() < o.restart) P.iter_graph.resize(o.restart, nullptr);
  P.graph_opts = o;
  if (P.iter_graph[j]) return hipSuccess;
  hipError_t e = hipSuccess;
  if (!P.cap) e = hipStreamCreateWithFlags(&P.cap, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipStreamBeginCapture(P.cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  issue_iteration(P, o, j, P.cap, false);
  hipError_t e2 = hipGetLastError();
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(P.cap, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&P.iter_graph[j], g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  return e;
}



// Algorithmic device-memory bytes (every entry a kernel must touch, once)
// of the solve's kernels: level l's residual SpMV, Vanka patch kernel +
// gather, restriction / prolongation; w = word bytes of the V-cycle.
double spmv_bytes_of(const DevLevel &L, double w) {
  return (double)L.nnzb * (L.b * L.b * w + 4) + 4.0 * (L.nrows + 1) + 3.0 * L.n * w + (double)L.n;
}
double smooth_bytes_of(const DevLevel &L, double w) {
  const int npc = w == 4 ? L.npc32 : L.npc64;
  const int npc2 = w == 4 ? L.blk.npc32 : L.blk.npc64;
  const double patch = (double)L.npatch * (L.np * (double)npc * w + 2.0 * L.np * w + L.nl * 4.0) +
                       (double)L.blk.npatch * (L.blk.np * (double)npc2 * w + 2.0 * L.blk.np * w + L.blk.nl * 4.0);
  const double slots = (double)L.npatch * L.nl + (double)L.blk.npatch * L.blk.nl;
  const double gather = slots * L.b * w + 4.0 * (L.nrows + 1) + 4.0 * slots + 3.0 * L.n * w + (double)L.n;
  return patch + gather;
}
double vcycle_bytes_of(const fsimg_hier *h) {
  const double w = h->opts.precision == FSIMG_MIXED ? 4.0 : 8.0;
  const int L = (int)h->lev.size(), nu1 = h->opts.nu_pre, nu2 = h->opts.nu_post;
  double t = 0.0;
  for (int l = 0; l + 1 < L; ++l) {
    const DevLevel &F = h->lev[l], &C = h->lev[l + 1];
    const int nres = (nu1 > 0 ? nu1 - 1 : 0) + 1 + nu2;
    t += (nu1 + nu2) * smooth_bytes_of(F, w) + nres * spmv_bytes_of(F, w);
    t += (double)(F.n + C.n) * w + C.n;            // restriction
    t += (double)(2 * F.n + C.n) * w + F.n;        // prolongation
  }
  const DevLevel &C = h->lev.back();
  t += (double)C.nfree * C.nfree * 8.0 + 2.0 * C.n * 8.0 + (w == 4 ? 2.0 * C.n * (4 + 8) : 0.0);
  if (w == 4) t += 2.0 * h->lev[0].n * (8 + 4);    // FP64 <-> FP32 copies of v_j and z_j
  return t;
}
// one FGMRES iteration j: V-cycle, A z_j (FP64), two Gram-Schmidt passes,
// the norm and the scaling of v_{j+1}
double iteration_bytes_of(const fsimg_hier *h, int j) {
  const DevLevel &F = h->lev[0];
  return vcycle_bytes_of(h) + spmv_bytes_of(F, 8.0) + (3.0 * (j + 1) + 8.0) * F.n * 8.0;
}
// the end of a restart cycle with k directions: x += Z y, true residual, norm
double restart_bytes_of(const fsimg_hier *h, int k) {
  const DevLevel &F = h->lev[0];
  return (k + 2.0) * F.n * 8.0 + spmv_bytes_of(F, 8.0) + F.n * 8.0;
}

// the cached descriptor tables of this batch composition (built on first
// use), moved to the front of the context's LRU list
fsimg_status acquire_plan(fsimg_ctx *ctx, int n, fsimg_hier *const *hs, BatchPlan **out) {
  BatchPlan *P = nullptr;
  for (size_t c = 0; c < ctx->plans.size() && !P; ++c) {
    BatchPlan *q = ctx->plans[c];
    bool same = (int)q->key.size() == n;
    for (int i = 0; same && i < n; ++i) same = q->key[i] == hs[i]->uid;
    if (same) {
      P = q;
      ctx->plans.erase(ctx->plans.begin() + (long)c);
    }
  }
  if (!P) {
    while (ctx->plans.size() >= kPlanCache) {  // least recently used first
      destroy_plan(ctx->plans.back());
      ctx->plans.pop_back();
    }
    fsimg_status st = build_plan(ctx, n, hs, &P);
    if (st != FSIMG_OK) return st;
  }
  ctx->plans.insert(ctx->plans.begin(), P);  // most recent first
  *out = P;
  return FSIMG_OK;
}

}  // namespace

namespace {
fsimg_status run_batch(BatchPlan *P, int n, fsimg_hier *const *hs, const double *const *b,
                       double *const *x, fsimg_stats *stats, hipStream_t s, bool use_graph, bool prof);
fsimg_status check_batch(fsimg_ctx *ctx, int n, fsimg_hier *const *hs, const double *const *b,
                         double *const *x);
}  // namespace

fsimg_status solve_batch(fsimg_ctx *ctx, int n, fsimg_hier *const *hs, const double *const *b,
                         double *const *x, fsimg_stats *stats, hipStream_t s) {
  {
    const fsimg_status st = check_batch(ctx, n, hs, b, x);
    if (st != FSIMG_OK) return st;
  }
  BatchPlan *P = nullptr;
  {
    fsimg_status st = acquire_plan(ctx, n, hs, &P);
    if (st != FSIMG_OK) return st;
  }
  const bool prof = hs[0]->opts.profile != 0;
  return run_batch(P, n, hs, b, x, stats, s, hs[0]->opts.graphs != 0 && !prof, prof);
}

namespace {
fsimg_status check_batch(fsimg_ctx *ctx, int n, fsimg_hier *const *hs, const double *const *b,
                         double *const *x) {
  if (n < 1 || !hs || !b || !x) return set_error(FSIMG_ERR_ARG, "empty batch or null arrays");
  const fsimg_opts &o = hs[0]->opts;
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || !b[i] || !x[i]) return set_error(FSIMG_ERR_ARG, "null hierarchy or vector in batch");
    if (hs[i]->ctx != ctx) return set_error(FSIMG_ERR_ARG, "batch hierarchies must share one context");
    if (!hs[i]->factored) return set_error(FSIMG_ERR_STATE, "fsimg_factor must run before the solve");
    const fsimg_opts &q = hs[i]->opts;
    if (q.precision != o.precision || hs[i]->lev[0].b != hs[0]->lev[0].b ||
        hs[i]->lev[0].dim != hs[0]->lev[0].dim || q.omega != o.omega || q.nu_pre != o.nu_pre ||
        q.nu_post != o.nu_post || q.restart != o.restart || q.rtol != o.rtol ||
        q.max_iter != o.max_iter)
      return set_error(FSIMG_ERR_ARG, "batch hierarchies must share precision, block size, "
                                      "dimension and solver options");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return set_error(FSIMG_ERR_ARG, "a hierarchy appears twice in a batch");
  }
  return FSIMG_OK;
}

// FGMRES(m) + V-cycle of the n instances of plan P (eager launches or one
// graph per iteration).  The Givens update, the stop test and the
// least-squares solve run on the device (kb_kry_*), so the host never waits
// inside a restart cycle for the GPU: it keeps up to `lookahead` iterations
// in flight and reads each iteration's active flags (copied into a pinned
// ring) only to stop launching once every instance has stopped; with
// lookahead 2 the GPU runs iteration j + 1 while the host reads j's flags.
// The host does not speculate past an iteration that every active instance
// expects to finish on (the device's flag 2), so an iteration with no active
// instance (its kernels return at once) runs only after a wrong guess.  The host reads the
// control state once per restart cycle (continue flags and directions) and
// the counters once at the end.
fsimg_status run_batch(BatchPlan *P, int n, fsimg_hier *const *hs, const double *const *b,
                       double *const *x, fsimg_stats *stats, hipStream_t s, bool use_graph, bool prof) {
  const fsimg_opts &o = hs[0]->opts;
  const auto t0 = std::chrono::steady_clock::now();
  P->tv.begin_solve();
  P->ts.begin_solve();
  P->tr.begin_solve();
  P->tp.begin_solve();
  const int m = o.restart;
  // the no-allocation plan stages through pageable host arrays and has no
  // events: one iteration at a time, waits on the stream
  const int depth = P->fixed ? 1 : std::max(1, std::min(o.krylov_lookahead, 2));
  for (int i = 0; i < n; ++i) {
    fsimg_hier *h = hs[i];
    DKry &K = P->hkry[i];
    K.V = h->V; K.Z = h->Z; K.w = h->w; K.partial = h->partial;
    K.b = b[i]; K.x = x[i]; K.n = h->lev[0].n; K.nblk = krylov_blocks(K.n); K.pad = 0;
  }
  int *cyc_h = P->int_host, *k_h = P->int_host + n;
#define FSIMG_BHIP(expr)                                                                        \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return set_error(FSIMG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)
  // the continue flags and direction counts of a finished cycle
  auto read_cycle = [&]() {
    hipError_t e = hipMemcpyAsync(cyc_h, P->cyc, n * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(k_h, P->kcnt, n * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
  };
  FSIMG_BHIP(hipMemcpyAsync(P->dkry, P->hkry.data(), n * sizeof(DKry), hipMemcpyHostToDevice, s));
  std::vector<double> bytes(n, 0.0);
  launch_kry_reset(P->active, P->flags, P->cnt, n, s);
  launch_b_spmv<double>(P->b, BS_RESID, P->rpw0, P->dlev, P->dkry, P->active, P->ws_row0, 0, s);
  launch_b_nonfinite(P->dkry, P->active, P->ws_vec0, P->flags, s);
  launch_b_multidot(P->dkry, P->active, P->ws_kry, 1, true, P->hs, kOffSS, P->cnt, s);
  launch_kry_start(P->gv, P->hs, P->flags, P->active, P->cyc, n, o.rtol, o.max_iter, s);
  for (int i = 0; i < n; ++i) k_h[i] = 0;
  FSIMG_BHIP(hipMemcpyAsync(cyc_h, P->cyc, n * sizeof(int), hipMemcpyDeviceToHost, s));
  FSIMG_BHIP(hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i)
    bytes[i] = spmv_bytes_of(hs[i]->lev[0], 8.0) + 2.0 * hs[i]->lev[0].n * 8.0;  // r_0, its checks
  while (true) {
    bool any = false;
    for (int i = 0; i < n; ++i) any |= cyc_h[i] != 0;
    if (!any) break;
    if (P->mixed)  // v_0 = r / ||r||
      launch_b_scale<float>(P->dkry, P->active, P->ws_vec0, P->hs, 0, P->dlev, s);
    else
      launch_b_scale<double>(P->dkry, P->active, P->ws_vec0, P->hs, 0, P->dlev, s);
    // speculate: launch the next iteration before the previous one's flags
    // are read, unless every active instance expects to stop (active = 2)
    // at the iteration in flight, which would leave the speculative one empty
    int launched = 0, checked = 0;
    bool live = true, speculate = true;
    while (live && (launched < m || checked < launched)) {
      if (launched < m && launched - checked < depth && (launched == checked || speculate)) {
        const int j = launched++;
        if (use_graph) {
          FSIMG_BHIP(iteration_graph(*P, o, j));
          FSIMG_BHIP(hipGraphLaunch(P->iter_graph[j], s));
        } else {
          issue_iteration(*P, o, j, s, prof);
        }
        if (!P->fixed) FSIMG_BHIP(hipEventRecord(P->ev[j], s));
        continue;
      }
      FSIMG_BHIP(P->fixed ? hipStreamSynchronize(s) : hipEventSynchronize(P->ev[checked]));
      const int *fl = P->ring_host + (size_t)checked * n;
      live = false;
      speculate = false;
      for (int i = 0; i < n; ++i) {
        live |= fl[i] != 0;
        speculate |= fl[i] == 1;
      }
      ++checked;
    }
    // x += Z y for every instance of this cycle, then the true residual
    launch_kry_ysolve(P->gv, P->hs, P->active, P->kcnt, n, s);
    launch_b_combine(P->dkry, P->active, P->ws_vec0, P->hs, P->kcnt, launched, s);
    launch_b_spmv<double>(P->b, BS_RESID, P->rpw0, P->dlev, P->dkry, P->active, P->ws_row0, 0, s);
    launch_b_multidot(P->dkry, P->active, P->ws_kry, 1, true, P->hs, kOffSS, P->cnt, s);
    launch_kry_restart(P->gv, P->hs, P->active, P->cyc, n, s);
    FSIMG_BHIP(read_cycle());
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < k_h[i]; ++j) bytes[i] += iteration_bytes_of(hs[i], j);
      if (k_h[i] > 0) bytes[i] += restart_bytes_of(hs[i], k_h[i]);
    }
  }
  FSIMG_BHIP(hipMemcpyAsync(P->gv_host, P->gv, n * sizeof(DGiv), hipMemcpyDeviceToHost, s));
  FSIMG_BHIP(hipStreamSynchronize(s));
  FSIMG_BHIP(hipGetLastError());
  double vms = 0.0, sms = 0.0, rms = 0.0, pms = 0.0;
  int vn = 0, sn = 0, rn = 0, pn = 0;
  if (prof) {
    FSIMG_BHIP(hipStreamSynchronize(s));
    vms = P->tv.total_ms(&vn);
    sms = P->ts.total_ms(&sn);
    rms = P->tr.total_ms(&rn);
    pms = P->tp.total_ms(&pn);
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  fsimg_status ret = FSIMG_OK;
  for (int i = 0; i < n; ++i) {
    const DGiv &q = P->gv_host[i];
    if (stats) {
      fsimg_stats &st = stats[i];
      st = fsimg_stats{};
      st.status = q.status;
      st.iters = q.it;
      st.restarts = q.restarts;
      st.rel_res = q.beta0 > 0.0 ? q.rnorm / q.beta0 : 0.0;
      st.solve_ms = ms;
      st.vanka_ms = vms; st.vanka_launches = vn;
      st.spmv_ms = sms; st.spmv_launches = sn;
      st.restrict_ms = rms; st.restrict_launches = rn;
      st.prolong_ms = pms; st.prolong_launches = pn;
      st.setup_ms = hs[i]->setup_ms;
      st.factor_ms = hs[i]->factor_ms;
      st.bytes_moved = bytes[i];
      st.nhist = std::min(q.nhist, FSIMG_HIST);
      for (int t = 0; t < st.nhist; ++t) st.res_hist[t] = q.hist[t];
    }
    if (ret == FSIMG_OK && q.status != FSIMG_OK) ret = (fsimg_status)q.status;
  }
#undef FSIMG_BHIP
  if (ret == FSIMG_ERR_NOCONV) return set_error(ret, "an instance reached max_iter without converging");
  if (ret == FSIMG_ERR_NONFINITE) return set_error(ret, "non-finite residual in an instance");
  return ret;
}
}  // namespace


// ------------------------------------------------- one hierarchy, one step
namespace {
template <typename T> struct HV;
template <> struct HV<double> {
  static double *r(DevLevel &L) { return L.r64; }
  static double *x(DevLevel &L) { return L.x64; }
  static double *d(DevLevel &L) { return L.d64; }
};
template <> struct HV<float> {
  static float *r(DevLevel &L) { return L.r32; }
  static float *x(DevLevel &L) { return L.x32; }
  static float *d(DevLevel &L) { return L.d32; }
};

template <typename T>
fsimg_status single_step_t(fsimg_hier *h, int op, int l, const void *a, const void *b, void *out,
                           hipStream_t s) {
  BatchPlan *P = nullptr;
  fsimg_status st = acquire_plan(h->ctx, 1, &h, &P);
  if (st != FSIMG_OK) return st;
  launch_b_activate(P->active, 1, s);
  const fsimg_opts &o = h->opts;
  const DLev *dl = P->dlev + l;  // one instance: one descriptor per level
  DevLevel &F = h->lev[l];
  hipError_t e = hipSuccess;
  auto cp = [&](void *dst, const void *src, int64_t n) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, (size_t)n * sizeof(T), hipMemcpyDeviceToDevice, s);
  };
  switch (op) {
    case ONE_RESIDUAL:  // out = a - A_l b
      cp(HV<T>::r(F), a, F.n);
      cp(HV<T>::x(F), b, F.n);
      launch_b_spmv<T>(P->b, BS_VCYCLE, P->rpw[l], dl, P->dkry, P->active, P->ws_spmv[l], 0, s);
      cp(out, HV<T>::d(F), F.n);
      break;
    case ONE_VANKA:  // out += Vanka correction of the residual a - A_l out
      cp(HV<T>::r(F), a, F.n);
      cp(HV<T>::x(F), out, F.n);
      launch_b_spmv<T>(P->b, BS_VCYCLE, P->rpw[l], dl, P->dkry, P->active, P->ws_spmv[l], 0, s);
      launch_b_vanka_blocks<T>(P->np2, P->b, P->nl2, P->npc2, P->ppw2[l], false, dl, P->active,
                               P->ws_patch2[l], s);
      launch_b_vanka<T>(P->np, P->b, P->nl, P->npc, P->ppw[l], (T)o.omega, false, false, dl, P->active,
                        P->ws_patch[l], P->ws_gather[l], s, nullptr, nullptr);
      cp(out, HV<T>::x(F), F.n);
      break;
    case ONE_RESTRICT:  // out = R a (level l -> l + 1)
      cp(HV<T>::d(F), a, F.n);
      launch_b_restrict<T>(P->b, P->dim, dl, dl + 1, P->active, P->ws_restrict[l], s);
      cp(out, HV<T>::r(h->lev[l + 1]), h->lev[l + 1].n);
      break;
    case ONE_PROLONG:  // out += P a (level l + 1 -> l)
      cp(HV<T>::x(h->lev[l + 1]), a, h->lev[l + 1].n);
      cp(HV<T>::x(F), out, F.n);
      launch_b_prolong<T>(P->b, P->dim, dl, dl + 1, P->active, P->ws_prolong[l], s);
      cp(out, HV<T>::x(F), F.n);
      break;
    case ONE_COARSE:  // out = A_{L-1}^{-1} a (FP64 hierarchies)
      cp(HV<T>::r(F), a, F.n);
      launch_b_coarse<T>(dl, P->active, P->ws_cn[l], P->ws_cf[l], s);
      cp(out, HV<T>::x(F), F.n);
      break;
    case ONE_VCYCLE:  // out = V-cycle(a) on level 0
      cp(HV<T>::r(F), a, F.n);
      (void)vcycle_batch<T>(*P, o, s, false);
      cp(out, HV<T>::x(F), F.n);
      break;
    default:
      return set_error(FSIMG_ERR_ARG, "unknown single-step operation");
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return set_error(FSIMG_ERR_HIP, std::string("single step: ") + hipGetErrorString(e));
  return FSIMG_OK;
}
}  // namespace

fsimg_status single_step(fsimg_hier *h, int op, int level, const void *a, const void *b, void *out,
                         hipStream_t s) {
  if (h->opts.precision == FSIMG_MIXED) return single_step_t<float>(h, op, level, a, b, out, s);
  return single_step_t<double>(h, op, level, a, b, out, s);
}


// ------------------------------------------ solve without any allocation
// The per-solve tables of one instance (level descriptors, work lists,
// Krylov descriptor, flags, Hessenberg column: about 30 KB for five levels)
// live in this fixed array; every GPU the library runs on holds its own copy
// until the process ends.  Host code never uses the array's name as an
// address: the device address of each GPU's copy is looked up once per
// device (noalloc_init, called when a context is created on it).
constexpr size_t kScratchBytes = size_t(64) << 10;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

fsimg_status noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return set_error(FSIMG_ERR_ARG, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return FSIMG_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));  // `device` is current
  if (e != hipSuccess || !ptr)
    return set_error(FSIMG_ERR_HIP, std::string("scratch array lookup: ") + hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return FSIMG_OK;
}

size_t noalloc_scratch_bytes() { return kScratchBytes; }

fsimg_status solve_noalloc(fsimg_hier *h, const double *b, double *x, fsimg_stats *stats,
                           hipStream_t s) {
  if (!h || !b || !x) return set_error(FSIMG_ERR_ARG, "null argument");
  if (h->opts.vanka_schedule != FSIMG_VANKA_GATHER || h->opts.smoother != FSIMG_SMOOTHER_VANKA)
    return set_error(FSIMG_ERR_ARG, "the no-allocation solve needs the GATHER schedule and the Vanka "
                                    "smoother");
  {
    const fsimg_status st = check_batch(h->ctx, 1, &h, &b, &x);
    if (st != FSIMG_OK) return st;
  }
  const int dev = h->ctx->device;
  void *ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ptr = (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
  }
  if (!ptr) return set_error(FSIMG_ERR_STATE, "no scratch array address for this device");
  BatchPlan *P = nullptr;
  {
    const fsimg_status st = build_plan(h->ctx, 1, &h, &P, ptr, kScratchBytes, s);
    if (st != FSIMG_OK) return st;
  }
  const fsimg_status st = run_batch(P, 1, &h, &b, &x, stats, s, false, false);
  destroy_plan(P);  // host side only: the tables stay in the scratch array
  return st;
}

}  // namespace fsimg
