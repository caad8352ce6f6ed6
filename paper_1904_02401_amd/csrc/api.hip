// Host runtime of the fsimg library: contexts and HBM accounting, hierarchy
// setup (patches, colouring, transfer data), factorisation driver, V-cycle,
// flexible GMRES, and the extern "C" entry points declared in fsimg.h.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "hier.h"

using namespace fsimg;

namespace {
thread_local std::string g_err;

fsimg_status fail(fsimg_status s, const std::string &msg) {
  g_err = msg;
  return s;
}
std::atomic<uint64_t> g_uid{1};
}  // namespace

fsimg_status fsimg::set_error(fsimg_status s, const std::string &msg) { return fail(s, msg); }

#define FSIMG_HIP(expr)                                                                         \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return fail(FSIMG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)
#define FSIMG_TRY(expr)                     \
  do {                                      \
    fsimg_status st_ = (expr);              \
    if (st_ != FSIMG_OK) return st_;        \
  } while (0)

namespace {

// small device buffer offsets (doubles)
constexpr int kH1 = 0, kH2 = 32, kH = 64, kSS = 96, kY = 128;

template <typename T>
fsimg_status dalloc(fsimg_hier *h, T **p, size_t count) {
  *p = nullptr;
  const size_t bytes = count * sizeof(T);
  if (bytes == 0) return FSIMG_OK;
  if (h->ctx->budget && h->ctx->in_use + bytes > h->ctx->budget)
    return fail(FSIMG_ERR_BUDGET, "allocation of " + std::to_string(bytes) +
                                      " bytes exceeds the context's HBM budget");
  void *q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FSIMG_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  h->ctx->in_use += bytes;
  h->allocs.push_back({q, bytes});
  *p = static_cast<T *>(q);
  return FSIMG_OK;
}

inline int npc_for(int np, int elem_bytes) {
  const int g = 16 / elem_bytes;
  return (np + g - 1) / g * g;
}

// --------------------------------------------------------- validation
fsimg_status validate_levels(const fsimg_level_desc *d, int nlev) {
  if (!d || nlev < 1 || nlev > 16) return fail(FSIMG_ERR_ARG, "need 1..16 levels");
  for (int l = 0; l < nlev; ++l) {
    const fsimg_level_desc &L = d[l];
    const std::string at = "level " + std::to_string(l) + ": ";
    if (L.dim < 2 || L.dim > 3) return fail(FSIMG_ERR_ARG, at + "dim must be 2 or 3");
    if (L.block < 1 || L.block > 4) return fail(FSIMG_ERR_ARG, at + "block must be 1..4");
    if (L.block != d[0].block || L.dim != d[0].dim)
      return fail(FSIMG_ERR_ARG, at + "block and dim must agree on all levels");
    int64_t nr = 1;
    for (int a = 0; a < 3; ++a) {
      const int c = L.cells[a];
      if (a < L.dim && c < 1) return fail(FSIMG_ERR_ARG, at + "cells must be >= 1");
      if (a >= L.dim && c != 1) return fail(FSIMG_ERR_ARG, at + "unused axes must have 1 cell");
      if (a < L.dim) nr *= 2 * (int64_t)c + 1;
      if (l > 0 && a < L.dim && d[l - 1].cells[a] != 2 * c)
        return fail(FSIMG_ERR_ARG, at + "cells must halve from the finer level");
    }
    if (nr != L.nrows) return fail(FSIMG_ERR_ARG, at + "nrows != prod(2*cells+1)");
    if (L.nrows >= INT_MAX / 8 || L.nnzb >= INT_MAX)
      return fail(FSIMG_ERR_ARG, at + "too many rows / blocks for int32 structure");
    if (!L.rowptr || !L.colind || !L.vals || !L.dirichlet)
      return fail(FSIMG_ERR_ARG, at + "null array");
    if (L.rowptr[0] != 0 || L.rowptr[L.nrows] != L.nnzb)
      return fail(FSIMG_ERR_ARG, at + "rowptr must start at 0 and end at nnzb");
    for (int64_t r = 0; r < L.nrows; ++r) {
      const int32_t s = L.rowptr[r], e = L.rowptr[r + 1];
      if (e < s) return fail(FSIMG_ERR_ARG, at + "rowptr not monotone");
      bool diag = false;
      for (int32_t j = s; j < e; ++j) {
        const int32_t c = L.colind[j];
        if (c < 0 || c >= L.nrows) return fail(FSIMG_ERR_ARG, at + "colind out of range");
        if (j > s && c <= L.colind[j - 1])
          return fail(FSIMG_ERR_ARG, at + "colind not strictly increasing in a row");
        diag |= (c == r);
      }
      if (!diag) return fail(FSIMG_ERR_ARG, at + "missing diagonal block in row " + std::to_string(r));
    }
    if (l == nlev - 1) {
      const int64_t n = L.nrows * L.block;
      if (n > 20000) return fail(FSIMG_ERR_ARG, "coarsest level too large for the dense solve (n > 20000)");
    }
  }
  return FSIMG_OK;
}

// element patches of one level: active = some dof is not an identity row
struct PatchPlan {
  std::vector<int64_t> elem;           // active patches, final order
  std::vector<int64_t> colour_start;   // ranges of equal colour (schedule != GATHER)
  std::vector<int32_t> nodes;          // [npatch*nl]
  std::vector<int32_t> gptr, gidx;
  // block patches (second group): first element of each active block, nodes
  int blk_nl = 0;
  std::vector<int64_t> blk_first;
  std::vector<int32_t> blk_nodes;      // [nblk*blk_nl]
};

void element_nodes(const fsimg_level_desc &L, int64_t e, int32_t *out) {
  int ea[3] = {0, 0, 0};
  int64_t r = e;
  for (int a = 0; a < L.dim; ++a) { ea[a] = (int)(r % L.cells[a]); r /= L.cells[a]; }
  const int nn[3] = {2 * L.cells[0] + 1, 2 * L.cells[1] + 1, 2 * L.cells[2] + 1};
  const int nl = L.dim == 2 ? 9 : 27;
  for (int i = 0; i < nl; ++i) {
    const int la[3] = {i % 3, (i / 3) % 3, i / 9};
    int64_t g = 0, stride = 1;
    for (int a = 0; a < L.dim; ++a) { g += stride * (2 * ea[a] + la[a]); stride *= nn[a]; }
    out[i] = (int32_t)g;
  }
}

// nodes of the 2 x 2 (x 2) element block whose first element has coordinates
// lo: the 5^d nodes of its node box, lexicographic (x fastest)
void block_nodes(const fsimg_level_desc &L, const int lo[3], int32_t *out) {
  const int nn[3] = {2 * L.cells[0] + 1, 2 * L.cells[1] + 1, 2 * L.cells[2] + 1};
  const int nl = L.dim == 2 ? 25 : 125;
  for (int i = 0; i < nl; ++i) {
    const int la[3] = {i % 5, (i / 5) % 5, i / 25};
    int64_t g = 0, stride = 1;
    for (int a = 0; a < L.dim; ++a) { g += stride * (2 * lo[a] + la[a]); stride *= nn[a]; }
    out[i] = (int32_t)g;
  }
}

// node -> Y slots of the patches containing it, in patch order: element
// patches (slot p*nl + local node), then block patches (slot npatch*nl +
// q*nlb + local node)
void build_gather(const fsimg_level_desc &L, int nl, const std::vector<int32_t> &nodes, int64_t npatch,
                  std::vector<int32_t> &gptr, std::vector<int32_t> &gidx, int nlb = 0,
                  const std::vector<int32_t> *bnodes = nullptr) {
  const int64_t nblk = (bnodes && nlb) ? (int64_t)bnodes->size() / nlb : 0;
  gptr.assign(L.nrows + 1, 0);
  for (int64_t p = 0; p < npatch; ++p)
    for (int l = 0; l < nl; ++l) gptr[nodes[p * nl + l] + 1]++;
  for (int64_t q = 0; q < nblk; ++q)
    for (int l = 0; l < nlb; ++l) gptr[(*bnodes)[q * nlb + l] + 1]++;
  for (int64_t i = 0; i < L.nrows; ++i) gptr[i + 1] += gptr[i];
  gidx.assign(gptr[L.nrows], 0);
  std::vector<int32_t> fill(gptr.begin(), gptr.end() - 1);
  for (int64_t p = 0; p < npatch; ++p)
    for (int l = 0; l < nl; ++l) gidx[fill[nodes[p * nl + l]]++] = (int32_t)(p * nl + l);
  for (int64_t q = 0; q < nblk; ++q)
    for (int l = 0; l < nlb; ++l)
      gidx[fill[(*bnodes)[q * nlb + l]]++] = (int32_t)(npatch * nl + q * nlb + l);
}

fsimg_status plan_patches(const fsimg_level_desc &L, int schedule, const uint8_t *cell_class,
                          PatchPlan &P, int patches = FSIMG_PATCH_ELEMENT) {
  const int nl = L.dim == 2 ? 9 : 27;
  const int b = L.block;
  int64_t ncell = 1;
  for (int a = 0; a < L.dim; ++a) ncell *= L.cells[a];
  std::vector<char> covered(ncell, 0);
  if (patches == FSIMG_PATCH_BLOCK) {
    // 2 x 2 (x 2) blocks at even element coordinates; in 3D only all-solid ones
    const int nlb = L.dim == 2 ? 25 : 125;
    P.blk_nl = nlb;
    const int nb[3] = {L.cells[0] / 2, L.dim > 1 ? L.cells[1] / 2 : 1,
                       L.dim > 2 ? L.cells[2] / 2 : 1};
    std::vector<int32_t> bn(nlb);
    for (int k = 0; k < (L.dim > 2 ? nb[2] : 1); ++k)
      for (int j = 0; j < nb[1]; ++j)
        for (int i = 0; i < nb[0]; ++i) {
          const int lo[3] = {2 * i, 2 * j, 2 * k};
          int64_t mem[8];
          int nm = 0;
          for (int dz = 0; dz < (L.dim > 2 ? 2 : 1); ++dz)
            for (int dy = 0; dy < 2; ++dy)
              for (int dx = 0; dx < 2; ++dx)
                mem[nm++] = (lo[0] + dx) + (int64_t)L.cells[0] * ((lo[1] + dy) +
                                                                 (int64_t)L.cells[1] * (lo[2] + dz));
          bool take = true;
          if (L.dim == 3)
            for (int m = 0; m < nm; ++m) take = take && cell_class && cell_class[mem[m]] != 0;
          if (!take) continue;
          for (int m = 0; m < nm; ++m) covered[mem[m]] = 1;
          block_nodes(L, lo, bn.data());
          bool any = false;
          for (int l = 0; l < nlb && !any; ++l)
            for (int c = 0; c < b; ++c)
              if (!L.dirichlet[(int64_t)bn[l] * b + c]) { any = true; break; }
          if (!any) continue;
          P.blk_first.push_back(mem[0]);
          P.blk_nodes.insert(P.blk_nodes.end(), bn.begin(), bn.end());
        }
  }
  std::vector<int64_t> act;
  std::vector<int32_t> tmp(nl);
  for (int64_t e = 0; e < ncell; ++e) {
    if (covered[e]) continue;
    element_nodes(L, e, tmp.data());
    bool any = false;
    for (int l = 0; l < nl && !any; ++l)
      for (int c = 0; c < b; ++c)
        if (!L.dirichlet[(int64_t)tmp[l] * b + c]) { any = true; break; }
    if (any) act.push_back(e);
  }
  const int64_t np_ = (int64_t)act.size();
  std::vector<int> colour(np_, 0);
  int ncol = 1;
  if (schedule == FSIMG_VANKA_PARITY) {
    ncol = 1 << L.dim;
    for (int64_t i = 0; i < np_; ++i) {
      int64_t r = act[i];
      int c = 0;
      for (int a = 0; a < L.dim; ++a) { c |= (int)((r % L.cells[a]) & 1) << a; r /= L.cells[a]; }
      colour[i] = c;
    }
  } else if (schedule == FSIMG_VANKA_GREEDY) {
    // the paper's greedy colouring (Sec. 5.5.3): walk the patches; an
    // unlabelled, unblocked patch takes the current colour and blocks every
    // patch sharing a node with it; repeat with the next colour.  Patches of
    // different classes (fluid / solid) never share a colour.
    std::vector<int32_t> nodes(np_ * nl);
    for (int64_t i = 0; i < np_; ++i) element_nodes(L, act[i], &nodes[i * nl]);
    std::vector<int32_t> gp, gi;
    build_gather(L, nl, nodes, np_, gp, gi);
    std::fill(colour.begin(), colour.end(), -1);
    std::vector<int> classes;
    for (int64_t i = 0; i < np_; ++i) {
      const int c = cell_class ? cell_class[act[i]] : 0;
      if (std::find(classes.begin(), classes.end(), c) == classes.end()) classes.push_back(c);
    }
    std::sort(classes.begin(), classes.end());
    int next = 0;
    std::vector<char> blocked(np_);
    for (int cls : classes) {
      int64_t left = 0;
      for (int64_t i = 0; i < np_; ++i) left += ((cell_class ? cell_class[act[i]] : 0) == cls);
      while (left > 0) {
        std::fill(blocked.begin(), blocked.end(), 0);
        for (int64_t i = 0; i < np_; ++i) {
          if (colour[i] >= 0 || blocked[i] || (cell_class ? cell_class[act[i]] : 0) != cls) continue;
          colour[i] = next;
          --left;
          for (int l = 0; l < nl; ++l) {
            const int32_t nd = nodes[i * nl + l];
            for (int32_t e = gp[nd]; e < gp[nd + 1]; ++e) blocked[gi[e] / nl] = 1;
          }
        }
        ++next;
      }
    }
    ncol = next;
  }
  // order: by colour (stable), lexicographic inside a colour
  std::vector<int64_t> order(np_);
  for (int64_t i = 0; i < np_; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return colour[x] < colour[y]; });
  P.elem.resize(np_);
  P.nodes.resize(np_ * nl);
  P.colour_start.assign(1, 0);
  for (int64_t i = 0; i < np_; ++i) {
    P.elem[i] = act[order[i]];
    element_nodes(L, P.elem[i], &P.nodes[i * nl]);
    if (i > 0 && colour[order[i]] != colour[order[i - 1]]) P.colour_start.push_back(i);
  }
  P.colour_start.push_back(np_);
  if (schedule == FSIMG_VANKA_GATHER) P.colour_start = {0, np_};
  build_gather(L, nl, P.nodes, np_, P.gptr, P.gidx, P.blk_nl, &P.blk_nodes);
  // validator: patches of one colour never share a node
  if (schedule != FSIMG_VANKA_GATHER) {
    std::vector<int> pc(np_);
    for (size_t c = 0; c + 1 < P.colour_start.size(); ++c)
      for (int64_t i = P.colour_start[c]; i < P.colour_start[c + 1]; ++i) pc[i] = (int)c;
    for (int64_t nd = 0; nd < L.nrows; ++nd)
      for (int32_t e = P.gptr[nd]; e < P.gptr[nd + 1]; ++e)
        for (int32_t f = e + 1; f < P.gptr[nd + 1]; ++f)
          if (pc[P.gidx[e] / nl] == pc[P.gidx[f] / nl])
            return fail(FSIMG_ERR_ARG, "colouring invalid: two patches of one colour share node " +
                                           std::to_string(nd));
  }
  (void)ncol;
  return FSIMG_OK;
}

// geometric multiplicity: number of cells containing the node
double node_mult(const fsimg_level_desc &L, int64_t node) {
  double m = 1.0;
  int64_t r = node;
  for (int a = 0; a < L.dim; ++a) {
    const int nn = 2 * L.cells[a] + 1;
    const int g = (int)(r % nn);
    r /= nn;
    if ((g & 1) == 0 && g > 0 && g < nn - 1) m *= 2.0;
  }
  return m;
}

int64_t count_free(const fsimg_level_desc &L) {
  int64_t f = 0;
  for (int64_t i = 0; i < L.nrows * L.block; ++i) f += L.dirichlet[i] == 0;
  return f;
}

size_t level_bytes(const fsimg_level_desc &L, int64_t npatch, int64_t ngidx, bool coarse,
                   const fsimg_opts &o, int64_t nblk = 0) {
  const bool mixed = o.precision == FSIMG_MIXED;
  const int b = L.block, nl = L.dim == 2 ? 9 : 27, np = nl * b;
  const int64_t n = L.nrows * b;
  const size_t ts = mixed ? 4 : 8;
  size_t s = (size_t)(L.nrows + 1) * 4 + (size_t)L.nnzb * 4 + (size_t)L.nnzb * b * b * 8 + (size_t)n;
  if (mixed) s += (size_t)L.nnzb * b * b * 4;
  if (!coarse && o.smoother == FSIMG_SMOOTHER_ILU) {
    s += (size_t)npatch * nl * 4 + (size_t)(L.nrows + 1) * 4 + (size_t)ngidx * 4;
    s += (size_t)L.nrows * ts + (size_t)3 * n * ts;  // scale; r, x, d
    s += (size_t)L.nnzb * b * b * 8 + (size_t)L.nrows * b * b * 8;  // FP64 factors, U_ii^-1
    if (mixed) s += (size_t)L.nnzb * b * b * 4 + (size_t)L.nrows * b * b * 4;
    s += (size_t)3 * L.nrows * 4 + (size_t)n * ts;  // diagonal positions, schedules, work
  } else if (!coarse) {
    s += (size_t)npatch * nl * 4 + (size_t)(L.nrows + 1) * 4 + (size_t)ngidx * 4;
    s += (size_t)npatch * np * npc_for(np, (int)ts) * ts;
    s += (size_t)L.nrows * ts;                       // scale
    s += (size_t)3 * n * ts + (size_t)npatch * np * ts;  // r, x, d, Y
    if (nblk > 0) {  // block patches: nodes, inverses, corrections, factorisation scratch
      const int nlb = L.dim == 2 ? 25 : 125, npb = nlb * b;
      s += (size_t)nblk * nlb * 4 + (size_t)nblk * npb * npc_for(npb, (int)ts) * ts +
           (size_t)nblk * npb * ts;
      if (npb > 128 || nlb > 27)
        s += (size_t)nblk * npb * npb * 8 + (size_t)nblk * npb * (2 * kCoarseStage * 8 + 4 + 4) +
             (size_t)nblk * 8;
    }
  } else {
    const int64_t nf = count_free(L);
    s += (size_t)nf * nf * 8 + (size_t)(nf + n) * 4 + (size_t)2 * n * 8 + (size_t)2 * n * ts;
    if (nf > 0)  // Gauss-Jordan workspace
      s += (size_t)nf * nf * 8 + (size_t)2 * kCoarseStage * nf * 8 + (size_t)2 * nf * 4 +
           (size_t)kRedBlocks * 8;
  }
  return s;
}

size_t krylov_bytes(int64_t n0, int m) {
  return (size_t)(2 * m + 2) * n0 * 8 + (size_t)kRedBlocks * kMaxVec * 8 + 256 * 8 + 64;
}

// -------------------------------------------------------- V-cycle
template <typename T> struct Sel;
template <> struct Sel<double> {
  static double *r(DevLevel &L) { return L.r64; }
  static double *x(DevLevel &L) { return L.x64; }
  static double *d(DevLevel &L) { return L.d64; }
  static double *Y(DevLevel &L) { return L.Y64; }
  static const double *vals(const DevLevel &L) { return L.vals64; }
  static const double *inv(const DevLevel &L) { return L.inv64; }
  static int npc(const DevLevel &L) { return L.npc64; }
  static const double *scale(const DevLevel &L) { return L.scale64; }
  static const double *binv(const DevLevel &L) { return L.blk.inv64; }
  static int bnpc(const DevLevel &L) { return L.blk.npc64; }
};
template <> struct Sel<float> {
  static float *r(DevLevel &L) { return L.r32; }
  static float *x(DevLevel &L) { return L.x32; }
  static float *d(DevLevel &L) { return L.d32; }
  static float *Y(DevLevel &L) { return L.Y32; }
  static const float *vals(const DevLevel &L) { return L.vals32; }
  static const float *inv(const DevLevel &L) { return L.inv32; }
  static int npc(const DevLevel &L) { return L.npc32; }
  static const float *scale(const DevLevel &L) { return L.scale32; }
  static const float *binv(const DevLevel &L) { return L.blk.inv32; }
  static int bnpc(const DevLevel &L) { return L.blk.npc32; }
};

template <typename T>
void residual(fsimg_hier *h, int l, const T *b, const T *x, T *d, hipStream_t s) {
  DevLevel &L = h->lev[l];
  const bool prof = h->profiling && l == 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof) { e0 = h->ts.next(); e1 = h->ts.next(); if (e0) (void)hipEventRecord(e0, s); }
  launch_bsr_spmv<T>(L, Sel<T>::vals(L), x, b, d, true, s);
  if (prof && e1) (void)hipEventRecord(e1, s);
}

// one Vanka step with the residual d already computed: x (+)= omega W sum R^T A^-1 R d
template <typename T>
void vanka_apply(fsimg_hier *h, int l, const T *d, T *x, bool assign, hipStream_t s) {
  DevLevel &L = h->lev[l];
  const T omega = (T)h->opts.omega;
  const bool prof = h->profiling && l == 0;
  if (h->opts.vanka_schedule == FSIMG_VANKA_GATHER) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof) { e0 = h->tv.next(); e1 = h->tv.next(); if (e0) (void)hipEventRecord(e0, s); }
    launch_vanka_patch<T>(L, Sel<T>::inv(L), Sel<T>::npc(L), d, Sel<T>::Y(L), 0, L.npatch, false,
                          nullptr, nullptr, omega, s);
    if (prof && e1) (void)hipEventRecord(e1, s);
    if (L.blk.npatch > 0)
      launch_vanka_blocks<T>(L, Sel<T>::binv(L), Sel<T>::bnpc(L), d, Sel<T>::Y(L) + L.blk.yofs, s);
    launch_vanka_gather<T>(L, Sel<T>::Y(L), Sel<T>::scale(L), omega, assign, x, s);
  } else {
    if (assign) launch_fill<T>(x, L.n, T(0), s);
    for (size_t c = 0; c + 1 < L.colour_start.size(); ++c) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (prof) { e0 = h->tv.next(); e1 = h->tv.next(); if (e0) (void)hipEventRecord(e0, s); }
      launch_vanka_patch<T>(L, Sel<T>::inv(L), Sel<T>::npc(L), d, nullptr, L.colour_start[c],
                            L.colour_start[c + 1], true, x, Sel<T>::scale(L), omega, s);
      if (prof && e1) (void)hipEventRecord(e1, s);
    }
  }
}

template <typename T> struct IluSel;
template <> struct IluSel<double> {
  static const double *F(const DevLevel &L) { return L.ilu64; }
  static const double *dinv(const DevLevel &L) { return L.dinv64; }
  static double *work(DevLevel &L) { return L.iw64; }
};
template <> struct IluSel<float> {
  static const float *F(const DevLevel &L) { return L.ilu32; }
  static const float *dinv(const DevLevel &L) { return L.dinv32; }
  static float *work(DevLevel &L) { return L.iw32; }
};

// the ILU level sweeps of level l (reading the level's residual buffer,
// writing its work vector) as a graph, captured the first time on the
// hierarchy's own stream
template <typename T>
hipError_t ilu_graph(fsimg_hier *h, int l, hipGraphExec_t *out) {
  DevLevel &L = h->lev[l];
  const int k = std::is_same<T, double>::value ? 0 : 1;
  if (!L.ilu_exec[k]) {
    hipError_t e = hipSuccess;
    if (!h->ilu_cap) e = hipStreamCreateWithFlags(&h->ilu_cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(h->ilu_cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    launch_ilu_solve<T>(L, IluSel<T>::F(L), IluSel<T>::dinv(L), Sel<T>::d(L), IluSel<T>::work(L),
                        h->ilu_cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->ilu_cap, &g);
    if (e == hipSuccess) e = hipGraphInstantiate(&L.ilu_exec[k], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      L.ilu_exec[k] = nullptr;
      return e;
    }
  }
  *out = L.ilu_exec[k];
  return hipSuccess;
}

// one smoothing step with the residual d already computed (Vanka or ILU)
template <typename T>
void smooth_apply(fsimg_hier *h, int l, const T *d, T *x, bool assign, hipStream_t s) {
  if (h->opts.smoother == FSIMG_SMOOTHER_ILU) {
    DevLevel &L = h->lev[l];
    T *dl = Sel<T>::d(L);
    if (d != dl) (void)hipMemcpyAsync(dl, d, L.n * sizeof(T), hipMemcpyDeviceToDevice, s);
    hipGraphExec_t g = nullptr;
    if (h->opts.graphs && ilu_graph<T>(h, l, &g) == hipSuccess)
      (void)hipGraphLaunch(g, s);
    else
      launch_ilu_solve<T>(L, IluSel<T>::F(L), IluSel<T>::dinv(L), dl, IluSel<T>::work(L), s);
    launch_ilu_axpy<T>(L, IluSel<T>::work(L), (T)h->opts.omega_ilu, assign, x, s);
    return;
  }
  vanka_apply<T>(h, l, d, x, assign, s);
}

void coarse_solve64(fsimg_hier *h, const double *r, double *x, hipStream_t s) {
  launch_coarse_gemv(h->lev.back(), r, x, s);
}

template <typename T>
void vcycle(fsimg_hier *h, int l, const T *r, T *x, hipStream_t s) {
  const int L = (int)h->lev.size();
  DevLevel &F = h->lev[l];
  if (l == L - 1) {
    if constexpr (std::is_same<T, double>::value) {
      coarse_solve64(h, r, x, s);
    } else {
      launch_cast_f2d(r, F.ct0, F.n, s);
      coarse_solve64(h, F.ct0, F.ct1, s);
      launch_cast_d2f(F.ct1, x, F.n, s);
    }
    return;
  }
  T *d = Sel<T>::d(F);
  const int nu1 = h->opts.nu_pre, nu2 = h->opts.nu_post;
  if (nu1 == 0) launch_fill<T>(x, F.n, T(0), s);
  for (int k = 0; k < nu1; ++k) {
    if (k == 0) {
      smooth_apply<T>(h, l, r, x, true, s);  // x = 0: the residual is r
    } else {
      residual<T>(h, l, r, x, d, s);
      smooth_apply<T>(h, l, d, x, false, s);
    }
  }
  residual<T>(h, l, r, x, d, s);
  DevLevel &C = h->lev[l + 1];
  launch_restrict<T>(F, C, d, Sel<T>::r(C), s);
  vcycle<T>(h, l + 1, Sel<T>::r(C), Sel<T>::x(C), s);
  launch_prolong_add<T>(F, C, Sel<T>::x(C), x, s);
  for (int k = 0; k < nu2; ++k) {
    residual<T>(h, l, r, x, d, s);
    smooth_apply<T>(h, l, d, x, false, s);
  }
}

// z = M^-1 v (FP64 in, FP64 out)
void precondition(fsimg_hier *h, const double *v, double *z, hipStream_t s) {
  DevLevel &F = h->lev[0];
  if (h->opts.precision == FSIMG_MIXED) {
    launch_cast_d2f(v, F.r32, F.n, s);
    vcycle<float>(h, 0, F.r32, F.x32, s);
    launch_cast_f2d(F.x32, z, F.n, s);
  } else {
    vcycle<double>(h, 0, v, z, s);
  }
}

bool hier_mixed(const fsimg_hier *h) { return h->opts.precision == FSIMG_MIXED; }

fsimg_status check_level(const fsimg_hier *h, int level, bool allow_coarsest) {
  if (!h) return fail(FSIMG_ERR_ARG, "null hierarchy");
  const int L = (int)h->lev.size();
  if (level < 0 || level >= L || (!allow_coarsest && level == L - 1))
    return fail(FSIMG_ERR_ARG, "level out of range");
  return FSIMG_OK;
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char *fsimg_last_error(void) { return g_err.c_str(); }

void fsimg_default_opts(fsimg_opts *o) {
  if (!o) return;
  o->omega = 0.8;
  o->rtol = 1e-8;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->restart = 20;
  o->max_iter = 200;
  o->precision = FSIMG_FP64;
  o->vanka_schedule = FSIMG_VANKA_GATHER;
  o->vanka_weighting = FSIMG_WEIGHT_MULT;
  o->profile = 0;
  o->graphs = 1;
  o->vanka_patches = FSIMG_PATCH_ELEMENT;
  o->smoother = FSIMG_SMOOTHER_VANKA;
  o->omega_ilu = 1.0;
  o->krylov_lookahead = 2;
  o->small_level_kib = 0;
}

fsimg_status fsimg_ctx_create(int device, size_t hbm_budget_bytes, fsimg_ctx **out) {
  if (!out) return fail(FSIMG_ERR_ARG, "null out");
  *out = nullptr;
  int ndev = 0;
  FSIMG_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(FSIMG_ERR_ARG, "no such device");
  FSIMG_HIP(hipSetDevice(device));
  FSIMG_TRY(noalloc_init(device));  // this device's no-allocation scratch array
  auto *c = new fsimg_ctx;
  c->device = device;
  c->budget = hbm_budget_bytes;
  *out = c;
  return FSIMG_OK;
}

void fsimg_ctx_destroy(fsimg_ctx *ctx) {
  if (!ctx) return;
  drop_plans(ctx);
  if (ctx->pstream) (void)hipStreamDestroy(ctx->pstream);
  delete ctx;
}

size_t fsimg_ctx_bytes_in_use(const fsimg_ctx *ctx) { return ctx ? ctx->in_use : 0; }

static fsimg_status validate_opts(const fsimg_opts *o) {
  if (!o) return fail(FSIMG_ERR_ARG, "null options");
  if (!(o->omega > 0.0) || !(o->rtol > 0.0)) return fail(FSIMG_ERR_ARG, "omega and rtol must be > 0");
  if (o->nu_pre < 0 || o->nu_post < 0 || o->nu_pre + o->nu_post == 0)
    return fail(FSIMG_ERR_ARG, "need at least one smoothing step");
  if (o->restart < 1 || o->restart > kMaxVec - 2) return fail(FSIMG_ERR_ARG, "restart must be 1..30");
  if (o->max_iter < 1) return fail(FSIMG_ERR_ARG, "max_iter must be >= 1");
  if (o->precision != FSIMG_FP64 && o->precision != FSIMG_MIXED) return fail(FSIMG_ERR_ARG, "bad precision");
  if (o->vanka_schedule < 0 || o->vanka_schedule > 2) return fail(FSIMG_ERR_ARG, "bad schedule");
  if (o->vanka_weighting < 0 || o->vanka_weighting > 1) return fail(FSIMG_ERR_ARG, "bad weighting");
  if (o->graphs < 0 || o->graphs > 1) return fail(FSIMG_ERR_ARG, "graphs must be 0 or 1");
  if (o->krylov_lookahead < 1 || o->krylov_lookahead > 2)
    return fail(FSIMG_ERR_ARG, "krylov_lookahead must be 1 or 2");
  if (o->small_level_kib < 0) return fail(FSIMG_ERR_ARG, "small_level_kib must be >= 0");
  if (o->vanka_patches < 0 || o->vanka_patches > 1) return fail(FSIMG_ERR_ARG, "bad patch shape");
  if (o->vanka_patches == FSIMG_PATCH_BLOCK && o->vanka_schedule != FSIMG_VANKA_GATHER)
    return fail(FSIMG_ERR_ARG, "block patches need the GATHER schedule");
  if (o->smoother != FSIMG_SMOOTHER_VANKA && o->smoother != FSIMG_SMOOTHER_ILU)
    return fail(FSIMG_ERR_ARG, "bad smoother");
  if (o->smoother == FSIMG_SMOOTHER_ILU && !(o->omega_ilu > 0.0))
    return fail(FSIMG_ERR_ARG, "omega_ilu must be > 0");
  return FSIMG_OK;
}

fsimg_status fsimg_hier_footprint(const fsimg_level_desc *levels, int nlev, const fsimg_opts *opts,
                                  size_t *bytes) {
  FSIMG_TRY(validate_opts(opts));
  FSIMG_TRY(validate_levels(levels, nlev));
  if (!bytes) return fail(FSIMG_ERR_ARG, "null out");
  size_t s = 0;
  for (int l = 0; l < nlev; ++l) {
    const bool coarse = l == nlev - 1;
    int64_t npatch = 0, ng = 0, nblk = 0;
    if (!coarse) {
      PatchPlan P;
      FSIMG_TRY(plan_patches(levels[l], FSIMG_VANKA_GATHER, levels[l].cell_class, P,
                             opts->vanka_patches));
      npatch = (int64_t)P.elem.size();
      ng = (int64_t)P.gidx.size();
      nblk = P.blk_nl ? (int64_t)P.blk_nodes.size() / P.blk_nl : 0;
    }
    s += level_bytes(levels[l], npatch, ng, coarse, *opts, nblk);
  }
  s += krylov_bytes(levels[0].nrows * levels[0].block, opts->restart);
  *bytes = s;
  return FSIMG_OK;
}

void fsimg_hier_destroy(fsimg_hier *h) {
  if (!h) return;
  (void)hipSetDevice(h->ctx->device);
  {  // cached batch plans that cover this hierarchy are stale
    auto &ps = h->ctx->plans;
    for (size_t i = 0; i < ps.size();) {
      if (plan_covers(ps[i], h->uid)) {
        destroy_plan(ps[i]);
        ps.erase(ps.begin() + (long)i);
      } else {
        ++i;
      }
    }
  }
  if (h->side) (void)hipStreamSynchronize(h->side);
  for (auto &a : h->allocs) {
    (void)hipFree(a.first);
    h->ctx->in_use -= a.second;
  }
  h->allocs.clear();
  for (auto &L : h->lev)
    for (hipGraphExec_t &g : L.ilu_exec)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  if (h->ilu_cap) (void)hipStreamDestroy(h->ilu_cap);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->hpin) (void)hipHostFree(h->hpin);
  if (h->hstatus) (void)hipHostFree(h->hstatus);
  delete h;
}

// Block ILU(0) data of one level: factor / inverse storage, the diagonal
// positions and the level schedules of the lower and upper triangles (level of
// row i = 1 + the largest level among the rows it depends on).
fsimg_status ilu_setup(fsimg_hier *h, const fsimg_level_desc &D, DevLevel &L, bool mixed,
                       hipStream_t s) {
  const int64_t n = D.nrows, bb = (int64_t)D.block * D.block;
  std::vector<int32_t> diag(n), lev(n);
  int maxrow = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t b0 = D.rowptr[i], b1 = D.rowptr[i + 1];
    maxrow = std::max(maxrow, (int)(b1 - b0));
    diag[i] = -1;
    for (int32_t p = b0; p < b1; ++p)
      if (D.colind[p] == i) diag[i] = p;
    if (diag[i] < 0) return fail(FSIMG_ERR_ARG, "ILU: block row without a diagonal block");
  }
  if (maxrow > kIluMaxRow)
    return fail(FSIMG_ERR_ARG, "ILU: block rows longer than " + std::to_string(kIluMaxRow));
  L.ilu_maxrow = maxrow;
  auto schedule = [&](bool lower, std::vector<int32_t> &order, std::vector<int64_t> &ptr) {
    int nl = 0;
    for (int64_t t = 0; t < n; ++t) {
      const int64_t i = lower ? t : n - 1 - t;
      int v = 0;
      for (int32_t p = D.rowptr[i]; p < D.rowptr[i + 1]; ++p) {
        const int32_t k = D.colind[p];
        if (lower ? k < i : k > i) v = std::max(v, lev[k] + 1);
      }
      lev[i] = v;
      nl = std::max(nl, v + 1);
    }
    ptr.assign(nl + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++ptr[lev[i] + 1];
    for (int v = 0; v < nl; ++v) ptr[v + 1] += ptr[v];
    std::vector<int64_t> at(ptr.begin(), ptr.end() - 1);
    order.resize(n);
    for (int64_t i = 0; i < n; ++i) order[at[lev[i]]++] = (int32_t)i;  // ascending within a level
  };
  std::vector<int32_t> lo, uo;
  schedule(true, lo, L.lptr);
  schedule(false, uo, L.uptr);
  FSIMG_TRY(dalloc(h, &L.ilu64, D.nnzb * bb));
  FSIMG_TRY(dalloc(h, &L.dinv64, n * bb));
  FSIMG_TRY(dalloc(h, &L.idiag, n));
  FSIMG_TRY(dalloc(h, &L.lorder, n));
  FSIMG_TRY(dalloc(h, &L.uorder, n));
  if (mixed) {
    FSIMG_TRY(dalloc(h, &L.ilu32, D.nnzb * bb));
    FSIMG_TRY(dalloc(h, &L.dinv32, n * bb));
    FSIMG_TRY(dalloc(h, &L.iw32, n * D.block));
  } else {
    FSIMG_TRY(dalloc(h, &L.iw64, n * D.block));
  }
  if (hipMemcpyAsync(L.idiag, diag.data(), n * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(L.lorder, lo.data(), n * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(L.uorder, uo.data(), n * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(FSIMG_ERR_HIP, "ILU schedule upload");
  return FSIMG_OK;
}

fsimg_status fsimg_hier_create(fsimg_ctx *ctx, const fsimg_level_desc *levels, int nlev,
                               const fsimg_opts *opts, void *stream, fsimg_hier **out) {
  if (!ctx || !out) return fail(FSIMG_ERR_ARG, "null argument");
  *out = nullptr;
  const auto t_create = std::chrono::steady_clock::now();
  FSIMG_TRY(validate_opts(opts));
  FSIMG_TRY(validate_levels(levels, nlev));
  FSIMG_HIP(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  size_t need = 0;
  FSIMG_TRY(fsimg_hier_footprint(levels, nlev, opts, &need));
  if (ctx->budget && ctx->in_use + need > ctx->budget)
    return fail(FSIMG_ERR_BUDGET, "hierarchy needs " + std::to_string(need) + " bytes, " +
                                      std::to_string(ctx->budget - ctx->in_use) + " left in the budget");
  auto *h = new fsimg_hier;
  h->uid = g_uid.fetch_add(1);
  h->ctx = ctx;
  h->opts = *opts;
  h->m = opts->restart;
  h->lev.resize(nlev);
  const bool mixed = opts->precision == FSIMG_MIXED;
  auto bail = [&](fsimg_status st) {
    std::string keep = g_err;
    fsimg_hier_destroy(h);
    g_err = keep;
    return st;
  };
#define FSIMG_CHK(expr)                      \
  do {                                       \
    fsimg_status st__ = (expr);              \
    if (st__ != FSIMG_OK) return bail(st__); \
  } while (0)
#define FSIMG_HIPC(expr)                                                                        \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return bail(fail(FSIMG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)));      \
  } while (0)
  for (int l = 0; l < nlev; ++l) {
    const fsimg_level_desc &D = levels[l];
    DevLevel &L = h->lev[l];
    L.tune = &ctx->tune;
    L.dim = D.dim;
    L.b = D.block;
    L.nl = D.dim == 2 ? 9 : 27;
    L.np = L.nl * L.b;
    L.npc64 = npc_for(L.np, 8);
    L.npc32 = npc_for(L.np, 4);
    for (int a = 0; a < 3; ++a) { L.cells[a] = D.cells[a]; L.nnode[a] = a < D.dim ? 2 * D.cells[a] + 1 : 1; }
    L.nrows = D.nrows;
    L.n = D.nrows * D.block;
    L.nnzb = D.nnzb;
    const int64_t bb = (int64_t)L.b * L.b;
    FSIMG_CHK(dalloc(h, &L.rowptr, L.nrows + 1));
    FSIMG_CHK(dalloc(h, &L.colind, L.nnzb));
    FSIMG_CHK(dalloc(h, &L.vals64, L.nnzb * bb));
    FSIMG_CHK(dalloc(h, &L.mask, L.n));
    FSIMG_HIPC(hipMemcpyAsync(L.rowptr, D.rowptr, (L.nrows + 1) * 4, hipMemcpyHostToDevice, s));
    FSIMG_HIPC(hipMemcpyAsync(L.colind, D.colind, L.nnzb * 4, hipMemcpyHostToDevice, s));
    FSIMG_HIPC(hipMemcpyAsync(L.vals64, D.vals, L.nnzb * bb * 8, hipMemcpyHostToDevice, s));
    FSIMG_HIPC(hipMemcpyAsync(L.mask, D.dirichlet, L.n, hipMemcpyHostToDevice, s));
    if (mixed) {
      FSIMG_CHK(dalloc(h, &L.vals32, L.nnzb * bb));
      launch_cast_d2f(L.vals64, L.vals32, L.nnzb * bb, s);
    }
    h->host_mask.emplace_back(D.dirichlet, D.dirichlet + L.n);
    const bool coarse = l == nlev - 1;
    if (!coarse) {
      PatchPlan P;
      FSIMG_CHK(plan_patches(D, opts->vanka_schedule, D.cell_class, P, opts->vanka_patches));
      L.npatch = (int64_t)P.elem.size();
      PatchBlocks &B = L.blk;
      B.npatch = P.blk_nl ? (int64_t)P.blk_nodes.size() / P.blk_nl : 0;
      if (B.npatch > 0) {
        B.nl = P.blk_nl;
        B.np = B.nl * L.b;
        B.npc64 = npc_for(B.np, 8);
        B.npc32 = npc_for(B.np, 4);
        B.yofs = L.npatch * L.np;
        FSIMG_CHK(dalloc(h, &B.pnodes, P.blk_nodes.size()));
        FSIMG_HIPC(hipMemcpyAsync(B.pnodes, P.blk_nodes.data(), P.blk_nodes.size() * 4,
                                  hipMemcpyHostToDevice, s));
        if (B.np > 128 || B.nl > 27) {
          FSIMG_CHK(dalloc(h, &B.work, B.npatch * B.np * B.np));
          FSIMG_CHK(dalloc(h, &B.ub, B.npatch * kCoarseStage * B.np));
          FSIMG_CHK(dalloc(h, &B.rb, B.npatch * kCoarseStage * B.np));
          FSIMG_CHK(dalloc(h, &B.piv, B.npatch * B.np));
          FSIMG_CHK(dalloc(h, &B.iwork, B.npatch * B.np));
          FSIMG_CHK(dalloc(h, &B.amax, B.npatch));
        }
      }
      const int64_t ylen = L.npatch * L.np + B.npatch * B.np;
      L.pelem = P.elem;
      L.colour_start = P.colour_start;
      FSIMG_CHK(dalloc(h, &L.pnodes, P.nodes.size()));
      FSIMG_CHK(dalloc(h, &L.gptr, P.gptr.size()));
      FSIMG_CHK(dalloc(h, &L.gidx, P.gidx.size()));
      FSIMG_HIPC(hipMemcpyAsync(L.pnodes, P.nodes.data(), P.nodes.size() * 4, hipMemcpyHostToDevice, s));
      FSIMG_HIPC(hipMemcpyAsync(L.gptr, P.gptr.data(), P.gptr.size() * 4, hipMemcpyHostToDevice, s));
      if (!P.gidx.empty())
        FSIMG_HIPC(hipMemcpyAsync(L.gidx, P.gidx.data(), P.gidx.size() * 4, hipMemcpyHostToDevice, s));
      std::vector<double> sc(L.nrows);
      for (int64_t i = 0; i < L.nrows; ++i) {
        // the number of patches containing the node: geometric for element
        // patches; counted over the plan with blocks (a node inside a block
        // belongs to that one patch)
        double mult = node_mult(D, i);
        if (opts->vanka_patches == FSIMG_PATCH_BLOCK)
          mult = std::max(1, P.gptr[i + 1] - P.gptr[i]);
        sc[i] = opts->vanka_weighting == FSIMG_WEIGHT_MULT ? 1.0 / mult : 1.0;
      }
      const bool vanka = opts->smoother == FSIMG_SMOOTHER_VANKA;
      if (mixed) {
        std::vector<float> sf(sc.begin(), sc.end());
        FSIMG_CHK(dalloc(h, &L.scale32, L.nrows));
        FSIMG_HIPC(hipMemcpyAsync(L.scale32, sf.data(), L.nrows * 4, hipMemcpyHostToDevice, s));
        if (vanka) {
          FSIMG_CHK(dalloc(h, &L.inv32, L.npatch * L.np * L.npc32));
          if (B.npatch > 0) FSIMG_CHK(dalloc(h, &B.inv32, B.npatch * B.np * B.npc32));
          FSIMG_CHK(dalloc(h, &L.Y32, ylen));
        }
        FSIMG_CHK(dalloc(h, &L.r32, L.n));
        FSIMG_CHK(dalloc(h, &L.x32, L.n));
        FSIMG_CHK(dalloc(h, &L.d32, L.n));
        FSIMG_HIPC(hipStreamSynchronize(s));
      } else {
        FSIMG_CHK(dalloc(h, &L.scale64, L.nrows));
        FSIMG_HIPC(hipMemcpyAsync(L.scale64, sc.data(), L.nrows * 8, hipMemcpyHostToDevice, s));
        if (vanka) {
          FSIMG_CHK(dalloc(h, &L.inv64, L.npatch * L.np * L.npc64));
          if (B.npatch > 0) FSIMG_CHK(dalloc(h, &B.inv64, B.npatch * B.np * B.npc64));
          FSIMG_CHK(dalloc(h, &L.Y64, ylen));
        }
        FSIMG_CHK(dalloc(h, &L.r64, L.n));
        FSIMG_CHK(dalloc(h, &L.x64, L.n));
        FSIMG_CHK(dalloc(h, &L.d64, L.n));
        FSIMG_HIPC(hipStreamSynchronize(s));
      }
      if (!vanka) FSIMG_CHK(ilu_setup(h, D, L, mixed, s));
    } else {
      std::vector<int32_t> cf, ci(L.n, -1);
      for (int64_t i = 0; i < L.n; ++i)
        if (!D.dirichlet[i]) { ci[i] = (int32_t)cf.size(); cf.push_back((int32_t)i); }
      L.nfree = (int64_t)cf.size();
      FSIMG_CHK(dalloc(h, &L.cidx, L.n));
      FSIMG_HIPC(hipMemcpyAsync(L.cidx, ci.data(), L.n * 4, hipMemcpyHostToDevice, s));
      if (L.nfree > 0) {
        FSIMG_CHK(dalloc(h, &L.cfree, L.nfree));
        FSIMG_HIPC(hipMemcpyAsync(L.cfree, cf.data(), L.nfree * 4, hipMemcpyHostToDevice, s));
      }
      FSIMG_CHK(dalloc(h, &L.cinv, L.nfree * L.nfree));
      if (L.nfree > 0) {
        FSIMG_CHK(dalloc(h, &L.gj_a, L.nfree * L.nfree));
        FSIMG_CHK(dalloc(h, &L.gj_rowk, (int64_t)kCoarseStage * L.nfree));
        FSIMG_CHK(dalloc(h, &L.gj_colk, (int64_t)kCoarseStage * L.nfree));
        FSIMG_CHK(dalloc(h, &L.gj_piv, L.nfree));
        FSIMG_CHK(dalloc(h, &L.gj_colmap, L.nfree));
        FSIMG_CHK(dalloc(h, &L.gj_part, kRedBlocks));
      }
      FSIMG_CHK(dalloc(h, &L.ct0, L.n));
      FSIMG_CHK(dalloc(h, &L.ct1, L.n));
      if (mixed) {
        FSIMG_CHK(dalloc(h, &L.r32, L.n));
        FSIMG_CHK(dalloc(h, &L.x32, L.n));
      } else {
        FSIMG_CHK(dalloc(h, &L.r64, L.n));
        FSIMG_CHK(dalloc(h, &L.x64, L.n));
      }
    }
  }
  const int64_t n0 = h->lev[0].n;
  FSIMG_CHK(dalloc(h, &h->V, (size_t)(h->m + 1) * n0));
  FSIMG_CHK(dalloc(h, &h->Z, (size_t)h->m * n0));
  FSIMG_CHK(dalloc(h, &h->w, n0));
  FSIMG_CHK(dalloc(h, &h->partial, (size_t)kRedBlocks * kMaxVec));
  FSIMG_CHK(dalloc(h, &h->small, 256));
  FSIMG_CHK(dalloc(h, &h->dstatus, 16));
  FSIMG_HIPC(hipHostMalloc((void **)&h->hpin, 256 * sizeof(double), hipHostMallocDefault));
  FSIMG_HIPC(hipHostMalloc((void **)&h->hstatus, 16 * sizeof(int), hipHostMallocDefault));
  FSIMG_HIPC(hipStreamSynchronize(s));
#undef FSIMG_CHK
#undef FSIMG_HIPC
  h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_create).count();
  *out = h;
  return FSIMG_OK;
}

fsimg_status fsimg_hier_info(const fsimg_hier *h, int level, fsimg_level_info *out) {
  FSIMG_TRY(check_level(h, level, true));
  if (!out) return fail(FSIMG_ERR_ARG, "null out");
  const DevLevel &L = h->lev[level];
  out->nrows = L.nrows;
  out->n = L.n;
  out->nnzb = L.nnzb;
  out->npatch = L.npatch;
  out->np = L.np;
  out->ncolours = L.colour_start.empty() ? 0 : (int)L.colour_start.size() - 1;
  size_t bytes = 0;
  const void *ptrs[] = {L.rowptr, L.colind, L.vals64, L.vals32, L.mask, L.pnodes, L.inv64, L.inv32,
                        L.gptr, L.gidx, L.scale64, L.scale32, L.r64, L.x64, L.d64, L.Y64,
                        L.r32, L.x32, L.d32, L.Y32, L.cinv, L.ct0, L.ct1, L.cfree, L.cidx,
                        L.gj_a, L.gj_rowk, L.gj_colk, L.gj_piv, L.gj_colmap, L.gj_part,
                        L.ilu64, L.ilu32, L.dinv64, L.dinv32, L.iw64, L.iw32, L.idiag, L.lorder,
                        L.uorder};
  for (const void *p : ptrs)
    for (const auto &a : h->allocs)
      if (p && a.first == p) bytes += a.second;
  out->bytes = bytes;
  out->factor_ms = L.factor_ms;
  return FSIMG_OK;
}

fsimg_status fsimg_hier_set_profile(fsimg_hier *h, int on) {
  if (!h) return fail(FSIMG_ERR_ARG, "null hierarchy");
  h->opts.profile = on ? 1 : 0;
  return FSIMG_OK;
}

fsimg_status fsimg_hier_update_values(fsimg_hier *h, int level, const double *vals, int on_device,
                                      void *stream) {
  FSIMG_TRY(check_level(h, level, true));
  if (!vals) return fail(FSIMG_ERR_ARG, "null values");
  FSIMG_HIP(hipSetDevice(h->ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevLevel &L = h->lev[level];
  const int64_t cnt = L.nnzb * L.b * L.b;
  FSIMG_HIP(hipMemcpyAsync(L.vals64, vals, cnt * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  if (L.vals32) launch_cast_d2f(L.vals64, L.vals32, cnt, s);
  FSIMG_HIP(hipGetLastError());
  h->factored = false;
  return FSIMG_OK;
}

static fsimg_status factor_impl(fsimg_hier *h, void *stream);

fsimg_status fsimg_factor(fsimg_hier *h, void *stream) {
  if (!h) return fail(FSIMG_ERR_ARG, "null hierarchy");
  const auto t0 = std::chrono::steady_clock::now();
  const fsimg_status st = factor_impl(h, stream);
  h->factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

static fsimg_status factor_impl(fsimg_hier *h, void *stream) {
  FSIMG_HIP(hipSetDevice(h->ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool mixed = hier_mixed(h);
  const int nlev = (int)h->lev.size();
  const bool prof = h->opts.profile != 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (prof) {
    FSIMG_HIP(hipEventCreate(&ev[0]));
    FSIMG_HIP(hipEventCreate(&ev[1]));
  }
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      for (int i = 0; i < 2; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } ev_guard{ev};
  // coarsest level: dense Gauss-Jordan inverse in FP64 on the side stream,
  // concurrently with the patch factorisations of the finer levels (it needs
  // only the coarsest matrix and its own workspace and status slots 8, 9).
  // The dense matrix and its largest entry (the pivot threshold) are taken
  // first on the caller's stream; the chain of Gauss-Jordan launches is
  // enqueued on the side stream right after the first patch kernel has been
  // launched, so that the host enqueues it while that kernel runs.
  DevLevel &C = h->lev.back();
  const int64_t n = C.nfree;
  bool coarse = false;
  double amax = 0.0;
  if (n > 0) {
    if (!h->side) FSIMG_HIP(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
    if (!h->ev_fork) FSIMG_HIP(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    if (!h->ev_join) FSIMG_HIP(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    launch_fill<double>(C.gj_a, n * n, 0.0, s);
    launch_densify(C, C.gj_a, s);
    launch_absmax(C.gj_a, n * n, C.gj_part, s);
    std::vector<double> hp(kRedBlocks);
    if (hipMemcpyAsync(hp.data(), C.gj_part, kRedBlocks * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(FSIMG_ERR_HIP, "coarse absmax copy");
    for (double v : hp) amax = std::max(amax, v);
    FSIMG_HIP(hipEventRecord(h->ev_fork, s));
  }
  // the patch kernels' stream: with a coarse inverse to overlap, a stream
  // restricted to all CUs but kReservedCus (created once; if the runtime
  // refuses the CU mask, the caller's stream), ordered after everything the
  // caller's stream holds (ev_fork)
  hipStream_t ps = s;
  // worth it only while the patch work is about as long as the coarse chain:
  // patch kernels at ~15 TFLOP/s against ~3.4 us of chain per coarse dof
  // (C2: 5.3 and 6.4 ms); at C3 the patch kernels take 41 ms and hide the
  // chain on all CUs anyway
  double pflops = 0.0;
  for (int l = 0; l + 1 < nlev; ++l) {
    const DevLevel &L = h->lev[l];
    pflops += 2.0 * L.npatch * L.np * (double)L.np * L.np +
              2.0 * L.blk.npatch * L.blk.np * (double)L.blk.np * L.blk.np;
  }
  const bool mask_patches = n > 0 && pflops / 15e12 < 1.5 * 3.4e-6 * (double)n;
  fsimg_ctx *cx = h->ctx;
  if (mask_patches) {
    if (!cx->pstream_tried) {
      cx->pstream_tried = true;
      int ncu = 0;
      if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->ctx->device) == hipSuccess &&
          ncu > 2 * kReservedCus) {
        std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
        for (int c = 0; c < ncu - kReservedCus; ++c) mask[c / 32] |= 1u << (c % 32);
        if (hipExtStreamCreateWithCUMask(&cx->pstream, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
          (void)hipGetLastError();
          cx->pstream = nullptr;
        }
      }
    }
    if (cx->pstream) {
      ps = cx->pstream;
      FSIMG_HIP(hipStreamWaitEvent(ps, h->ev_fork, 0));
    }
  }
  auto start_coarse = [&]() -> fsimg_status {
    if (n == 0 || coarse) return FSIMG_OK;
    hipStream_t c = h->side;
    double *a = C.gj_a, *rowk = C.gj_rowk, *colk = C.gj_colk;
    int *piv = C.gj_piv, *colmap = C.gj_colmap;
    FSIMG_HIP(hipStreamWaitEvent(c, h->ev_fork, 0));
    h->hstatus[10] = 0;
    h->hstatus[11] = INT_MAX;
    FSIMG_HIP(hipMemcpyAsync(h->dstatus + 8, h->hstatus + 10, 2 * sizeof(int), hipMemcpyHostToDevice, c));
    coarse = true;  // from here on the side stream has work to join
    if (!launch_coarse_gj_blocked(n, a, piv, colmap, colk, rowk, 1e-15 * amax, h->dstatus + 8, C.cinv,
                                  c)) {
      // beyond the blocked kernel's size: one pivot and one update launch per column
      for (int64_t k = 0; k < n; ++k) {
        launch_gj_pivot(n, k, a, piv, rowk, colk, 1e-15 * amax, h->dstatus + 8, c);
        launch_gj_update(n, k, a, rowk, colk, c);
      }
      launch_gj_finish(n, a, piv, colmap, C.cinv, c);
    }
    FSIMG_HIP(hipGetLastError());
    FSIMG_HIP(hipMemcpyAsync(h->hstatus + 8, h->dstatus + 8, 2 * sizeof(int), hipMemcpyDeviceToHost, c));
    FSIMG_HIP(hipEventRecord(h->ev_join, c));
    return FSIMG_OK;
  };
  auto patches = [&]() -> fsimg_status {
    for (int l = 0; l + 1 < nlev; ++l) {
      DevLevel &L = h->lev[l];
      L.factor_ms = 0.0;
      if (h->opts.smoother == FSIMG_SMOOTHER_ILU) {
        const int64_t nv = L.nnzb * L.b * L.b;
        const int init[2] = {0, INT_MAX};
        FSIMG_HIP(hipMemcpyAsync(h->dstatus, init, sizeof(init), hipMemcpyHostToDevice, ps));
        FSIMG_HIP(hipMemcpyAsync(L.ilu64, L.vals64, nv * 8, hipMemcpyDeviceToDevice, ps));
        if (prof) FSIMG_HIP(hipEventRecord(ev[0], ps));
        launch_ilu_factor(L, h->dstatus, ps);
        FSIMG_HIP(hipGetLastError());
        FSIMG_TRY(start_coarse());
        if (prof) FSIMG_HIP(hipEventRecord(ev[1], ps));
        if (mixed) {
          launch_cast_d2f(L.ilu64, L.ilu32, nv, ps);
          launch_cast_d2f(L.dinv64, L.dinv32, L.nrows * L.b * L.b, ps);
        }
        FSIMG_HIP(hipMemcpyAsync(h->hstatus, h->dstatus, 2 * sizeof(int), hipMemcpyDeviceToHost, ps));
        FSIMG_HIP(hipStreamSynchronize(ps));
        if (prof) {
          float ms = 0.0f;
          FSIMG_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
          L.factor_ms = ms;
        }
        if (h->hstatus[0])
          return fail(FSIMG_ERR_SINGULAR, "singular diagonal block in the ILU factors of level " +
                                              std::to_string(l) + ": block row " +
                                              std::to_string(h->hstatus[1]));
        continue;
      }
      for (int g = 0; g < 2; ++g) {  // element patches, then block patches
        const int64_t np_ = g == 0 ? L.npatch : L.blk.npatch;
        if (np_ == 0) continue;
        const int init[2] = {0, INT_MAX};
        FSIMG_HIP(hipMemcpyAsync(h->dstatus, init, sizeof(init), hipMemcpyHostToDevice, ps));
        if (prof) FSIMG_HIP(hipEventRecord(ev[0], ps));
        if (g == 0) {
          if (mixed) launch_patch_factor<float>(L, L.inv32, L.npc32, h->dstatus, ps);
          else launch_patch_factor<double>(L, L.inv64, L.npc64, h->dstatus, ps);
        } else {
          if (mixed) launch_patch_factor_blocks<float>(L, L.blk.inv32, L.blk.npc32, h->dstatus, ps);
          else launch_patch_factor_blocks<double>(L, L.blk.inv64, L.blk.npc64, h->dstatus, ps);
        }
        FSIMG_HIP(hipGetLastError());
        FSIMG_TRY(start_coarse());
        if (prof) FSIMG_HIP(hipEventRecord(ev[1], ps));
        FSIMG_HIP(hipMemcpyAsync(h->hstatus, h->dstatus, 2 * sizeof(int), hipMemcpyDeviceToHost, ps));
        FSIMG_HIP(hipStreamSynchronize(ps));
        if (prof) {
          float ms = 0.0f;
          FSIMG_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
          L.factor_ms += ms;
        }
        if (h->hstatus[0]) {
          const int64_t p = h->hstatus[1];
          return fail(FSIMG_ERR_SINGULAR,
                      std::string("singular ") + (g == 0 ? "patch" : "block patch") +
                          " matrix on level " + std::to_string(l) + ": patch " + std::to_string(p) +
                          (g == 0 ? " (cell " + std::to_string(p >= 0 && p < L.npatch ? L.pelem[p] : -1) +
                                        ")"
                                  : std::string()));
        }
      }
    }
    return FSIMG_OK;
  };
  fsimg_status pst = patches();
  if (pst == FSIMG_OK) pst = start_coarse();  // no patch kernel ran
  if (coarse) {  // join: the caller's stream waits for the coarse inverse
    if (pst != FSIMG_OK) {  // nothing of the side stream may outlive a failed call
      (void)hipStreamSynchronize(h->side);
      return pst;
    }
    if (hipEventSynchronize(h->ev_join) != hipSuccess || hipStreamWaitEvent(s, h->ev_join, 0) != hipSuccess) {
      (void)hipStreamSynchronize(h->side);
      return fail(FSIMG_ERR_HIP, "coarse factor join");
    }
  }
  if (pst != FSIMG_OK) return pst;
  if (coarse && h->hstatus[8])
    return fail(FSIMG_ERR_SINGULAR, "singular coarse matrix (level " + std::to_string(nlev - 1) +
                                        ", pivot column " + std::to_string(h->hstatus[9]) + ")");
  h->factored = true;
  return FSIMG_OK;
}

fsimg_status fsimg_solve_batch(int n, fsimg_hier *const *hiers, const double *const *b_dev,
                               double *const *x_dev, fsimg_stats *stats, void *stream) {
  if (n < 1 || !hiers || !hiers[0]) return fail(FSIMG_ERR_ARG, "empty batch");
  for (int k = 0; k < n; ++k)
    if (hiers[k] && hiers[k]->opts.smoother != FSIMG_SMOOTHER_VANKA)
      return fail(FSIMG_ERR_ARG, "batched solves take Vanka hierarchies only (ILU: fsimg_solve)");
  FSIMG_HIP(hipSetDevice(hiers[0]->ctx->device));
  return solve_batch(hiers[0]->ctx, n, hiers, b_dev, x_dev, stats, static_cast<hipStream_t>(stream));
}

fsimg_status fsimg_solve_noalloc(fsimg_hier *h, const double *b, double *x, fsimg_stats *stats,
                                 void *stream) {
  if (!h) return fail(FSIMG_ERR_ARG, "null hierarchy");
  FSIMG_HIP(hipSetDevice(h->ctx->device));
  return solve_noalloc(h, b, x, stats, static_cast<hipStream_t>(stream));
}

fsimg_status fsimg_solve(fsimg_hier *h, const double *b, double *x, fsimg_stats *stats, void *stream) {
  if (!h || !b || !x) return fail(FSIMG_ERR_ARG, "null argument");
  if (!h->factored) return fail(FSIMG_ERR_STATE, "fsimg_factor must run before fsimg_solve");
  FSIMG_HIP(hipSetDevice(h->ctx->device));
  if (h->opts.vanka_schedule == FSIMG_VANKA_GATHER &&
      h->opts.smoother == FSIMG_SMOOTHER_VANKA)  // the batched driver with one instance
    return solve_batch(h->ctx, 1, &h, &b, &x, stats, static_cast<hipStream_t>(stream));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  DevLevel &F = h->lev[0];
  const int64_t n = F.n;
  const int m = h->m;
  double *sm = h->small;
  double *hp = h->hpin;
  h->profiling = h->opts.profile != 0;
  h->tv.begin_solve();
  h->ts.begin_solve();
  fsimg_stats st{};
  st.status = FSIMG_OK;
  // r0 = b - A x (masked), non-finite check
  launch_bsr_spmv<double>(F, F.vals64, x, b, h->w, true, s);
  h->hstatus[0] = 0;
  FSIMG_HIP(hipMemcpyAsync(h->dstatus, h->hstatus, sizeof(int), hipMemcpyHostToDevice, s));
  launch_nonfinite_count(h->w, n, h->dstatus, s);
  launch_multidot(h->w, 1, n, h->w, h->partial, s);
  launch_reduce_partials(h->partial, 1, sm + kSS, s);
  FSIMG_HIP(hipMemcpyAsync(hp + kSS, sm + kSS, 8, hipMemcpyDeviceToHost, s));
  FSIMG_HIP(hipMemcpyAsync(h->hstatus, h->dstatus, sizeof(int), hipMemcpyDeviceToHost, s));
  FSIMG_HIP(hipStreamSynchronize(s));
  if (h->hstatus[0]) {
    st.status = FSIMG_ERR_NONFINITE;
    if (stats) *stats = st;
    return fail(FSIMG_ERR_NONFINITE, "non-finite entries in b or the initial residual");
  }
  const double beta0 = std::sqrt(hp[kSS]);
  double rnorm = beta0;
  int it = 0, restarts = 0;
  bool converged = beta0 == 0.0;
  const double tol = h->opts.rtol * beta0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  while (!converged && it < h->opts.max_iter) {
    launch_scale_by_rsqrt(h->w, sm + kSS, h->V, n, s);  // v_0 = r / ||r||
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = rnorm;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      double *vj = h->V + (size_t)j * n;
      double *zj = h->Z + (size_t)j * n;
      precondition(h, vj, zj, s);
      // w = A z_j, zero at identity rows (b = 0 residual, negated below by the sign of h)
      launch_bsr_spmv<double>(F, F.vals64, zj, nullptr, h->w, false, s);
      launch_mask_zero(h->w, F.mask, n, s);
      // classical Gram-Schmidt, two passes
      launch_multidot(h->V, j + 1, n, h->w, h->partial, s);
      launch_reduce_partials(h->partial, j + 1, sm + kH1, s);
      launch_axpy_dot(h->V, j + 1, n, sm + kH1, h->w, h->partial, s);
      launch_reduce_partials(h->partial, j + 1, sm + kH2, s);
      launch_axpy_norm(h->V, j + 1, n, sm + kH2, h->w, h->partial, s);
      launch_reduce_partials(h->partial, 1, sm + kSS, s);
      launch_add_small(sm + kH1, sm + kH2, sm + kH, j + 1, s);
      launch_scale_by_rsqrt(h->w, sm + kSS, h->V + (size_t)(j + 1) * n, n, s);
      FSIMG_HIP(hipMemcpyAsync(hp + kH, sm + kH, (j + 1) * 8, hipMemcpyDeviceToHost, s));
      FSIMG_HIP(hipMemcpyAsync(hp + kSS, sm + kSS, 8, hipMemcpyDeviceToHost, s));
      FSIMG_HIP(hipStreamSynchronize(s));
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hp[kH + i];
      const double hn = std::sqrt(hp[kSS]);
      H[(size_t)(j + 1) * m + j] = hn;
      for (int i = 0; i < j; ++i) {
        const double a0 = H[(size_t)i * m + j], a1 = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a0 + sn[i] * a1;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a0 + cs[i] * a1;
      }
      const double hjj = H[(size_t)j * m + j];
      const double den = std::hypot(hjj, hn);
      cs[j] = hjj / den;
      sn[j] = hn / den;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      k = j + 1;
      if (st.nhist < FSIMG_HIST) st.res_hist[st.nhist++] = std::fabs(g[j + 1]) / beta0;
      if (!std::isfinite(g[j + 1])) break;
      if (std::fabs(g[j + 1]) <= tol || it >= h->opts.max_iter || hn == 0.0) break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int c = i + 1; c < k; ++c) t -= H[(size_t)i * m + c] * y[c];
      y[i] = t / H[(size_t)i * m + i];
    }
    FSIMG_HIP(hipMemcpyAsync(sm + kY, y.data(), k * 8, hipMemcpyHostToDevice, s));
    launch_combine(h->Z, k, n, sm + kY, x, s);
    launch_bsr_spmv<double>(F, F.vals64, x, b, h->w, true, s);
    launch_multidot(h->w, 1, n, h->w, h->partial, s);
    launch_reduce_partials(h->partial, 1, sm + kSS, s);
    FSIMG_HIP(hipMemcpyAsync(hp + kSS, sm + kSS, 8, hipMemcpyDeviceToHost, s));
    FSIMG_HIP(hipStreamSynchronize(s));
    ++restarts;
    rnorm = std::sqrt(hp[kSS]);
    if (!std::isfinite(rnorm)) { st.status = FSIMG_ERR_NONFINITE; break; }
    if (rnorm <= tol) converged = true;
  }
  FSIMG_HIP(hipGetLastError());
  st.iters = it;
  st.restarts = restarts;
  st.rel_res = beta0 > 0.0 ? rnorm / beta0 : 0.0;
  st.setup_ms = h->setup_ms;
  st.factor_ms = h->factor_ms;
  if (st.status == FSIMG_OK && !converged) st.status = FSIMG_ERR_NOCONV;
  if (h->profiling) {
    FSIMG_HIP(hipStreamSynchronize(s));
    st.vanka_ms = h->tv.total_ms(&st.vanka_launches);
    st.spmv_ms = h->ts.total_ms(&st.spmv_launches);
  }
  h->profiling = false;
  st.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  if (st.status == FSIMG_ERR_NOCONV)
    return fail(FSIMG_ERR_NOCONV, "no convergence in " + std::to_string(it) + " iterations (rel. residual " +
                                      std::to_string(st.rel_res) + ")");
  if (st.status == FSIMG_ERR_NONFINITE) return fail(FSIMG_ERR_NONFINITE, "non-finite residual");
  return FSIMG_OK;
}

fsimg_status fsimg_deform_update(int64_t nnodes, int dim, const uint8_t *mask, double k, double theta,
                                 const double *v_new, int v_stride, int v_offset, const double *u_old,
                                 const double *v_old, double *u_new, void *stream) {
  if (nnodes < 0 || dim < 1 || dim > 3 || !mask || !v_new || !u_new || v_stride < dim ||
      v_offset < 0 || v_offset + dim > v_stride)
    return fail(FSIMG_ERR_ARG, "bad deformation-update arguments");
  launch_deform(nnodes, dim, mask, k, theta, v_new, v_stride, v_offset, u_old, v_old, u_new,
                static_cast<hipStream_t>(stream));
  FSIMG_HIP(hipGetLastError());
  return FSIMG_OK;
}

// ------------------------------------------------------- single steps
static bool batched_steps(const fsimg_hier *h, int precision);

fsimg_status fsimg_level_apply(fsimg_hier *h, int level, int precision, const void *x, void *y,
                               void *stream) {
  FSIMG_TRY(check_level(h, level, true));
  if (!x || !y) return fail(FSIMG_ERR_ARG, "null vector");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevLevel &L = h->lev[level];
  if (precision == FSIMG_FP64) {
    launch_bsr_spmv<double>(L, L.vals64, (const double *)x, nullptr, (double *)y, false, s);
  } else {
    if (!L.vals32) return fail(FSIMG_ERR_ARG, "FP32 matrices exist only in mixed mode");
    launch_bsr_spmv<float>(L, L.vals32, (const float *)x, nullptr, (float *)y, false, s);
  }
  FSIMG_HIP(hipGetLastError());
  return FSIMG_OK;
}

fsimg_status fsimg_level_residual(fsimg_hier *h, int level, int precision, const void *b,
                                  const void *x, void *d, void *stream) {
  FSIMG_TRY(check_level(h, level, true));
  if (!x || !b || !d) return fail(FSIMG_ERR_ARG, "null vector");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (level + 1 < (int)h->lev.size() && batched_steps(h, precision))
    return single_step(h, ONE_RESIDUAL, level, b, x, d, s);
  DevLevel &L = h->lev[level];
  if (precision == FSIMG_FP64) {
    launch_bsr_spmv<double>(L, L.vals64, (const double *)x, (const double *)b, (double *)d, true, s);
  } else {
    if (!L.vals32) return fail(FSIMG_ERR_ARG, "FP32 matrices exist only in mixed mode");
    launch_bsr_spmv<float>(L, L.vals32, (const float *)x, (const float *)b, (float *)d, true, s);
  }
  FSIMG_HIP(hipGetLastError());
  return FSIMG_OK;
}

// hierarchies whose solve runs the batched kernels (GATHER schedule, Vanka
// smoother): their single steps run the same kernels, with one instance
static bool batched_steps(const fsimg_hier *h, int precision) {
  return h->opts.vanka_schedule == FSIMG_VANKA_GATHER && h->opts.smoother == FSIMG_SMOOTHER_VANKA &&
         (precision == FSIMG_MIXED) == hier_mixed(h);
}

static fsimg_status check_prec(const fsimg_hier *h, int precision) {
  if ((precision == FSIMG_MIXED) != hier_mixed(h))
    return fail(FSIMG_ERR_ARG, "precision must match the hierarchy's precision for this step");
  return FSIMG_OK;
}

fsimg_status fsimg_vanka_step(fsimg_hier *h, int level, int precision, const void *b, void *x,
                              void *stream) {
  FSIMG_TRY(check_level(h, level, false));
  FSIMG_TRY(check_prec(h, precision));
  if (!h->factored) return fail(FSIMG_ERR_STATE, "fsimg_factor must run first");
  if (h->opts.smoother != FSIMG_SMOOTHER_VANKA)
    return fail(FSIMG_ERR_STATE, "the hierarchy uses the ILU smoother");
  if (!b || !x) return fail(FSIMG_ERR_ARG, "null vector");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batched_steps(h, precision)) return single_step(h, ONE_VANKA, level, b, nullptr, x, s);
  if (precision == FSIMG_FP64) {
    residual<double>(h, level, (const double *)b, (const double *)x, h->lev[level].d64, s);
    vanka_apply<double>(h, level, h->lev[level].d64, (double *)x, false, s);
  } else {
    residual<float>(h, level, (const float *)b, (const float *)x, h->lev[level].d32, s);
    vanka_apply<float>(h, level, h->lev[level].d32, (float *)x, false, s);
  }
  FSIMG_HIP(hipGetLastError());
  return FSIMG_OK;
}

fsimg_status fsimg_ilu_step(fsimg_hier *h, int level, int precision, const void *b, void *x,
                            void *stream) {
  FSIMG_TRY(check_level(h, level, false));
  FSIMG_TRY(check_prec(h, precision));
  if (h->opts.smoother != FSIMG_SMOOTHER_ILU)
    return fail(FSIMG_ERR_STATE, "the hierarchy uses the Vanka smoother");
  if (!h->factored) return fail(FSIMG_ERR_STATE, "fsimg_factor must run first");
  if (!b || !x) return fail(FSIMG_ERR_ARG, "null vector");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == FSIMG_FP64) {
    residual<double>(h, level, (const double *)b, (const double *)x, h->lev[level].d64, s);
    smooth_apply<double>(h, level, h->lev[level].d64, (double *)x, false, s);
  } else {
    residual<float>(h, level, (const float *)b, (const float *)x, h->lev[level].d32, s);
    smooth_apply<float>(h, level, h->lev[level].d32, (float *)x, false, s);
  }
  FSIMG_HIP(hipGetLastError());
  return FSIMG_OK;
}

fsimg_status fsimg_ilu_factors(fsimg_hier *h, int level, double *out) {
  FSIMG_TRY(check_level(h, level, false));
  if (h->opts.smoother != FSIMG_SMOOTHER_ILU)
    return fail(FSIMG_ERR_STATE, "the hierarchy uses the Vanka smoother");
  if (!h->factored) return fail(FSIMG_ERR_STATE, "fsimg_factor must run first");
  if (!out) return fail(FSIMG_ERR_ARG, "null out");
  FSIMG_HIP(hipSetDevice(h->ctx->device));
  const DevLevel &L = h->lev[level];
  FSIMG_HIP(hipMemcpy(out, L.ilu64, (size_t)L.nnzb * L.b * L.b * 8, hipMemcpyDeviceToHost));
  return FSIMG_OK;
}

fsimg_status fsimg_restrict(fsimg_hier *h, int level, int precision, const void *rf, void *rc,
                            void *stream) {
  FSIMG_TRY(check_level(h, level, false));
  if (!rf || !rc) return fail(FSIMG_ERR_ARG, "null vector");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batched_steps(h, precision)) return single_step(h, ONE_RESTRICT, level, rf, nullptr, rc, s);
  if (precision == FSIMG_FP64)
    launch_restrict<double>(h->lev[level], h->lev[level + 1], (const double *)rf, (double *)rc, s);
  else
    launch_restrict<float>(h->lev[level], h->lev[level + 1], (const float *)rf, (float *)rc, s);
  FSIMG_HIP(hipGetLastError());
  return FSIMG_OK;
}

fsimg_status fsimg_prolong_add(fsimg_hier *h, int level, int precision, const void *xc, void *xf,
                               void *stream) {
  FSIMG_TRY(check_level(h, level, false));
  if (!xc || !xf) return fail(FSIMG_ERR_ARG, "null vector");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batched_steps(h, precision)) return single_step(h, ONE_PROLONG, level, xc, nullptr, xf, s);
  if (precision == FSIMG_FP64)
    launch_prolong_add<double>(h->lev[level], h->lev[level + 1], (const double *)xc, (double *)xf, s);
  else
    launch_prolong_add<float>(h->lev[level], h->lev[level + 1], (const float *)xc, (float *)xf, s);
  FSIMG_HIP(hipGetLastError());
  return FSIMG_OK;
}

fsimg_status fsimg_coarse_solve(fsimg_hier *h, const double *r, double *x, void *stream) {
  if (!h || !r || !x) return fail(FSIMG_ERR_ARG, "null argument");
  if (!h->factored) return fail(FSIMG_ERR_STATE, "fsimg_factor must run first");
  if (batched_steps(h, FSIMG_FP64))
    return single_step(h, ONE_COARSE, (int)h->lev.size() - 1, r, nullptr, x,
                       static_cast<hipStream_t>(stream));
  coarse_solve64(h, r, x, static_cast<hipStream_t>(stream));
  FSIMG_HIP(hipGetLastError());
  return FSIMG_OK;
}

fsimg_status fsimg_vcycle(fsimg_hier *h, int precision, const void *r, void *z, void *stream) {
  if (!h || !r || !z) return fail(FSIMG_ERR_ARG, "null argument");
  FSIMG_TRY(check_prec(h, precision));
  if (!h->factored) return fail(FSIMG_ERR_STATE, "fsimg_factor must run first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batched_steps(h, precision)) return single_step(h, ONE_VCYCLE, 0, r, nullptr, z, s);
  if (precision == FSIMG_FP64) vcycle<double>(h, 0, (const double *)r, (double *)z, s);
  else vcycle<float>(h, 0, (const float *)r, (float *)z, s);
  FSIMG_HIP(hipGetLastError());
  return FSIMG_OK;
}

fsimg_status fsimg_patch_inverse(fsimg_hier *h, int level, int64_t patch, double *out, int64_t *elem,
                                 void *stream) {
  FSIMG_TRY(check_level(h, level, false));
  if (!h->factored) return fail(FSIMG_ERR_STATE, "fsimg_factor must run first");
  if (h->opts.smoother != FSIMG_SMOOTHER_VANKA)
    return fail(FSIMG_ERR_STATE, "the hierarchy uses the ILU smoother");
  DevLevel &L = h->lev[level];
  if (patch < 0 || patch >= L.npatch || !out) return fail(FSIMG_ERR_ARG, "bad patch index");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool mixed = hier_mixed(h);
  const int np = L.np, npc = mixed ? L.npc32 : L.npc64, G = mixed ? 4 : 2;
  std::vector<double> raw((size_t)np * npc);
  if (mixed) {
    std::vector<float> rf((size_t)np * npc);
    FSIMG_HIP(hipMemcpyAsync(rf.data(), L.inv32 + patch * (int64_t)np * npc, rf.size() * 4,
                             hipMemcpyDeviceToHost, s));
    FSIMG_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < rf.size(); ++i) raw[i] = rf[i];
  } else {
    FSIMG_HIP(hipMemcpyAsync(raw.data(), L.inv64 + patch * (int64_t)np * npc, raw.size() * 8,
                             hipMemcpyDeviceToHost, s));
    FSIMG_HIP(hipStreamSynchronize(s));
  }
  for (int r = 0; r < np; ++r)
    for (int c = 0; c < np; ++c) out[(size_t)r * np + c] = raw[((size_t)(c / G) * np + r) * G + c % G];
  if (elem) *elem = L.pelem[patch];
  return FSIMG_OK;
}

}  // extern "C"
