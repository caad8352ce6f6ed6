// Internal declarations shared by the HIP kernel files and the host runtime.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fsimg.h"

namespace fsimg {

// Launch shapes that do not change any result bit (rows per wavefront of the
// SpMV, patches per workgroup of the Vanka apply), chosen per (operation,
// block size or patch size, word size, size bucket = floor(log2 size)) by
// measurement (fsimg_hier_tune) or by the built-in defaults.  Owned by a
// context; read by every launch of its hierarchies.
struct TuneTable;
int spmv_rows_per_wave(const TuneTable *t, int b, int word, int64_t nrows);  // 1, 2 or 4
int vanka_patches_per_wg(const TuneTable *t, int np, int word, int64_t npatch);

// Rows one wavefront of the SpMV covers per row group: 1 for the whole-wave
// mapping (FP64, b >= 3), else 64 / lanes-per-row of the row-group mapping
// (FP32 b = 4: 32 lanes per row; b <= 3 in FP32, b <= 2 in FP64: 16).  A
// launch with R row groups per wave covers 4 * R * this many rows per
// 256-thread workgroup.
constexpr int spmv_group_rows(int b, int word) {
  return (word == 8 && b >= 3) ? 1 : (b == 4 ? 2 : 4);
}

constexpr int kMaxVec = 32;     // FGMRES: restart length + 1 must not exceed this
constexpr int kRedBlocks = 1024; // blocks of the two-stage reductions
constexpr int kCoarseStage = 32;  // panel width of the coarse Gauss-Jordan (staged pivot rows)
constexpr int kReservedCus = 16;  // CUs the patch factorisations leave to the coarse inverse
constexpr int kIluMaxRow = 256;   // longest block row the ILU factorisation stages in LDS

// Block patches (2 x 2 (x 2) elements, 5^d nodes) of a level: the second
// patch group, empty unless requested.  Their corrections follow those of
// the element patches in the level's Y buffer.
struct PatchBlocks {
  int nl = 0, np = 0, npc64 = 0, npc32 = 0;
  int64_t npatch = 0;
  int32_t *pnodes = nullptr;            // [npatch*nl]
  double *inv64 = nullptr;              // [npatch*np*npc64]
  float *inv32 = nullptr;               // [npatch*np*npc32]
  int64_t yofs = 0;                     // offset in Y (entries): npatch * np of the element group
  // batched blocked Gauss-Jordan scratch of the factorisation when np > 128
  double *work = nullptr;               // [npatch*np*np]
  double *ub = nullptr, *rb = nullptr;  // [npatch*kCoarseStage*np] panel updates, staged pivot rows
  double *amax = nullptr;               // [npatch]
  int *piv = nullptr, *iwork = nullptr; // [npatch*np]: pivot rows; used flags, then the inverse order
};

// One multigrid level on the device.  Vectors of the V-cycle exist in the
// precision of the hierarchy (T = double for FP64, float for mixed).
struct DevLevel {
  const TuneTable *tune = nullptr;      // launch shapes (the owning context's table)
  int dim = 0, b = 0, nl = 0, np = 0;   // nl = 3^d nodes per patch, np = nl*b
  int npc64 = 0, npc32 = 0;             // padded column counts of stored inverses
  double factor_ms = 0.0;               // event time of the last patch factorisation (profiling)
  int cells[3] = {1, 1, 1}, nnode[3] = {1, 1, 1};
  int64_t nrows = 0, n = 0, nnzb = 0;
  int32_t *rowptr = nullptr, *colind = nullptr;
  double *vals64 = nullptr;
  float *vals32 = nullptr;
  uint8_t *mask = nullptr;
  // Vanka patches (active ones only), ordered by the smoothing schedule
  int64_t npatch = 0;
  int32_t *pnodes = nullptr;            // [npatch*nl]
  std::vector<int64_t> pelem;           // host: cell of each active patch
  std::vector<int64_t> colour_start;    // host: patch ranges per colour
  double *inv64 = nullptr;              // [npatch*np*npc64]
  float *inv32 = nullptr;               // [npatch*np*npc32]
  int32_t *gptr = nullptr, *gidx = nullptr;  // node -> Y slot (patch*nl + local node; block
                                             // patches after the element ones), patch order
  PatchBlocks blk;
  double *scale64 = nullptr;            // per node weight of the summed correction
  float *scale32 = nullptr;
  // V-cycle work vectors (one precision is allocated)
  double *r64 = nullptr, *x64 = nullptr, *d64 = nullptr, *Y64 = nullptr;
  float *r32 = nullptr, *x32 = nullptr, *d32 = nullptr, *Y32 = nullptr;
  // coarsest level: dense FP64 inverse restricted to the non-identity dofs
  int64_t nfree = 0;
  int32_t *cfree = nullptr;             // [nfree] free dof -> dof
  int32_t *cidx = nullptr;              // [n] dof -> free index or -1
  double *cinv = nullptr;               // [nfree*nfree]
  double *ct0 = nullptr, *ct1 = nullptr;  // FP64 coarse work vectors (mixed mode casts)
  // Gauss-Jordan workspace of the coarse factorisation, allocated with the
  // hierarchy so that refactoring never allocates
  double *gj_a = nullptr, *gj_rowk = nullptr, *gj_colk = nullptr, *gj_part = nullptr;
  int *gj_piv = nullptr, *gj_colmap = nullptr;
  // block ILU(0) smoother (smoother == ILU): factors in the matrix's layout
  // (L strictly left of the diagonal block, U from it on), inverses of the
  // diagonal blocks of U, and the level schedules of the lower and upper
  // triangles (rows of one level are independent)
  double *ilu64 = nullptr, *dinv64 = nullptr;
  float *ilu32 = nullptr, *dinv32 = nullptr;
  double *iw64 = nullptr;               // triangular-solve work vector (one precision)
  float *iw32 = nullptr;
  int32_t *idiag = nullptr;             // [nrows] position of the diagonal block
  int32_t *lorder = nullptr, *uorder = nullptr;  // [nrows] rows sorted by level
  std::vector<int64_t> lptr, uptr;      // host: level boundaries in lorder / uorder
  int ilu_maxrow = 0;                   // longest block row (LDS of the factorisation)
  hipGraphExec_t ilu_exec[2] = {nullptr, nullptr};  // captured sweeps (FP64, FP32)
};

// ------------------------------------------------- batched execution
// Device view of one level of one instance (hierarchy) for the batched
// kernels: every batched launch covers one level of many instances.
struct DLev {
  const int32_t *rowptr, *colind;
  const double *v64;
  const float *v32;
  const uint8_t *mask;
  int64_t nrows, n;
  int cells[4];
  int64_t npatch;
  const int32_t *pnodes;
  const double *inv64;
  const float *inv32;
  int64_t npatch2, yofs2;   // block patches (second group)
  const int32_t *pnodes2;
  const double *inv64_2;
  const float *inv32_2;
  const int32_t *gptr, *gidx;
  const double *sc64;
  const float *sc32;
  double *r64, *x64, *d64, *Y64;
  float *r32, *x32, *d32, *Y32;
  int64_t nfree;
  const int32_t *cfree;
  const double *cinv;
  double *ct0, *ct1;
};

// Krylov state of one instance (FP64): basis V, preconditioned directions
// Z, work vector w, reduction partials, and the caller's b / x.
struct DKry {
  double *V, *Z, *w, *partial;
  const double *b;
  double *x;
  int64_t n;
  int nblk;  // reduction blocks of this instance (depends on n only)
  int pad;
};

// One batched launch: the instances it covers and the prefix sums of their
// work blocks (pre[s] = first block of instance inst[s]).
struct WorkSet {
  const int32_t *inst;
  const int64_t *pre;
  int nset;
  int64_t nblocks;
};

constexpr int kHS = 160;  // per-instance small vector: h1[32] h2[32] h[32] ss y[32]
constexpr int kOffH1 = 0, kOffH2 = 32, kOffH = 64, kOffSS = 96, kOffY = 128;

int krylov_blocks(int64_t n);  // reduction blocks of a vector of length n

// FGMRES control state of one instance, kept on the device and written only by
// the kb_kry_* kernels: the counters and outcome the host reads after the
// solve, then the least-squares data of the current restart cycle (rotated
// Hessenberg columns R, column j at R[j * kMaxVec + r] for r <= j, the Givens
// rotations and the rotated right-hand side g).
struct DGiv {
  double beta0, tol, rnorm;   // ||r_0||, stop threshold rtol ||r_0||, last true residual
  double rprev;               // the previous iteration's residual estimate
  int it, k, restarts, status;
  int nhist, incyc, maxit, pad;
  double hist[FSIMG_HIST];    // |g_{j+1}| / ||r_0|| after each of the first iterations
  double cs[kMaxVec], sn[kMaxVec], g[kMaxVec + 1];
  double R[kMaxVec * kMaxVec];
};

enum BatchSpmvSrc { BS_VCYCLE = 0, BS_AZ = 1, BS_RESID = 2 };

// rpw: block rows per wavefront (the work set counts workgroups of 4 * rpw rows)
template <typename T>
void launch_b_spmv(int b, int src, int rpw, const DLev *lev, const DKry *kry, const int *active,
                   const WorkSet &ws, int j, hipStream_t s);
// ppw: patches per workgroup (the work set counts workgroups of ppw patches);
// zj >= 0: the gather also writes z_zj = x in FP64 (kry[i].Z, finest level)
template <typename T>
void launch_b_vanka(int np, int b, int nl, int npc, int ppw, T omega, bool first, bool assign,
                    const DLev *lev, const int *active, const WorkSet &wp, const WorkSet &wg,
                    hipStream_t s, hipEvent_t e0, hipEvent_t e1, const DKry *kry = nullptr,
                    int zj = -1);
// the block-patch group's local corrections (before launch_b_vanka's gather)
template <typename T>
void launch_b_vanka_blocks(int np, int b, int nl, int npc, int ppw, bool first, const DLev *lev,
                           const int *active, const WorkSet &wp, hipStream_t s);
template <typename T>
void launch_b_fill_x(const DLev *lev, const int *active, const WorkSet &ws, hipStream_t s);
// 3D: the work set counts tiles (restrict3_blocks of the coarse level), 2D
// workgroups of 256 coarse nodes
template <typename T>
void launch_b_restrict(int b, int dim, const DLev *levF, const DLev *levC, const int *active,
                       const WorkSet &ws, hipStream_t s);
int64_t restrict3_blocks(int cx, int cy, int cz);
// the levels of each listed instance below tfrom[i] in one workgroup of
// tail_threads<T>() threads (kb_vcycle_tail): up = false pre-smooths, forms
// the residual and restricts on levels tfrom[i] .. coarse - 1; up = true
// prolongs and post-smooths them bottom up
template <typename T>
constexpr int tail_threads() { return sizeof(T) == 8 ? 512 : 1024; }
template <typename T>
void launch_b_tail(int b, int dim, const DLev *lev, int n, const int *active, const int32_t *tinst,
                   int ninst, const int32_t *tfrom, int coarse, bool up, int np, int npc, int nl,
                   int np2, int npc2, int nl2, T omega, int nu_pre, int nu_post, hipStream_t s);
template <typename T>
void launch_b_prolong(int b, int dim, const DLev *levF, const DLev *levC, const int *active,
                      const WorkSet &ws, hipStream_t s);
template <typename T>
void launch_b_coarse(const DLev *lev, const int *active, const WorkSet &wn, const WorkSet &wf,
                     hipStream_t s);
template <typename T>
void launch_b_copy_in(const DLev *lev0, const DKry *kry, const int *active, const WorkSet &ws,
                      int j, hipStream_t s);
template <typename T>
void launch_b_copy_out(const DLev *lev0, const DKry *kry, const int *active, const WorkSet &ws,
                       int j, hipStream_t s);
// Krylov reductions: each instance's nblk workgroups write partials and the
// last one to finish (counted in cnt[i], zero between passes) sums them in
// a fixed order into hs[i kHS + off ..]
// V[0..nvec)^T w, or w.w (norm_w)
void launch_b_multidot(const DKry *kry, const int *active, const WorkSet &wk, int nvec, bool norm_w,
                       double *hs, int off, int *cnt, hipStream_t s);
// w -= V h with h = hs[hoff ..], then V^T w or w.w (norm); with norm and
// gv != nullptr the Givens step of FGMRES column j (h = h1 + h2, stop test)
void launch_b_axpy_red(const DKry *kry, int *active, const WorkSet &wk, int nvec, bool norm, double *hs,
                       int hoff, int off, int *cnt, DGiv *gv, int j, hipStream_t s);
// V[target] = w / sqrt(hs[kOffSS]), also into the finest level's r in T
template <typename T>
void launch_b_scale(const DKry *kry, const int *active, const WorkSet &wv, const double *hs,
                    int target, const DLev *lev0, hipStream_t s);
void launch_b_combine(const DKry *kry, const int *active, const WorkSet &wv, const double *hs,
                      const int *kcnt, int kmax, hipStream_t s);
void launch_b_nonfinite(const DKry *kry, const int *active, const WorkSet &wv, int *flags,
                        hipStream_t s);
void launch_b_activate(int *active, int n, hipStream_t s);  // active[0..n) = 1
// device-side FGMRES control, one thread per instance (see DGiv):
// reset: active = 1, flags = 0 and the reduction counters 0 before the first residual
void launch_kry_reset(int *active, int *flags, int *cnt, int n, hipStream_t s);
// start: beta0 = ||r_0|| from hs[kOffSS]; an instance with a non-finite or
// zero residual is done; the others open their first cycle (active = cyc = 1)
void launch_kry_start(DGiv *gv, const double *hs, const int *flags, int *active, int *cyc, int n,
                      double rtol, int max_iter, hipStream_t s);
// (the Givens step of iteration j runs in the last workgroup of its w.w
// pass, launch_b_axpy_red: active = 0 once |g_{j+1}| <= tol, max_iter is
// reached, the column breaks down (h_{j+1,j} = 0) or g is not finite; else
// active = 2 when the next iteration is expected to stop it (the last
// residual reduction factor repeated reaches tol, or max_iter is next),
// 1 otherwise; kernels treat any non-zero value as active)
// end of a cycle: y = R^-1 g into hs[kOffY..], kcnt = k; active = in cycle
void launch_kry_ysolve(DGiv *gv, double *hs, int *active, int *kcnt, int n, hipStream_t s);
// after the true residual: stop test, next cycle's g; active = cyc = continues
void launch_kry_restart(DGiv *gv, const double *hs, int *active, int *cyc, int n, hipStream_t s);

// ---------------------------------------------------------------- kernels
template <typename T>
void launch_bsr_spmv(const DevLevel &L, const T *vals, const T *x, const T *b, T *y, bool resid,
                     hipStream_t s);
template <typename T>
void launch_vanka_patch(const DevLevel &L, const T *inv, int npc, const T *d, T *Y, int64_t p0,
                        int64_t p1, bool scatter, T *x, const T *scale, T omega, hipStream_t s);
// threads of a Vanka workgroup holding ppw patches of np rows (whole waves)
inline int vanka_threads(int np, int ppw) { return (ppw * np + 63) / 64 * 64; }
// default patches per workgroup: the fewest idle lanes (ties: smaller group)
int vanka_default_ppw(int np);
// SpMV with an explicit shape (for the tuner's measurements)
template <typename T>
void launch_bsr_spmv_rpw(const DevLevel &L, const T *vals, const T *x, const T *b, T *y,
                         bool resid, int rpw, hipStream_t s);
// all patches of group grp (0 element, 1 block) with ppw patches per workgroup
template <typename T>
void launch_vanka_patch_ppw(const DevLevel &L, int grp, const T *inv, int npc, const T *d, T *Y,
                            int ppw, hipStream_t s);
// the block patches' local corrections into Y (= the level's Y + L.blk.yofs)
template <typename T>
void launch_vanka_blocks(const DevLevel &L, const T *inv, int npc, const T *d, T *Y,
                         hipStream_t s);
template <typename T>
void launch_vanka_gather(const DevLevel &L, const T *Y, const T *scale, T omega, bool assign, T *x,
                         hipStream_t s);
// block ILU(0): factor level L in place (ilu64 = vals64 on entry, then L / U;
// dinv64 the inverted diagonal blocks of U); status[0] = 1, status[1] = row
// on a singular diagonal block
void launch_ilu_factor(const DevLevel &L, int *status, hipStream_t s);
// work = (L U)^{-1} d by the level sweeps (fixed buffers: graph-capturable)
template <typename T>
void launch_ilu_solve(const DevLevel &L, const T *F, const T *dinv, const T *d, T *work,
                      hipStream_t s);
// x (+)= omega z, identity dofs kept (assign: x = omega z, 0 at identity dofs)
template <typename T>
void launch_ilu_axpy(const DevLevel &L, const T *z, T omega, bool assign, T *x, hipStream_t s);
template <typename T>
void launch_restrict(const DevLevel &F, const DevLevel &C, const T *rf, T *rc, hipStream_t s);
template <typename T>
void launch_prolong_add(const DevLevel &F, const DevLevel &C, const T *xc, T *xf, hipStream_t s);
template <typename T>
void launch_fill(T *x, int64_t n, T v, hipStream_t s);
void launch_cast_d2f(const double *x, float *y, int64_t n, hipStream_t s);
void launch_cast_f2d(const float *x, double *y, int64_t n, hipStream_t s);
void launch_mask_zero(double *x, const uint8_t *mask, int64_t n, hipStream_t s);

// Krylov (FP64).  Two-stage deterministic reductions: per-block partials,
// then one block per output in fixed order.
void launch_multidot(const double *V, int nvec, int64_t n, const double *w, double *partial,
                     hipStream_t s);
void launch_axpy_dot(const double *V, int nvec, int64_t n, const double *h, double *w,
                     double *partial, hipStream_t s);   // w -= V h; partial of V^T w
void launch_axpy_norm(const double *V, int nvec, int64_t n, const double *h, double *w,
                      double *partial, hipStream_t s);  // w -= V h; partial of w.w
void launch_reduce_partials(const double *partial, int nvec, double *out, hipStream_t s);
void launch_add_small(const double *a, const double *b, double *out, int n, hipStream_t s);
void launch_scale_by_rsqrt(const double *w, const double *ss, double *v, int64_t n, hipStream_t s);
void launch_combine(const double *Z, int k, int64_t n, const double *y, double *x, hipStream_t s);
void launch_nonfinite_count(const double *x, int64_t n, int *flag, hipStream_t s);

// factorisation
size_t patch_factor_lds_bytes(int np);
template <typename Tout>
void launch_patch_factor(const DevLevel &L, Tout *inv, int npc, int *status, hipStream_t s);
// the block patches of L (MFMA kernel up to 128 dofs, batched Gauss-Jordan
// in L.blk.work beyond)
template <typename Tout>
void launch_patch_factor_blocks(const DevLevel &L, Tout *inv, int npc, int *status,
                                hipStream_t s);
void launch_densify(const DevLevel &L, double *dense, hipStream_t s);  // free x free block
void launch_gj_pivot(int64_t n, int64_t k, double *a, int *piv, double *rowk, double *colk,
                     double thr, int *status, hipStream_t s);
void launch_gj_update(int64_t n, int64_t k, double *a, const double *rowk, const double *colk,
                      hipStream_t s);
void launch_gj_finish(int64_t n, const double *a, const int *piv, int *colmap, double *out,
                      hipStream_t s);
// Blocked Gauss-Jordan inverse of the dense n x n matrix a (destroyed) into
// out, for n <= 4096 (returns false otherwise, launching nothing).  piv, iwork:
// int[n]; ub, rb: double[kCoarseStage * n].
bool launch_coarse_gj_blocked(int64_t n, double *a, int *piv, int *iwork, double *ub, double *rb,
                              double thr, int *status, double *out, hipStream_t s);
void launch_absmax(const double *a, int64_t n, double *partial, hipStream_t s);
void launch_coarse_gemv(const DevLevel &C, const double *x, double *y, hipStream_t s);
void launch_deform(int64_t nnodes, int dim, const uint8_t *mask, double k, double theta,
                   const double *v_new, int v_stride, int v_offset, const double *u_old,
                   const double *v_old, double *u_new, hipStream_t s);

// ------------------------------------------- element assembly (Newton loop)
// Device view of one level of the tensor Q2 mesh for the element kernels.
struct AsmLevel {
  const double *coord[3];          // per-axis node coordinates (2*cells[a]+1)
  const double *xyz;               // [nrows][D] node positions (isoparametric cells) or null
  const uint8_t *solid;            // [prod(cells)] 1 = solid cell
  const int32_t *rowptr, *colind;  // block pattern of the momentum matrix
  const uint8_t *mask;             // [nrows*(d+1)] identity rows of the momentum matrix
  int cells[3], nnode[3];
  int structured;                  // 1: the pattern is exactly the full Q2 stencil (every node
                                   // coupled with the nodes of its cells, lexicographic), so
                                   // block positions follow from the node coordinates
};
// material and time-stepping parameters (eq. aletime:2)
struct AsmPhys {
  double rho_f, nu_f, rho_s, mu_s, lambda_s, k, theta, alpha0;
};
// a state: x = (p, v) per node [nrows*(d+1)], u [nrows*d]; x_old, u_old at t_{n-1}
struct AsmState {
  const double *x, *u, *xo, *uo;
};
// the approximate Jacobian into vals [nnzb*(d+1)^2] (zeroed first, identity
// rows and columns of L.mask applied); flag[0] = 1 if det F <= 0 at a Gauss
// point, flag[1] = 1 if the pattern lacks an element coupling.  ev (nullable):
// 2 events per parity colour, recorded around that colour's launch
void launch_asm_jacobian(const AsmLevel &L, int dim, const AsmPhys &P, const AsmState &S,
                         double *vals, int64_t nrows, int64_t nnzb, int *flag, hipStream_t s,
                         hipEvent_t *ev = nullptr);
// res = -A(U) (zero at identity rows), flags and events as above
void launch_asm_residual(const AsmLevel &L, int dim, const AsmPhys &P, const AsmState &S,
                         double *res, int64_t nrows, int *flag, hipStream_t s,
                         hipEvent_t *ev = nullptr);
void launch_inject(const double *f, double *c, const int *nnode_f, const int *nnode_c, int comps,
                   hipStream_t s);
void launch_axpy_to(const double *x, const double *z, double omega, double *y, int64_t n,
                    hipStream_t s);
void launch_neg_free(double *y, const uint8_t *mask, int64_t n, hipStream_t s);
void launch_absmax_u64(const double *x, int64_t n, unsigned long long *out, hipStream_t s);
// *bad = 1 unless L's block pattern is exactly the full Q2 stencil of its mesh
void launch_check_structured(const AsmLevel &L, int dim, int64_t nrows, int *bad, hipStream_t s);
// r = u_old + k theta v + k (1 - theta) v_old - u at mask nodes, 0 elsewhere
void launch_cond_residual(int64_t nnodes, int dim, const uint8_t *mask, double k, double theta,
                          const double *x, const double *xo, const double *u, const double *uo, double *r,
                          hipStream_t s);

}  // namespace fsimg
