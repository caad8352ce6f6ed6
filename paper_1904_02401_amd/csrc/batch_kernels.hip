// Batched kernels: one launch covers one operation on one multigrid level of
// many independent instances (hierarchies of uneven size).  A workgroup finds
// its instance by binary search in the launch's prefix of work blocks; every
// per-instance computation (rows, patches, nodes, reduction blocking) depends
// on that instance alone, so an instance's result does not depend on which
// other instances share the launch.
#include <algorithm>
#include <type_traits>

#include "device_ops.h"

namespace fsimg {

namespace {

using dev::kWave;

__device__ __forceinline__ int seg_of(const WorkSet &ws, int64_t blk) {
  int lo = 0, hi = ws.nset - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ws.pre[mid] <= blk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T> struct LV;
template <> struct LV<double> {
  static __device__ __forceinline__ const double *vals(const DLev &L) { return L.v64; }
  static __device__ __forceinline__ double *r(const DLev &L) { return L.r64; }
  static __device__ __forceinline__ double *x(const DLev &L) { return L.x64; }
  static __device__ __forceinline__ double *d(const DLev &L) { return L.d64; }
  static __device__ __forceinline__ double *Y(const DLev &L) { return L.Y64; }
  static __device__ __forceinline__ const double *inv(const DLev &L) { return L.inv64; }
  static __device__ __forceinline__ const double *inv2(const DLev &L) { return L.inv64_2; }
  static __device__ __forceinline__ const double *sc(const DLev &L) { return L.sc64; }
};
template <> struct LV<float> {
  static __device__ __forceinline__ const float *vals(const DLev &L) { return L.v32; }
  static __device__ __forceinline__ float *r(const DLev &L) { return L.r32; }
  static __device__ __forceinline__ float *x(const DLev &L) { return L.x32; }
  static __device__ __forceinline__ float *d(const DLev &L) { return L.d32; }
  static __device__ __forceinline__ float *Y(const DLev &L) { return L.Y32; }
  static __device__ __forceinline__ const float *inv(const DLev &L) { return L.inv32; }
  static __device__ __forceinline__ const float *inv2(const DLev &L) { return L.inv32_2; }
  static __device__ __forceinline__ const float *sc(const DLev &L) { return L.sc32; }
};

// ------------------------------------------------------------ SpMV
// SRC BS_VCYCLE: d = r - A x on the level's work vectors (T);
//     BS_AZ:     w = A z_j, 0 at identity rows (FP64, level 0);
//     BS_RESID:  w = b - A x with the caller's b, x (FP64, level 0).
template <int B, typename T, int SRC, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void kb_spmv(const DLev *__restrict__ lev,
                                               const DKry *__restrict__ kry,
                                               const int *__restrict__ active, WorkSet ws, int j) {
  const int64_t lb = dev::xcd_block(blockIdx.x, gridDim.x);
  const int s = seg_of(ws, lb);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DLev &L = lev[i];
  const int lane = threadIdx.x & (kWave - 1);
  constexpr int GR = spmv_group_rows(B, SRC == BS_VCYCLE ? (int)sizeof(T) : 8);
  const int64_t row0 = ((lb - ws.pre[s]) * 4 + threadIdx.x / kWave) * R * GR;
  if (row0 >= L.nrows) return;
  if constexpr (SRC == BS_VCYCLE) {
    dev::spmv_rows<B, T, 1, R>(row0, L.nrows, lane, L.rowptr, L.colind, LV<T>::vals(L),
                               LV<T>::x(L), LV<T>::r(L), L.mask, LV<T>::d(L));
  } else if constexpr (SRC == BS_AZ) {
    const DKry &K = kry[i];
    dev::spmv_rows<B, double, 2, R>(row0, L.nrows, lane, L.rowptr, L.colind, L.v64,
                                    K.Z + (int64_t)j * K.n, nullptr, L.mask, K.w);
  } else {
    const DKry &K = kry[i];
    dev::spmv_rows<B, double, 1, R>(row0, L.nrows, lane, L.rowptr, L.colind, L.v64, K.x, K.b,
                                    L.mask, K.w);
  }
}

// ------------------------------------------------------------ Vanka
// grp 0: element patches; grp 1: block patches (corrections at Y + yofs2)
template <typename T>
__global__ __launch_bounds__(1024) void kb_vanka_patch(const DLev *__restrict__ lev,
                                                       const int *__restrict__ active, WorkSet ws,
                                                       int np, int npc, int b, int nl, int ppw,
                                                       int first, int grp) {
  extern __shared__ unsigned char smem_raw[];
  const int64_t lb = dev::xcd_block(blockIdx.x, gridDim.x);
  const int s = seg_of(ws, lb);
  const int i = ws.inst[s];
  if (!active[i]) return;  // uniform per workgroup
  const DLev &L = lev[i];
  const int64_t pfirst = (lb - ws.pre[s]) * ppw;
  const bool g2 = grp != 0;
  dev::vanka_patch_wg<T>(pfirst, g2 ? L.npatch2 : L.npatch, np, npc, b, nl, ppw,
                         g2 ? L.pnodes2 : L.pnodes, g2 ? LV<T>::inv2(L) : LV<T>::inv(L),
                         first ? LV<T>::r(L) : LV<T>::d(L), LV<T>::Y(L) + (g2 ? L.yofs2 : 0), 0,
                         nullptr, nullptr, L.mask, T(0), reinterpret_cast<T *>(smem_raw));
}

// One dof of the additive Vanka update, the sum of dev::vanka_gather_dof
// (same order, same bits) with the node's first 8 slot indices, and then
// their values, requested before any is summed: two round trips per wave
// instead of two per slot (a Q2 vertex node lies in 8 element patches);
// slots past the 8th, where block patches add some, follow in a loop.
template <typename T>
__device__ __forceinline__ void gather_dof(int64_t dof, int b, const int32_t *gptr_, const int32_t *gidx_,
                                           const T *Y_, const T *scale_, const uint8_t *mask_, T omega,
                                           int assign, T *x_) {
  const dev::gptr<const int32_t> gp = dev::glb(gptr_), gidx = dev::glb(gidx_);
  const dev::gptr<const T> Y = dev::glb(Y_), scale = dev::glb(scale_);
  const dev::gptr<T> x = dev::glb(x_);
  const int64_t node = dof / b;
  const int c = (int)(dof - node * b);
  const int e0 = gp[node], e1 = gp[node + 1], ne = e1 - e0;
  int32_t g[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) g[q] = q < ne ? gidx[e0 + q] : 0;
  T y[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) y[q] = q < ne ? Y[(int64_t)g[q] * b + c] : T(0);
  T s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (q < ne) s += y[q];
  for (int e = e0 + 8; e < e1; ++e) s += Y[(int64_t)gidx[e] * b + c];
  const T xv = assign ? T(0) : x[dof];
  x[dof] = dev::glb(mask_)[dof] ? xv : xv + omega * scale[node] * s;
}

// zj >= 0 (the last post-smoothing step on the finest level): also z_j =
// the updated x in FP64, the FGMRES direction of iteration zj
template <typename T>
__global__ __launch_bounds__(256) void kb_vanka_gather(const DLev *__restrict__ lev,
                                                       const int *__restrict__ active, WorkSet ws,
                                                       int b, T omega, int assign,
                                                       const DKry *__restrict__ kry, int zj) {
  const int64_t lb = dev::xcd_block(blockIdx.x, gridDim.x);
  const int s = seg_of(ws, lb);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DLev &L = lev[i];
  const int64_t dof = (lb - ws.pre[s]) * 256 + threadIdx.x;
  if (dof >= L.n) return;
  gather_dof<T>(dof, b, L.gptr, L.gidx, LV<T>::Y(L), LV<T>::sc(L), L.mask, omega, assign, LV<T>::x(L));
  if (zj >= 0) {
    const DKry &K = kry[i];
    K.Z[(int64_t)zj * K.n + dof] = (double)LV<T>::x(L)[dof];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void kb_fill_x(const DLev *__restrict__ lev,
                                                 const int *__restrict__ active, WorkSet ws) {
  const int s = seg_of(ws, blockIdx.x);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DLev &L = lev[i];
  const int64_t k = (blockIdx.x - ws.pre[s]) * 256 + threadIdx.x;
  if (k < L.n) LV<T>::x(L)[k] = T(0);
}

// ------------------------------------------------------------ transfers
template <int B, int DIM, typename T>
__global__ __launch_bounds__(256) void kb_restrict(const DLev *__restrict__ levF,
                                                   const DLev *__restrict__ levC,
                                                   const int *__restrict__ active, WorkSet ws) {
  const int s = seg_of(ws, blockIdx.x);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DLev &C = levC[i];
  const int64_t node = (blockIdx.x - ws.pre[s]) * 256 + threadIdx.x;
  if (node >= C.nrows) return;
  dev::restrict_node<B, DIM, T>(node, C.cells[0], C.cells[1], C.cells[2], LV<T>::d(levF[i]),
                                LV<T>::r(C), C.mask);
}

// 3D restriction by slabs: a workgroup owns one coarse plane Z and a slab of
// at most kRTY coarse rows by at most kRTXM coarse columns (the columns of a
// row split evenly over the fewest slabs).  Each thread first restricts
// along z for the fine (x, y) positions of the slab and its 3-node halo (the
// <= 5 fine planes coarse plane Z reaches, loads independent of one another)
// into LDS; after one barrier each coarse node of the slab sums the <= 5 x 5
// x-y taps from LDS.  No sequential walk over planes: every load of a
// workgroup is in flight at once, and the grid has NZ * slabs workgroups.
constexpr int kRTXM = 64, kRTY = 4;

__host__ __device__ inline void restrict3_slabs(int NX, int NY, int &ntx, int &wx, int &nty) {
  ntx = (NX + kRTXM - 1) / kRTXM;
  wx = (NX + ntx - 1) / ntx;
  nty = (NY + kRTY - 1) / kRTY;
}

// the fine taps of coarse node I along one axis (fine nodes 0 .. nf-1) in
// five fixed slots: a vertex reaches 2I, 2I +- 1, 2I +- 3, a mid node 2I,
// 2I +- 1; a slot outside the mesh or unused points at 2I with weight 0, so
// every index stays in range and the slots live in registers
template <typename T>
__device__ __forceinline__ void taps_1d(int I, int nf, int *f, T *w) {
  const bool vtx = (I & 1) == 0;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const int d = q == 0 ? 0 : (q == 1 ? -1 : (q == 2 ? 1 : (q == 3 ? -3 : 3)));
    const T wv = q == 0 ? T(1) : (q < 3 ? T(0.375) : T(-0.125));
    const T wm = q == 0 ? T(1) : (q < 3 ? T(0.75) : T(0));
    const int g = 2 * I + d;
    const bool ok = g >= 0 && g < nf;
    f[q] = ok ? g : 2 * I;
    w[q] = ok ? (vtx ? wv : wm) : T(0);
  }
}

template <int B, typename T>
__global__ __launch_bounds__(256) void kb_restrict3(const DLev *__restrict__ levF,
                                                    const DLev *__restrict__ levC,
                                                    const int *__restrict__ active, WorkSet ws) {
  constexpr int FYW = 2 * kRTY + 5, FXWM = 2 * kRTXM + 5;
  __shared__ T s_f[FYW * FXWM * B];  // z-restricted fine rows of the slab and halo
  const int64_t lb = dev::xcd_block(blockIdx.x, gridDim.x);
  const int sg = seg_of(ws, lb);
  const int inst = ws.inst[sg];
  if (!active[inst]) return;  // uniform per workgroup
  const DLev &C = levC[inst];
  const DLev &F = levF[inst];
  const int NX = 2 * C.cells[0] + 1, NY = 2 * C.cells[1] + 1;
  const int FX = 4 * C.cells[0] + 1, FY = 4 * C.cells[1] + 1, FZ = 4 * C.cells[2] + 1;
  int ntx, wx, nty;
  restrict3_slabs(NX, NY, ntx, wx, nty);
  int64_t blk = lb - ws.pre[sg];
  const int ty = (int)(blk % nty);
  blk /= nty;
  const int tx = (int)(blk % ntx), Z = (int)(blk / ntx);
  const int X0 = tx * wx, Y0 = ty * kRTY;
  const int X1 = X0 + wx < NX ? X0 + wx : NX, Y1 = Y0 + kRTY < NY ? Y0 + kRTY : NY;
  const int fx0 = 2 * X0 - 3, fy0 = 2 * Y0 - 3, fxw = 2 * (X1 - X0) + 5;
  const int t = threadIdx.x;
  const T *rf = LV<T>::d(F);
  T *rc = LV<T>::r(C);
  int fzt[5];
  T wzt[5];
  taps_1d<T>(Z, FZ, fzt, wzt);
#pragma unroll 2
  for (int it = t; it < FYW * fxw; it += 256) {
    const int yy = it / fxw, xx = it - yy * fxw;
    const int gx = fx0 + xx, gy = fy0 + yy;
    T a[B];
#pragma unroll
    for (int c = 0; c < B; ++c) a[c] = T(0);
    if (gx >= 0 && gx < FX && gy >= 0 && gy < FY) {
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        if (wzt[q] != T(0)) {  // uniform: the slab's plane Z decides
          const T *src = rf + (((int64_t)fzt[q] * FY + gy) * FX + gx) * B;
#pragma unroll
          for (int c = 0; c < B; ++c) a[c] += wzt[q] * src[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < B; ++c) s_f[it * B + c] = a[c];
  }
  __syncthreads();
  const int nxs = X1 - X0;
  for (int p = t; p < (Y1 - Y0) * nxs; p += 256) {
    const int ly = p / nxs, lx = p - ly * nxs;
    const int X = X0 + lx, Y = Y0 + ly;
    int fxt[5], fyt[5];
    T wxt[5], wyt[5];
    taps_1d<T>(X, FX, fxt, wxt);
    taps_1d<T>(Y, FY, fyt, wyt);
    T v[B];
#pragma unroll
    for (int c = 0; c < B; ++c) v[c] = T(0);
#pragma unroll
    for (int qy = 0; qy < 5; ++qy) {
      const T *row = s_f + (fyt[qy] - fy0) * fxw * B;
      T h[B];
#pragma unroll
      for (int c = 0; c < B; ++c) h[c] = T(0);
#pragma unroll
      for (int qx = 0; qx < 5; ++qx) {
        const T *e = row + (fxt[qx] - fx0) * B;
#pragma unroll
        for (int c = 0; c < B; ++c) h[c] += wxt[qx] * e[c];
      }
#pragma unroll
      for (int c = 0; c < B; ++c) v[c] += wyt[qy] * h[c];
    }
    const int64_t node = ((int64_t)Z * NY + Y) * NX + X;
#pragma unroll
    for (int c = 0; c < B; ++c) {
      const int64_t dof = node * B + c;
      rc[dof] = C.mask[dof] ? T(0) : v[c];
    }
  }
}

// one coarse node of the 3D restriction with the slab kernel's summation
// order (z taps, then x, then y), so both give the same bits
template <int B, typename T>
__device__ __forceinline__ void restrict3_node(int64_t node, const DLev &C, const T *rf_, T *rc_) {
  const dev::gptr<const T> rf = dev::glb(rf_);
  const dev::gptr<T> rc = dev::glb(rc_);
  const dev::gptr<const uint8_t> mask = dev::glb(C.mask);
  const int NX = 2 * C.cells[0] + 1, NY = 2 * C.cells[1] + 1;
  const int FX = 4 * C.cells[0] + 1, FY = 4 * C.cells[1] + 1, FZ = 4 * C.cells[2] + 1;
  const int X = (int)(node % NX), Y = (int)((node / NX) % NY), Z = (int)(node / ((int64_t)NX * NY));
  int fxt[5], fyt[5], fzt[5];
  T wxt[5], wyt[5], wzt[5];
  taps_1d<T>(X, FX, fxt, wxt);
  taps_1d<T>(Y, FY, fyt, wyt);
  taps_1d<T>(Z, FZ, fzt, wzt);
  T v[B];
#pragma unroll
  for (int c = 0; c < B; ++c) v[c] = T(0);
#pragma unroll 1
  for (int qy = 0; qy < 5; ++qy) {
    T h[B];
#pragma unroll
    for (int c = 0; c < B; ++c) h[c] = T(0);
#pragma unroll 1
    for (int qx = 0; qx < 5; ++qx) {
      T a[B];
#pragma unroll
      for (int c = 0; c < B; ++c) a[c] = T(0);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        if (wzt[q] != T(0)) {
          const dev::gptr<const T> src = rf + (((int64_t)fzt[q] * FY + fyt[qy]) * FX + fxt[qx]) * B;
#pragma unroll
          for (int c = 0; c < B; ++c) a[c] += wzt[q] * src[c];
        }
      }
#pragma unroll
      for (int c = 0; c < B; ++c) h[c] += wxt[qx] * a[c];
    }
#pragma unroll
    for (int c = 0; c < B; ++c) v[c] += wyt[qy] * h[c];
  }
#pragma unroll
  for (int c = 0; c < B; ++c) {
    const int64_t dof = node * B + c;
    rc[dof] = mask[dof] ? T(0) : v[c];
  }
}

// ------------------------------------------------------------ small levels
// The levels of an instance from tfrom[i] down to (excluding) its coarsest
// level `coarse`, in one workgroup per instance (1024 threads in FP32, 512 in
// FP64, where the register budget of 1024 threads would spill): every step
// of the V-cycle there (Vanka sweeps, residuals, transfers) as a loop of the
// same per-row / per-patch / per-dof device bodies the level-wide kernels
// run, with workgroup barriers between the steps instead of kernel
// boundaries.  A row, patch or dof is computed by the same lanes in the same
// order as in the level-wide kernels, so the results are the same bits.
// up = 0: pre-smoothing, residual and restriction of each level, top down;
// up = 1: prolongation and post-smoothing of each level, bottom up.  The
// coarse solve runs between the two launches.
template <int B, int DIM, typename T>
__device__ __forceinline__ void tail_residual(const DLev &F) {
  constexpr int GR = spmv_group_rows(B, (int)sizeof(T));
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nw = blockDim.x / kWave;
  for (int64_t row0 = (int64_t)(threadIdx.x / kWave) * GR; row0 < F.nrows; row0 += nw * GR)
    dev::spmv_rows<B, T, 1, 1>(row0, F.nrows, lane, F.rowptr, F.colind, LV<T>::vals(F), LV<T>::x(F),
                               LV<T>::r(F), F.mask, LV<T>::d(F));
  __syncthreads();
}

template <int B, typename T>
__device__ __forceinline__ void tail_smooth(const DLev &F, int np, int npc, int nl, int np2, int npc2,
                                            int nl2, T omega, bool first, T *dl) {
  const T *dsrc = first ? LV<T>::r(F) : LV<T>::d(F);
  if (F.npatch2 > 0) {  // block patches first, as the level-wide launches
    const int ppw = (int)blockDim.x / np2;
    for (int64_t pf = 0; pf < F.npatch2; pf += ppw) {
      dev::vanka_patch_wg<T>(pf, F.npatch2, np2, npc2, B, nl2, ppw, F.pnodes2, LV<T>::inv2(F), dsrc,
                             LV<T>::Y(F) + F.yofs2, 0, nullptr, nullptr, F.mask, T(0), dl);
      __syncthreads();
    }
  }
  if (F.npatch > 0) {
    const int ppw = (int)blockDim.x / np;
    for (int64_t pf = 0; pf < F.npatch; pf += ppw) {
      dev::vanka_patch_wg<T>(pf, F.npatch, np, npc, B, nl, ppw, F.pnodes, LV<T>::inv(F), dsrc,
                             LV<T>::Y(F), 0, nullptr, nullptr, F.mask, T(0), dl);
      __syncthreads();
    }
  }
  for (int64_t dof = threadIdx.x; dof < F.n; dof += blockDim.x)
    dev::vanka_gather_dof<T>(dof, B, F.gptr, F.gidx, LV<T>::Y(F), LV<T>::sc(F), F.mask, omega,
                             first ? 1 : 0, LV<T>::x(F));
  __syncthreads();
}

template <int B, int DIM, typename T>
__global__ __launch_bounds__(tail_threads<T>()) void kb_vcycle_tail(const DLev *__restrict__ lev, int n,
                                                       const int *__restrict__ active,
                                                       const int32_t *__restrict__ tinst,
                                                       const int32_t *__restrict__ tfrom, int coarse,
                                                       int up, int np, int npc, int nl, int np2,
                                                       int npc2, int nl2, T omega, int nu_pre,
                                                       int nu_post) {
  extern __shared__ unsigned char smem_raw[];
  T *dl = reinterpret_cast<T *>(smem_raw);
  const int i = tinst[blockIdx.x];
  if (!active[i]) return;  // uniform per workgroup
  const int l0 = tfrom[i];
  if (!up) {
    for (int l = l0; l < coarse; ++l) {
      const DLev &F = lev[(size_t)l * n + i];
      if (nu_pre == 0) {
        for (int64_t k = threadIdx.x; k < F.n; k += blockDim.x) LV<T>::x(F)[k] = T(0);
        __syncthreads();
      }
      for (int k = 0; k < nu_pre; ++k) {
        if (k > 0) tail_residual<B, DIM, T>(F);
        tail_smooth<B, T>(F, np, npc, nl, np2, npc2, nl2, omega, k == 0, dl);
      }
      tail_residual<B, DIM, T>(F);
      const DLev &C = lev[(size_t)(l + 1) * n + i];
      for (int64_t node = threadIdx.x; node < C.nrows; node += blockDim.x) {
        if constexpr (DIM == 3)
          restrict3_node<B, T>(node, C, LV<T>::d(F), LV<T>::r(C));
        else
          dev::restrict_node<B, DIM, T>(node, C.cells[0], C.cells[1], C.cells[2], LV<T>::d(F),
                                        LV<T>::r(C), C.mask);
      }
      __syncthreads();
    }
  } else {
    for (int l = coarse - 1; l >= l0; --l) {
      const DLev &F = lev[(size_t)l * n + i];
      const DLev &C = lev[(size_t)(l + 1) * n + i];
      for (int64_t node = threadIdx.x; node < F.nrows; node += blockDim.x)
        dev::prolong_node<B, DIM, T>(node, C.cells[0], C.cells[1], C.cells[2], LV<T>::x(C), LV<T>::x(F),
                                     F.mask);
      __syncthreads();
      for (int k = 0; k < nu_post; ++k) {
        tail_residual<B, DIM, T>(F);
        tail_smooth<B, T>(F, np, npc, nl, np2, npc2, nl2, omega, false, dl);
      }
    }
  }
}

// b = 4: the sums of dev::prolong_node, with the node's four components moved by one 16-byte
// load per coarse tap (two in FP64), one load and one store of the fine
// values and one 4-byte load of the mask bytes
template <int DIM, typename T>
__device__ __forceinline__ void prolong_node4(int64_t node, int cx, int cy, int cz,
                                              const T *xc_, T *xf_, const uint8_t *maskf_) {
  using V = typename dev::Vec16<T>::type;
  constexpr int G = dev::Vec16<T>::G, NV = 4 / G;
  const dev::gptr<const V> xc = reinterpret_cast<dev::gptr<const V>>(dev::glb(xc_));
  const dev::gptr<V> xf = reinterpret_cast<dev::gptr<V>>(dev::glb(xf_));
  const dev::gptr<const uint32_t> maskf = reinterpret_cast<dev::gptr<const uint32_t>>(dev::glb(maskf_));
  const int NX = 2 * cx + 1, NY = 2 * cy + 1;
  const int FX = 4 * cx + 1, FY = 4 * cy + 1;
  // block-row offsets are int32, so a level has fewer than 2^31 nodes and
  // 32-bit division gives the node's grid position
  const uint32_t nd = (uint32_t)node, ij = nd / (uint32_t)FX;
  const int i = (int)(nd - ij * (uint32_t)FX), j = (int)(ij % (uint32_t)FY), k = (int)(ij / (uint32_t)FY);
  int ix[3], iy[3], iz[3];
  T wx[3], wy[3], wz[3];
  const int nx = dev::prolong_1d<T>(i, ix, wx), ny = dev::prolong_1d<T>(j, iy, wy);
  int nz = 1;
  iz[0] = 0; wz[0] = T(1);
  if (DIM == 3) nz = dev::prolong_1d<T>(k, iz, wz);
  T acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = 0;
  for (int a = 0; a < nz; ++a)
    for (int bb = 0; bb < ny; ++bb) {
      const T wyz = wy[bb] * wz[a];
      const int64_t base = ((int64_t)iz[a] * NY + iy[bb]) * NX;
      for (int q = 0; q < nx; ++q) {
        const T w = wyz * wx[q];
        const dev::gptr<const V> src = xc + (base + ix[q]) * NV;
#pragma unroll
        for (int h = 0; h < NV; ++h) {
          const V v = src[h];
#pragma unroll
          for (int g = 0; g < G; ++g) acc[h * G + g] += w * dev::vget(v, g);
        }
      }
    }
  const uint32_t m = maskf[node];
#pragma unroll
  for (int h = 0; h < NV; ++h) {
    V v = xf[node * NV + h];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int c = h * G + g;
      v[g] = ((m >> (8 * c)) & 0xFFu) ? T(0) : v[g] + acc[c];
    }
    xf[node * NV + h] = v;
  }
}

template <int B, int DIM, typename T>
__global__ __launch_bounds__(256) void kb_prolong(const DLev *__restrict__ levF,
                                                  const DLev *__restrict__ levC,
                                                  const int *__restrict__ active, WorkSet ws) {
  const int64_t lb = dev::xcd_block(blockIdx.x, gridDim.x);
  const int s = seg_of(ws, lb);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DLev &F = levF[i];
  const DLev &C = levC[i];
  const int64_t node = (lb - ws.pre[s]) * 256 + threadIdx.x;
  if (node >= F.nrows) return;
  if constexpr (B == 4)
    prolong_node4<DIM, T>(node, C.cells[0], C.cells[1], C.cells[2], LV<T>::x(C), LV<T>::x(F), F.mask);
  else
    dev::prolong_node<B, DIM, T>(node, C.cells[0], C.cells[1], C.cells[2], LV<T>::x(C), LV<T>::x(F),
                                 F.mask);
}

// ------------------------------------------------------------ coarse solve
// x = A_{L-1}^{-1} r in one launch: the first ceil(nfree/4) workgroups of an
// instance take a wave per row of the free-dof inverse (FP64 arithmetic; in
// mixed precision the FP32 residual is widened as it is read and the result
// rounded as it is written), the remaining ceil(n/256) zero the identity-row
// entries of x.
template <typename T>
__global__ __launch_bounds__(256) void kb_coarse_gemv(const DLev *__restrict__ lev,
                                                      const int *__restrict__ active, WorkSet ws) {
  const int s = seg_of(ws, blockIdx.x);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DLev &L = lev[i];
  const int64_t b = blockIdx.x - ws.pre[s], nrb = (L.nfree + 3) / 4;
  if (b >= nrb) {
    const int64_t k = (b - nrb) * 256 + threadIdx.x;
    if (k < L.n && L.mask[k]) LV<T>::x(L)[k] = T(0);
    return;
  }
  const int64_t row = b * 4 + threadIdx.x / kWave;
  if (row >= L.nfree) return;
  const int lane = threadIdx.x & (kWave - 1);
  const T *in = LV<T>::r(L);
  const double *ar = L.cinv + row * L.nfree;
  double acc = 0.0;
  for (int64_t c = lane; c < L.nfree; c += kWave) acc += ar[c] * (double)in[L.cfree[c]];
  acc = dev::wave_sum(acc);
  if (lane == 0) LV<T>::x(L)[L.cfree[row]] = (T)acc;
}

// ------------------------------------------------------------ Krylov
template <typename T>
__global__ __launch_bounds__(256) void kb_copy_in(const DLev *__restrict__ lev0,
                                                  const DKry *__restrict__ kry,
                                                  const int *__restrict__ active, WorkSet ws, int j) {
  const int s = seg_of(ws, blockIdx.x);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DKry &K = kry[i];
  const int64_t k = (blockIdx.x - ws.pre[s]) * 256 + threadIdx.x;
  if (k < K.n) LV<T>::r(lev0[i])[k] = (T)K.V[(int64_t)j * K.n + k];
}

template <typename T>
__global__ __launch_bounds__(256) void kb_copy_out(const DLev *__restrict__ lev0,
                                                   const DKry *__restrict__ kry,
                                                   const int *__restrict__ active, WorkSet ws, int j) {
  const int s = seg_of(ws, blockIdx.x);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DKry &K = kry[i];
  const int64_t k = (blockIdx.x - ws.pre[s]) * 256 + threadIdx.x;
  if (k < K.n) K.Z[(int64_t)j * K.n + k] = (double)LV<T>::x(lev0[i])[k];
}

// The last of an instance's nblk workgroups to finish a reduction pass.
// Partials are written and read with device-scope relaxed atomics, which this
// chip keeps coherent across its per-XCD L2 caches (write-through stores,
// loads that do not hit a stale line); each workgroup's thread 0 waits until
// its partial stores have completed before it counts itself in cnt, so the
// workgroup that counts last (and resets cnt for the next pass) reads every
// partial.  No workgroup waits for another, and no workgroup writes back or
// invalidates its L2, which a device-scope fence would do.
__device__ __forceinline__ void put_partial(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double get_partial(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool last_of(int *cnt, int nblk, int *flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);  // this thread's partial stores are complete
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const int prev = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *flag = prev == nblk - 1;
    if (*flag) __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  return *flag != 0;
}

// hsi[k] = sum over the instance's workgroups b of partial[b nvec + k], in
// workgroup order with the block-sum tree (run by the last workgroup)
__device__ __forceinline__ void sum_partials(const DKry &K, int nvec, double *hsi, double *red) {
  for (int k = 0; k < nvec; ++k) {
    double t = 0.0;
    for (int b = threadIdx.x; b < K.nblk; b += blockDim.x) t += get_partial(K.partial + (int64_t)b * nvec + k);
    t = dev::block_sum(t, red);
    if (threadIdx.x == 0) hsi[k] = t;
  }
}

// FGMRES column j after both Gram-Schmidt passes: h = h1 + h2 and
// h_{j+1,j} = sqrt(ss), rotated by the previous rotations; a new rotation,
// g, the residual history and the stop test (see DGiv)
__device__ __forceinline__ void kry_givens_step(DGiv &G, const double *hc, int j, int *act) {
  double *col = G.R + j * kMaxVec;
  for (int r = 0; r <= j; ++r) col[r] = hc[kOffH1 + r] + hc[kOffH2 + r];
  const double hn = sqrt(hc[kOffSS]);
  for (int r = 0; r < j; ++r) {
    const double a0 = col[r], a1 = col[r + 1];
    col[r] = G.cs[r] * a0 + G.sn[r] * a1;
    col[r + 1] = -G.sn[r] * a0 + G.cs[r] * a1;
  }
  const double hjj = col[j];
  const double den = hypot(hjj, hn);
  G.cs[j] = hjj / den;
  G.sn[j] = hn / den;
  col[j] = den;
  const double gj = G.g[j];
  G.g[j + 1] = -G.sn[j] * gj;
  G.g[j] = G.cs[j] * gj;
  ++G.it;
  G.k = j + 1;
  const double res = fabs(G.g[j + 1]);
  if (G.nhist < FSIMG_HIST) G.hist[G.nhist++] = res / G.beta0;
  if (!isfinite(G.g[j + 1]) || res <= G.tol || G.it >= G.maxit || hn == 0.0) {
    *act = 0;
  } else {
    const double rho = G.rprev > 0.0 ? res / G.rprev : 1.0;
    *act = (res * rho <= G.tol || G.it + 1 >= G.maxit) ? 2 : 1;
  }
  G.rprev = res;
}

// V[0..nvec)^T w (or w.w) into hs[off ..]: per-workgroup partials, summed by
// the instance's last workgroup; each instance owns nblk workgroups and
// strides over its own vector only
template <int NV, int NORM>
__global__ __launch_bounds__(256) void kb_multidot(const DKry *__restrict__ kry,
                                                   const int *__restrict__ active, WorkSet ws,
                                                   int nvec, double *__restrict__ hs, int off,
                                                   int *__restrict__ cnt) {
  __shared__ double red[4];
  __shared__ int flag;
  const int s = seg_of(ws, blockIdx.x);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DKry &K = kry[i];
  const int64_t lb = blockIdx.x - ws.pre[s];
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  const double *V = NORM ? K.w : K.V;
  const int64_t stride = (int64_t)K.nblk * 256;
  for (int64_t t = lb * 256 + threadIdx.x; t < K.n; t += stride) {
    const double wi = K.w[t];
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nvec) acc[k] += V[(int64_t)k * K.n + t] * wi;
  }
#pragma unroll
  for (int k = 0; k < NV; ++k)
    if (k < nvec) {
      const double tt = dev::block_sum(acc[k], red);
      if (threadIdx.x == 0) put_partial(K.partial + lb * nvec + k, tt);
    }
  if (last_of(cnt + i, K.nblk, &flag)) sum_partials(K, nvec, hs + (int64_t)i * kHS + off, red);
}

// w -= V h (h = hs[hoff ..]), then V^T w (NORM 0) or w.w (NORM 1) into
// hs[off ..] as kb_multidot; with NORM 1 and gv != nullptr the last
// workgroup also takes the Givens step of column j, which may clear the
// instance's active flag
template <int NV, int NORM>
__global__ __launch_bounds__(256) void kb_axpy_red(const DKry *__restrict__ kry,
                                                   int *__restrict__ active, WorkSet ws, int nvec,
                                                   double *__restrict__ hs, int hoff, int off,
                                                   int *__restrict__ cnt, DGiv *__restrict__ gv,
                                                   int j) {
  __shared__ double red[4];
  __shared__ double hv[NV];
  __shared__ int flag;
  const int s = seg_of(ws, blockIdx.x);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DKry &K = kry[i];
  if (threadIdx.x < NV) hv[threadIdx.x] = threadIdx.x < nvec ? hs[(int64_t)i * kHS + hoff + threadIdx.x] : 0.0;
  __syncthreads();
  const int64_t lb = blockIdx.x - ws.pre[s];
  double acc[NORM ? 1 : NV];
#pragma unroll
  for (int k = 0; k < (NORM ? 1 : NV); ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)K.nblk * 256;
  for (int64_t t = lb * 256 + threadIdx.x; t < K.n; t += stride) {
    double v[NV];
    double wi = K.w[t];
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nvec) {
        v[k] = K.V[(int64_t)k * K.n + t];
        wi -= hv[k] * v[k];
      }
    K.w[t] = wi;
    if (NORM) {
      acc[0] += wi * wi;
    } else {
#pragma unroll
      for (int k = 0; k < NV; ++k)
        if (k < nvec) acc[k] += v[k] * wi;
    }
  }
  if (NORM) {
    const double tt = dev::block_sum(acc[0], red);
    if (threadIdx.x == 0) put_partial(K.partial + lb, tt);
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nvec) {
        const double tt = dev::block_sum(acc[k], red);
        if (threadIdx.x == 0) put_partial(K.partial + lb * nvec + k, tt);
      }
  }
  if (last_of(cnt + i, K.nblk, &flag)) {
    double *hsi = hs + (int64_t)i * kHS;
    sum_partials(K, NORM ? 1 : nvec, hsi + off, red);
    if (NORM && gv && threadIdx.x == 0) kry_givens_step(gv[i], hsi, j, active + i);
  }
}

// V[target] = w / sqrt(ss), and the same vector in the V-cycle's precision
// as the finest level's right-hand side (the next iteration's input)
template <typename T>
__global__ __launch_bounds__(256) void kb_scale(const DKry *__restrict__ kry,
                                                const int *__restrict__ active, WorkSet ws,
                                                const double *__restrict__ hs, int target,
                                                const DLev *__restrict__ lev0) {
  const int s = seg_of(ws, blockIdx.x);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DKry &K = kry[i];
  const int64_t k = (blockIdx.x - ws.pre[s]) * 256 + threadIdx.x;
  if (k < K.n) {
    const double v = K.w[k] / sqrt(hs[(int64_t)i * kHS + kOffSS]);
    K.V[(int64_t)target * K.n + k] = v;
    LV<T>::r(lev0[i])[k] = (T)v;
  }
}

// x += Z y with this instance's k directions
template <int NV>
__global__ __launch_bounds__(256) void kb_combine(const DKry *__restrict__ kry,
                                                  const int *__restrict__ active, WorkSet ws,
                                                  const double *__restrict__ hs,
                                                  const int *__restrict__ kcnt) {
  __shared__ double ys[NV];
  const int s = seg_of(ws, blockIdx.x);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DKry &K = kry[i];
  const int kk = kcnt[i];
  if (threadIdx.x < NV) ys[threadIdx.x] = threadIdx.x < kk ? hs[(int64_t)i * kHS + kOffY + threadIdx.x] : 0.0;
  __syncthreads();
  const int64_t t = (blockIdx.x - ws.pre[s]) * 256 + threadIdx.x;
  if (t >= K.n) return;
  double acc = 0.0;
#pragma unroll
  for (int jj = 0; jj < NV; ++jj)
    if (jj < kk) acc += ys[jj] * K.Z[(int64_t)jj * K.n + t];
  K.x[t] += acc;
}

__global__ __launch_bounds__(256) void kb_nonfinite(const DKry *__restrict__ kry,
                                                    const int *__restrict__ active, WorkSet ws,
                                                    int *__restrict__ flags) {
  const int s = seg_of(ws, blockIdx.x);
  const int i = ws.inst[s];
  if (!active[i]) return;
  const DKry &K = kry[i];
  const int64_t k = (blockIdx.x - ws.pre[s]) * 256 + threadIdx.x;
  if (k < K.n && !isfinite(K.w[k])) atomicOr(&flags[i], 1);
}

__global__ __launch_bounds__(256) void kb_activate(int *__restrict__ active, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) active[i] = 1;
}

// ------------------------------------------------ FGMRES control (device)
// One thread per instance.  The arithmetic is that of FGMRES with Givens
// rotations (Saad, Iterative Methods for Sparse Linear Systems, Alg. 9.6):
// each new Hessenberg column is rotated by the previous rotations, a new
// rotation zeroes its subdiagonal, and |g_{j+1}| is the residual norm of the
// least-squares solution.
__global__ __launch_bounds__(64) void kb_kry_reset(int *__restrict__ active, int *__restrict__ flags,
                                                   int *__restrict__ cnt, int n) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  active[i] = 1;
  flags[i] = 0;
  cnt[i] = 0;
}

__device__ __forceinline__ void kry_open_cycle(DGiv &G, double rn) {
  G.g[0] = rn;
  for (int r = 1; r <= kMaxVec; ++r) G.g[r] = 0.0;
  G.k = 0;
}

__global__ __launch_bounds__(64) void kb_kry_start(DGiv *__restrict__ gv, const double *__restrict__ hs,
                                                   const int *__restrict__ flags,
                                                   int *__restrict__ active, int *__restrict__ cyc,
                                                   int n, double rtol, int max_iter) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  DGiv &G = gv[i];
  const double beta0 = sqrt(hs[(int64_t)i * kHS + kOffSS]);
  G.beta0 = beta0;
  G.rnorm = beta0;
  G.rprev = 0.0;
  G.tol = rtol * beta0;
  G.it = 0;
  G.restarts = 0;
  G.nhist = 0;
  G.maxit = max_iter;
  G.status = FSIMG_OK;
  int go = 1;
  if (flags[i] || !isfinite(beta0)) {
    G.status = FSIMG_ERR_NONFINITE;
    go = 0;
  } else if (beta0 == 0.0) {
    go = 0;
  }
  kry_open_cycle(G, beta0);
  G.incyc = go;
  active[i] = go;
  cyc[i] = go;
}

__global__ __launch_bounds__(64) void kb_kry_ysolve(DGiv *__restrict__ gv, double *__restrict__ hs,
                                                    int *__restrict__ active, int *__restrict__ kcnt,
                                                    int n) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  DGiv &G = gv[i];
  if (!G.incyc) {
    active[i] = 0;
    kcnt[i] = 0;
    return;
  }
  const int k = G.k;
  double *y = hs + (int64_t)i * kHS + kOffY;
  for (int r = k - 1; r >= 0; --r) {
    double t = G.g[r];
    for (int c = r + 1; c < k; ++c) t -= G.R[c * kMaxVec + r] * y[c];
    y[r] = t / G.R[r * kMaxVec + r];
  }
  kcnt[i] = k;
  active[i] = 1;
}

__global__ __launch_bounds__(64) void kb_kry_restart(DGiv *__restrict__ gv, const double *__restrict__ hs,
                                                     int *__restrict__ active, int *__restrict__ cyc,
                                                     int n) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  DGiv &G = gv[i];
  if (!G.incyc) {
    active[i] = 0;
    cyc[i] = 0;
    return;
  }
  ++G.restarts;
  const double rn = sqrt(hs[(int64_t)i * kHS + kOffSS]);
  G.rnorm = rn;
  int go = 1;
  if (!isfinite(rn)) {
    G.status = FSIMG_ERR_NONFINITE;
    go = 0;
  } else if (rn <= G.tol) {
    go = 0;
  } else if (G.it >= G.maxit) {
    G.status = FSIMG_ERR_NOCONV;
    go = 0;
  }
  if (go) kry_open_cycle(G, rn);
  G.incyc = go;
  active[i] = go;
  cyc[i] = go;
}

inline dim3 grid_of(const WorkSet &ws) { return dim3((unsigned)ws.nblocks); }

}  // namespace

int64_t restrict3_blocks(int cx, int cy, int cz) {
  int ntx, wx, nty;
  restrict3_slabs(2 * cx + 1, 2 * cy + 1, ntx, wx, nty);
  return (int64_t)(2 * cz + 1) * ntx * nty;
}

int krylov_blocks(int64_t n) {
  const int64_t nb = (n + 1023) / 1024;
  return (int)(nb < 1 ? 1 : (nb > kRedBlocks ? kRedBlocks : nb));
}

template <typename T>
void launch_b_spmv(int b, int src, int rpw, const DLev *lev, const DKry *kry, const int *active,
                   const WorkSet &ws, int j, hipStream_t s) {
  if (ws.nblocks == 0) return;
#define FSIMG_BS(BV, SV, TT, RV)                                                                 \
  if (b == BV && src == SV && rpw == RV) {                                                       \
    hipLaunchKernelGGL((kb_spmv<BV, TT, SV, RV>), grid_of(ws), dim3(256), 0, s, lev, kry, active, \
                       ws, j);                                                                   \
    return;                                                                                      \
  }
#define FSIMG_BS_R(BV, SV, TT) FSIMG_BS(BV, SV, TT, 1) FSIMG_BS(BV, SV, TT, 2) FSIMG_BS(BV, SV, TT, 4)
  FSIMG_BS_R(1, BS_VCYCLE, T) FSIMG_BS_R(2, BS_VCYCLE, T) FSIMG_BS_R(3, BS_VCYCLE, T)
  FSIMG_BS_R(4, BS_VCYCLE, T)
  if constexpr (std::is_same<T, double>::value) {
    FSIMG_BS_R(1, BS_AZ, double) FSIMG_BS_R(2, BS_AZ, double) FSIMG_BS_R(3, BS_AZ, double)
    FSIMG_BS_R(4, BS_AZ, double)
    FSIMG_BS_R(1, BS_RESID, double) FSIMG_BS_R(2, BS_RESID, double)
    FSIMG_BS_R(3, BS_RESID, double) FSIMG_BS_R(4, BS_RESID, double)
  }
#undef FSIMG_BS_R
#undef FSIMG_BS
}

template <typename T>
void launch_b_vanka(int np, int b, int nl, int npc, int ppw, T omega, bool first, bool assign,
                    const DLev *lev, const int *active, const WorkSet &wp, const WorkSet &wg,
                    hipStream_t s, hipEvent_t e0, hipEvent_t e1, const DKry *kry, int zj) {
  if (e0) (void)hipEventRecord(e0, s);
  if (wp.nblocks > 0)
    hipLaunchKernelGGL((kb_vanka_patch<T>), grid_of(wp), dim3(vanka_threads(np, ppw)),
                       sizeof(T) * (size_t)ppw * npc, s, lev, active, wp, np, npc, b, nl, ppw,
                       first ? 1 : 0, 0);
  if (e1) (void)hipEventRecord(e1, s);
  if (wg.nblocks > 0)
    hipLaunchKernelGGL((kb_vanka_gather<T>), grid_of(wg), dim3(256), 0, s, lev, active, wg, b, omega,
                       assign ? 1 : 0, kry, zj);
}

template <typename T>
void launch_b_vanka_blocks(int np, int b, int nl, int npc, int ppw, bool first, const DLev *lev,
                           const int *active, const WorkSet &wp, hipStream_t s) {
  if (wp.nblocks > 0)
    hipLaunchKernelGGL((kb_vanka_patch<T>), grid_of(wp), dim3(vanka_threads(np, ppw)),
                       sizeof(T) * (size_t)ppw * npc, s, lev, active, wp, np, npc, b, nl, ppw,
                       first ? 1 : 0, 1);
}

template <typename T>
void launch_b_fill_x(const DLev *lev, const int *active, const WorkSet &ws, hipStream_t s) {
  if (ws.nblocks > 0)
    hipLaunchKernelGGL((kb_fill_x<T>), grid_of(ws), dim3(256), 0, s, lev, active, ws);
}

template <typename T>
void launch_b_restrict(int b, int dim, const DLev *levF, const DLev *levC, const int *active,
                       const WorkSet &ws, hipStream_t s) {
  if (ws.nblocks == 0) return;
#define FSIMG_BR(BV, DV)                                                                         \
  if (b == BV && dim == DV) {                                                                    \
    hipLaunchKernelGGL((kb_restrict<BV, DV, T>), grid_of(ws), dim3(256), 0, s, levF, levC, active, \
                       ws);                                                                      \
    return;                                                                                      \
  }
#define FSIMG_BR3(BV)                                                                            \
  if (b == BV && dim == 3) {                                                                     \
    hipLaunchKernelGGL((kb_restrict3<BV, T>), grid_of(ws), dim3(256), 0, s, levF, levC, active,  \
                       ws);                                                                      \
    return;                                                                                      \
  }
  FSIMG_BR(1, 2) FSIMG_BR(2, 2) FSIMG_BR(3, 2) FSIMG_BR(4, 2)
  FSIMG_BR3(1) FSIMG_BR3(2) FSIMG_BR3(3) FSIMG_BR3(4)
#undef FSIMG_BR3
#undef FSIMG_BR
}

template <typename T>
void launch_b_prolong(int b, int dim, const DLev *levF, const DLev *levC, const int *active,
                      const WorkSet &ws, hipStream_t s) {
  if (ws.nblocks == 0) return;
#define FSIMG_BP(BV, DV)                                                                         \
  if (b == BV && dim == DV) {                                                                    \
    hipLaunchKernelGGL((kb_prolong<BV, DV, T>), grid_of(ws), dim3(256), 0, s, levF, levC, active, \
                       ws);                                                                      \
    return;                                                                                      \
  }
  FSIMG_BP(1, 2) FSIMG_BP(2, 2) FSIMG_BP(3, 2) FSIMG_BP(4, 2)
  FSIMG_BP(1, 3) FSIMG_BP(2, 3) FSIMG_BP(3, 3) FSIMG_BP(4, 3)
#undef FSIMG_BP
}

template <typename T>
void launch_b_tail(int b, int dim, const DLev *lev, int n, const int *active, const int32_t *tinst,
                   int ninst, const int32_t *tfrom, int coarse, bool up, int np, int npc, int nl,
                   int np2, int npc2, int nl2, T omega, int nu_pre, int nu_post, hipStream_t s) {
  if (ninst == 0) return;
  constexpr int nt = tail_threads<T>();
  size_t lds = (size_t)(nt / np) * npc;
  if (np2 > 0) lds = std::max(lds, (size_t)(nt / np2) * npc2);
  lds *= sizeof(T);
#define FSIMG_BT(BV, DV)                                                                          \
  if (b == BV && dim == DV) {                                                                     \
    hipLaunchKernelGGL((kb_vcycle_tail<BV, DV, T>), dim3((unsigned)ninst), dim3(nt), lds,          \
                       s, lev, n, active, tinst, tfrom, coarse, up ? 1 : 0, np, npc, nl, np2, npc2, \
                       nl2, omega, nu_pre, nu_post);                                              \
    return;                                                                                       \
  }
  FSIMG_BT(1, 2) FSIMG_BT(2, 2) FSIMG_BT(3, 2) FSIMG_BT(4, 2)
  FSIMG_BT(1, 3) FSIMG_BT(2, 3) FSIMG_BT(3, 3) FSIMG_BT(4, 3)
#undef FSIMG_BT
}

template <typename T>
void launch_b_coarse(const DLev *lev, const int *active, const WorkSet &wn, const WorkSet &wf,
                     hipStream_t s) {
  (void)wn;  // wf covers the identity rows as well
  if (wf.nblocks > 0) hipLaunchKernelGGL((kb_coarse_gemv<T>), grid_of(wf), dim3(256), 0, s, lev, active, wf);
}

template <typename T>
void launch_b_copy_in(const DLev *lev0, const DKry *kry, const int *active, const WorkSet &ws,
                      int j, hipStream_t s) {
  if (ws.nblocks > 0)
    hipLaunchKernelGGL((kb_copy_in<T>), grid_of(ws), dim3(256), 0, s, lev0, kry, active, ws, j);
}

template <typename T>
void launch_b_copy_out(const DLev *lev0, const DKry *kry, const int *active, const WorkSet &ws,
                       int j, hipStream_t s) {
  if (ws.nblocks > 0)
    hipLaunchKernelGGL((kb_copy_out<T>), grid_of(ws), dim3(256), 0, s, lev0, kry, active, ws, j);
}

#define FSIMG_NVB(nvec, KER)            \
  do {                                  \
    if ((nvec) <= 8) KER(8);            \
    else if ((nvec) <= 16) KER(16);     \
    else KER(32);                       \
  } while (0)

void launch_b_multidot(const DKry *kry, const int *active, const WorkSet &wk, int nvec, bool norm_w,
                       double *hs, int off, int *cnt, hipStream_t s) {
  if (wk.nblocks == 0) return;
  if (norm_w) {
    hipLaunchKernelGGL((kb_multidot<8, 1>), grid_of(wk), dim3(256), 0, s, kry, active, wk, 1, hs, off, cnt);
    return;
  }
#define K(NV) hipLaunchKernelGGL((kb_multidot<NV, 0>), grid_of(wk), dim3(256), 0, s, kry, active, wk, nvec, hs, off, cnt)
  FSIMG_NVB(nvec, K);
#undef K
}

void launch_b_axpy_red(const DKry *kry, int *active, const WorkSet &wk, int nvec, bool norm, double *hs,
                       int hoff, int off, int *cnt, DGiv *gv, int j, hipStream_t s) {
  if (wk.nblocks == 0) return;
  if (norm) {
#define K(NV) hipLaunchKernelGGL((kb_axpy_red<NV, 1>), grid_of(wk), dim3(256), 0, s, kry, active, wk, nvec, hs, hoff, off, cnt, gv, j)
    FSIMG_NVB(nvec, K);
#undef K
  } else {
#define K(NV) hipLaunchKernelGGL((kb_axpy_red<NV, 0>), grid_of(wk), dim3(256), 0, s, kry, active, wk, nvec, hs, hoff, off, cnt, gv, j)
    FSIMG_NVB(nvec, K);
#undef K
  }
}

template <typename T>
void launch_b_scale(const DKry *kry, const int *active, const WorkSet &wv, const double *hs,
                    int target, const DLev *lev0, hipStream_t s) {
  if (wv.nblocks > 0)
    hipLaunchKernelGGL((kb_scale<T>), grid_of(wv), dim3(256), 0, s, kry, active, wv, hs, target, lev0);
}

void launch_b_combine(const DKry *kry, const int *active, const WorkSet &wv, const double *hs,
                      const int *kcnt, int kmax, hipStream_t s) {
  if (wv.nblocks == 0) return;
#define K(NV) hipLaunchKernelGGL((kb_combine<NV>), grid_of(wv), dim3(256), 0, s, kry, active, wv, hs, kcnt)
  FSIMG_NVB(kmax, K);
#undef K
}

void launch_b_nonfinite(const DKry *kry, const int *active, const WorkSet &wv, int *flags,
                        hipStream_t s) {
  if (wv.nblocks > 0)
    hipLaunchKernelGGL(kb_nonfinite, grid_of(wv), dim3(256), 0, s, kry, active, wv, flags);
}

void launch_b_activate(int *active, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(kb_activate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, active, n);
}

namespace {
dim3 kry_grid(int n) { return dim3((unsigned)((n + 63) / 64)); }
}  // namespace

void launch_kry_reset(int *active, int *flags, int *cnt, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(kb_kry_reset, kry_grid(n), dim3(64), 0, s, active, flags, cnt, n);
}
void launch_kry_start(DGiv *gv, const double *hs, const int *flags, int *active, int *cyc, int n,
                      double rtol, int max_iter, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(kb_kry_start, kry_grid(n), dim3(64), 0, s, gv, hs, flags, active, cyc, n, rtol,
                       max_iter);
}
void launch_kry_ysolve(DGiv *gv, double *hs, int *active, int *kcnt, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(kb_kry_ysolve, kry_grid(n), dim3(64), 0, s, gv, hs, active, kcnt, n);
}
void launch_kry_restart(DGiv *gv, const double *hs, int *active, int *cyc, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(kb_kry_restart, kry_grid(n), dim3(64), 0, s, gv, hs, active, cyc, n);
}

#define FSIMG_BINST(T)                                                                           \
  template void launch_b_spmv<T>(int, int, int, const DLev *, const DKry *, const int *,         \
                                 const WorkSet &, int, hipStream_t);                             \
  template void launch_b_vanka<T>(int, int, int, int, int, T, bool, bool, const DLev *,          \
                                  const int *,                                                   \
                                  const WorkSet &, const WorkSet &, hipStream_t, hipEvent_t,     \
                                  hipEvent_t, const DKry *, int);                                \
  template void launch_b_vanka_blocks<T>(int, int, int, int, int, bool, const DLev *, const int *, \
                                         const WorkSet &, hipStream_t);                          \
  template void launch_b_fill_x<T>(const DLev *, const int *, const WorkSet &, hipStream_t);     \
  template void launch_b_tail<T>(int, int, const DLev *, int, const int *, const int32_t *, int,  \
                                 const int32_t *, int, bool, int, int, int, int, int, int, T, int,  \
                                 int, hipStream_t);                                               \
  template void launch_b_restrict<T>(int, int, const DLev *, const DLev *, const int *,          \
                                     const WorkSet &, hipStream_t);                              \
  template void launch_b_prolong<T>(int, int, const DLev *, const DLev *, const int *,           \
                                    const WorkSet &, hipStream_t);                               \
  template void launch_b_coarse<T>(const DLev *, const int *, const WorkSet &, const WorkSet &,  \
                                   hipStream_t);                                                 \
  template void launch_b_scale<T>(const DKry *, const int *, const WorkSet &, const double *, int,   \
                                  const DLev *, hipStream_t);                                      \
  template void launch_b_copy_in<T>(const DLev *, const DKry *, const int *, const WorkSet &, int, \
                                    hipStream_t);                                                \
  template void launch_b_copy_out<T>(const DLev *, const DKry *, const int *, const WorkSet &,   \
                                     int, hipStream_t);
FSIMG_BINST(double)
FSIMG_BINST(float)
#undef FSIMG_BINST

}  // namespace fsimg
