// Bandwidth-bound kernels of the single-hierarchy path on gfx950 (wave64):
// block-CSR residual SpMV, additive Vanka apply, Q2 grid transfers, casts.
// The per-row / per-patch / per-node bodies live in device_ops.h and are
// shared with the batched kernels.
#include "device_ops.h"

namespace fsimg {

namespace {

using dev::kWave;

template <int B, typename T, int MODE, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_bsr_spmv(int64_t nrows, const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colind,
                                                  const T *__restrict__ vals,
                                                  const T *__restrict__ x,
                                                  const T *__restrict__ b,
                                                  const uint8_t *__restrict__ mask,
                                                  T *__restrict__ y) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t lb = dev::xcd_block(blockIdx.x, gridDim.x);
  const int64_t row0 = (lb * (blockDim.x / kWave) + (threadIdx.x / kWave)) * R *
                       spmv_group_rows(B, (int)sizeof(T));
  if (row0 >= nrows) return;  // uniform per wave
  dev::spmv_rows<B, T, MODE, R>(row0, nrows, lane, rowptr, colind, vals, x, b, mask, y);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_vanka_patch(
    int64_t p0, int64_t p1, int np, int npc, int b, int nl, int ppw,
    const int32_t *__restrict__ pnodes, const T *__restrict__ inv, const T *__restrict__ d,
    T *__restrict__ Y, int scatter, T *__restrict__ x, const T *__restrict__ scale,
    const uint8_t *__restrict__ mask, T omega) {
  extern __shared__ unsigned char smem_raw[];
  dev::vanka_patch_wg<T>(p0 + dev::xcd_block(blockIdx.x, gridDim.x) * ppw, p1, np, npc, b, nl, ppw,
                         pnodes, inv, d, Y,
                         scatter, x, scale, mask, omega, reinterpret_cast<T *>(smem_raw));
}

template <typename T>
__global__ __launch_bounds__(256) void k_vanka_gather(int64_t n, int b,
                                                      const int32_t *__restrict__ gptr,
                                                      const int32_t *__restrict__ gidx,
                                                      const T *__restrict__ Y,
                                                      const T *__restrict__ scale,
                                                      const uint8_t *__restrict__ mask, T omega,
                                                      int assign, T *__restrict__ x) {
  const int64_t dof = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (dof >= n) return;
  dev::vanka_gather_dof<T>(dof, b, gptr, gidx, Y, scale, mask, omega, assign, x);
}

template <int B, int DIM, typename T>
__global__ __launch_bounds__(256) void k_restrict(int cx, int cy, int cz, const T *__restrict__ rf,
                                                  T *__restrict__ rc,
                                                  const uint8_t *__restrict__ maskc) {
  const int64_t nn = (int64_t)(2 * cx + 1) * (2 * cy + 1) * (DIM == 3 ? 2 * cz + 1 : 1);
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nn) return;
  dev::restrict_node<B, DIM, T>(node, cx, cy, cz, rf, rc, maskc);
}

template <int B, int DIM, typename T>
__global__ __launch_bounds__(256) void k_prolong_add(int cx, int cy, int cz,
                                                     const T *__restrict__ xc, T *__restrict__ xf,
                                                     const uint8_t *__restrict__ maskf) {
  const int64_t nn = (int64_t)(4 * cx + 1) * (4 * cy + 1) * (DIM == 3 ? 4 * cz + 1 : 1);
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nn) return;
  dev::prolong_node<B, DIM, T>(node, cx, cy, cz, xc, xf, maskf);
}

template <typename T>
__global__ void k_fill(T *x, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
__global__ void k_cast_d2f(const double *x, float *y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}
__global__ void k_cast_f2d(const float *x, double *y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}
__global__ void k_mask_zero(double *x, const uint8_t *mask, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && mask[i]) x[i] = 0.0;
}

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

}  // namespace

// Patches per workgroup for the Vanka apply: the workgroup holds ppw patches
// of np row-threads rounded up to whole wavefronts; the default ppw leaves
// the fewest idle lanes (ties: the smaller workgroup).
int vanka_default_ppw(int np) {
  double best = -1.0;
  int ppw = 1;
  for (int p = 1; p * np <= 1024; ++p) {
    const double u = (double)(p * np) / vanka_threads(np, p);
    if (u > best + 1e-12) { best = u; ppw = p; }
  }
  return ppw;
}

template <typename T>
void launch_bsr_spmv_rpw(const DevLevel &L, const T *vals, const T *x, const T *b, T *y,
                         bool resid, int rpw, hipStream_t s) {
  const unsigned grid = grid_for(L.nrows, 4 * rpw * spmv_group_rows(L.b, (int)sizeof(T)));
#define FSIMG_SPMV_CASE(BV, RV)                                                                  \
  if (L.b == BV && rpw == RV) {                                                                  \
    if (resid)                                                                                   \
      hipLaunchKernelGGL((k_bsr_spmv<BV, T, 1, RV>), dim3(grid), dim3(256), 0, s, L.nrows,       \
                         L.rowptr, L.colind, vals, x, b, L.mask, y);                             \
    else                                                                                         \
      hipLaunchKernelGGL((k_bsr_spmv<BV, T, 0, RV>), dim3(grid), dim3(256), 0, s, L.nrows,       \
                         L.rowptr, L.colind, vals, x, b, L.mask, y);                             \
    return;                                                                                      \
  }
  FSIMG_SPMV_CASE(1, 1) FSIMG_SPMV_CASE(2, 1) FSIMG_SPMV_CASE(3, 1) FSIMG_SPMV_CASE(4, 1)
  FSIMG_SPMV_CASE(1, 2) FSIMG_SPMV_CASE(2, 2) FSIMG_SPMV_CASE(3, 2) FSIMG_SPMV_CASE(4, 2)
  FSIMG_SPMV_CASE(1, 4) FSIMG_SPMV_CASE(2, 4) FSIMG_SPMV_CASE(3, 4) FSIMG_SPMV_CASE(4, 4)
#undef FSIMG_SPMV_CASE
}

template <typename T>
void launch_bsr_spmv(const DevLevel &L, const T *vals, const T *x, const T *b, T *y, bool resid,
                     hipStream_t s) {
  launch_bsr_spmv_rpw<T>(L, vals, x, b, y, resid,
                         spmv_rows_per_wave(L.tune, L.b, (int)sizeof(T), L.nrows), s);
}

template <typename T>
void launch_vanka_patch_ppw(const DevLevel &L, int grp, const T *inv, int npc, const T *d, T *Y,
                            int ppw, hipStream_t s) {
  const int64_t npatch = grp ? L.blk.npatch : L.npatch;
  const int np = grp ? L.blk.np : L.np, nl = grp ? L.blk.nl : L.nl;
  if (npatch == 0) return;
  const unsigned grid = grid_for(npatch, ppw);
  const size_t lds = sizeof(T) * (size_t)ppw * npc;
  hipLaunchKernelGGL((k_vanka_patch<T>), dim3(grid), dim3(vanka_threads(np, ppw)), lds, s,
                     (int64_t)0, npatch, np, npc, L.b, nl, ppw, grp ? L.blk.pnodes : L.pnodes, inv,
                     d, Y, 0, (T *)nullptr, (const T *)nullptr, L.mask, T(0));
}

template <typename T>
void launch_vanka_patch(const DevLevel &L, const T *inv, int npc, const T *d, T *Y, int64_t p0,
                        int64_t p1, bool scatter, T *x, const T *scale, T omega, hipStream_t s) {
  if (p1 <= p0) return;
  const int ppw = vanka_patches_per_wg(L.tune, L.np, (int)sizeof(T), L.npatch);
  const unsigned grid = grid_for(p1 - p0, ppw);
  const size_t lds = sizeof(T) * (size_t)ppw * npc;
  hipLaunchKernelGGL((k_vanka_patch<T>), dim3(grid), dim3(vanka_threads(L.np, ppw)), lds, s, p0, p1,
                     L.np, npc, L.b, L.nl, ppw, L.pnodes, inv, d, Y, scatter ? 1 : 0, x, scale,
                     L.mask, omega);
}

template <typename T>
void launch_vanka_blocks(const DevLevel &L, const T *inv, int npc, const T *d, T *Y,
                         hipStream_t s) {
  const PatchBlocks &B = L.blk;
  if (B.npatch == 0) return;
  const int ppw = vanka_patches_per_wg(L.tune, B.np, (int)sizeof(T), B.npatch);
  const unsigned grid = grid_for(B.npatch, ppw);
  const size_t lds = sizeof(T) * (size_t)ppw * npc;
  hipLaunchKernelGGL((k_vanka_patch<T>), dim3(grid), dim3(vanka_threads(B.np, ppw)), lds, s,
                     (int64_t)0, B.npatch, B.np, npc, L.b, B.nl, ppw, B.pnodes, inv, d, Y, 0,
                     (T *)nullptr, (const T *)nullptr, L.mask, T(0));
}

template <typename T>
void launch_vanka_gather(const DevLevel &L, const T *Y, const T *scale, T omega, bool assign, T *x,
                         hipStream_t s) {
  hipLaunchKernelGGL((k_vanka_gather<T>), dim3(grid_for(L.n, 256)), dim3(256), 0, s, L.n, L.b,
                     L.gptr, L.gidx, Y, scale, L.mask, omega, assign ? 1 : 0, x);
}

template <typename T>
void launch_restrict(const DevLevel &F, const DevLevel &C, const T *rf, T *rc, hipStream_t s) {
  const unsigned grid = grid_for(C.nrows, 256);
#define FSIMG_R(BV, DV)                                                                          \
  if (C.b == BV && C.dim == DV) {                                                                \
    hipLaunchKernelGGL((k_restrict<BV, DV, T>), dim3(grid), dim3(256), 0, s, C.cells[0],         \
                       C.cells[1], C.cells[2], rf, rc, C.mask);                                  \
    return;                                                                                      \
  }
  FSIMG_R(1, 2) FSIMG_R(2, 2) FSIMG_R(3, 2) FSIMG_R(4, 2)
  FSIMG_R(1, 3) FSIMG_R(2, 3) FSIMG_R(3, 3) FSIMG_R(4, 3)
#undef FSIMG_R
  (void)F;
}

template <typename T>
void launch_prolong_add(const DevLevel &F, const DevLevel &C, const T *xc, T *xf, hipStream_t s) {
  const unsigned grid = grid_for(F.nrows, 256);
#define FSIMG_P(BV, DV)                                                                          \
  if (F.b == BV && F.dim == DV) {                                                                \
    hipLaunchKernelGGL((k_prolong_add<BV, DV, T>), dim3(grid), dim3(256), 0, s, C.cells[0],      \
                       C.cells[1], C.cells[2], xc, xf, F.mask);                                  \
    return;                                                                                      \
  }
  FSIMG_P(1, 2) FSIMG_P(2, 2) FSIMG_P(3, 2) FSIMG_P(4, 2)
  FSIMG_P(1, 3) FSIMG_P(2, 3) FSIMG_P(3, 3) FSIMG_P(4, 3)
#undef FSIMG_P
}

template <typename T>
void launch_fill(T *x, int64_t n, T v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n, 256)), dim3(256), 0, s, x, n, v);
}
void launch_cast_d2f(const double *x, float *y, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_cast_d2f, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, n);
}
void launch_cast_f2d(const float *x, double *y, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_cast_f2d, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, n);
}
void launch_mask_zero(double *x, const uint8_t *mask, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_mask_zero, dim3(grid_for(n, 256)), dim3(256), 0, s, x, mask, n);
}

#define FSIMG_INST(T)                                                                            \
  template void launch_bsr_spmv<T>(const DevLevel &, const T *, const T *, const T *, T *, bool, \
                                   hipStream_t);                                                 \
  template void launch_vanka_patch<T>(const DevLevel &, const T *, int, const T *, T *, int64_t, \
                                      int64_t, bool, T *, const T *, T, hipStream_t);            \
  template void launch_bsr_spmv_rpw<T>(const DevLevel &, const T *, const T *, const T *, T *,   \
                                       bool, int, hipStream_t);                                  \
  template void launch_vanka_patch_ppw<T>(const DevLevel &, int, const T *, int, const T *, T *,  \
                                          int, hipStream_t);                                     \
  template void launch_vanka_blocks<T>(const DevLevel &, const T *, int, const T *, T *,         \
                                       hipStream_t);                                             \
  template void launch_vanka_gather<T>(const DevLevel &, const T *, const T *, T, bool, T *,     \
                                       hipStream_t);                                             \
  template void launch_restrict<T>(const DevLevel &, const DevLevel &, const T *, T *,           \
                                   hipStream_t);                                                 \
  template void launch_prolong_add<T>(const DevLevel &, const DevLevel &, const T *, T *,        \
                                      hipStream_t);                                              \
  template void launch_fill<T>(T *, int64_t, T, hipStream_t);
FSIMG_INST(double)
FSIMG_INST(float)
#undef FSIMG_INST

}  // namespace fsimg
