// Block ILU(0) smoother: the comparison smoother of Sec. 5.5, read as an
// incomplete LU without fill-in on the matrix's block pattern (one b x b
// block per coupled node pair, the matrix's node order).
//
// Factorisation (row-oriented, restricted to the pattern): for block row i and
// its blocks k < i in ascending order, L_ik = A_ik U_kk^{-1}, then
// A_ij -= L_ik U_kj for the blocks j > k of row k that row i also holds.
// Row i needs only rows k < i of its own pattern, so the rows are processed
// by levels of the lower triangle's dependency graph, one launch per level;
// a row's blocks are staged in LDS while it is eliminated.
//
// Apply: y = L^{-1} d by levels of the lower triangle, z = U^{-1} y by levels
// of the upper triangle (U_ii^{-1} stored), then x += omega z.  One wavefront
// per block row, lanes over the row's blocks, fixed-order wave reductions.
// The two level sweeps read and write fixed buffers only, so a caller can
// capture them once as a graph.
#include <cfloat>

#include "fsimg_internal.h"

namespace fsimg {

namespace {

constexpr int kWave = 64;

template <typename T>
__device__ __forceinline__ T wave_sum_t(T v) {
  for (int m = kWave / 2; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// one workgroup (one wavefront) per block row of the level
template <int B>
__global__ __launch_bounds__(64) void k_ilu_factor(const int32_t *__restrict__ rows,
                                                   const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ colind,
                                                   const int32_t *__restrict__ idiag,
                                                   double *__restrict__ F,
                                                   double *__restrict__ dinv,
                                                   int *__restrict__ status) {
  constexpr int BB = B * B;
  extern __shared__ double sh[];
  const int l = threadIdx.x;
  const int i = rows[blockIdx.x];
  const int beg = rowptr[i], len = rowptr[i + 1] - beg, dp = idiag[i] - beg;
  // LDS: the row's blocks | work copy of U_ii | its inverse | column indices
  double *Ai = sh;
  double *W = Ai + (size_t)len * BB;
  double *Wi = W + BB;
  int32_t *ci = reinterpret_cast<int32_t *>(Wi + BB);
  for (int e = l; e < len * BB; e += kWave) Ai[e] = F[(int64_t)beg * BB + e];
  for (int e = l; e < len; e += kWave) ci[e] = colind[beg + e];
  __syncthreads();
  for (int pk = 0; pk < dp; ++pk) {
    const int k = ci[pk];
    const double *dk = dinv + (int64_t)k * BB;
    double Lk[BB];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) {
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < B; ++m) v = fma(Ai[pk * BB + r * B + m], dk[m * B + c], v);
        Lk[r * B + c] = v;
      }
    __syncthreads();  // every lane has read A_ik
#pragma unroll
    for (int e = 0; e < BB; ++e)
      if (l == e) Ai[pk * BB + e] = Lk[e];
    // A_ij -= L_ik U_kj over the blocks j > k of row k found in row i
    const int q1 = rowptr[k + 1];
    for (int q = idiag[k] + 1 + l; q < q1; q += kWave) {
      const int32_t j = colind[q];
      int lo = pk + 1, hi = len - 1, pos = -1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int32_t c = ci[mid];
        if (c == j) {
          pos = mid;
          break;
        }
        if (c < j) lo = mid + 1;
        else hi = mid - 1;
      }
      if (pos >= 0) {
        double U[BB];
#pragma unroll
        for (int e = 0; e < BB; ++e) U[e] = F[(int64_t)q * BB + e];
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
          for (int c = 0; c < B; ++c) {
            double v = Ai[pos * BB + r * B + c];
#pragma unroll
            for (int m = 0; m < B; ++m) v = fma(-Lk[r * B + m], U[m * B + c], v);
            Ai[pos * BB + r * B + c] = v;
          }
      }
    }
    __syncthreads();
  }
  // U_ii^{-1} by Gauss-Jordan with partial pivoting (one lane, LDS)
  if (l == 0) {
    double amax = 0.0;
    for (int e = 0; e < BB; ++e) {
      W[e] = Ai[dp * BB + e];
      Wi[e] = (e / B == e % B) ? 1.0 : 0.0;
      amax = fmax(amax, fabs(W[e]));
    }
    bool singular = false;
    for (int c = 0; c < B; ++c) {
      int pr = c;
      for (int r = c + 1; r < B; ++r)
        if (fabs(W[r * B + c]) > fabs(W[pr * B + c])) pr = r;
      if (!(fabs(W[pr * B + c]) > 1e-15 * amax)) singular = true;
      if (pr != c)
        for (int e = 0; e < B; ++e) {
          double t = W[c * B + e];
          W[c * B + e] = W[pr * B + e];
          W[pr * B + e] = t;
          t = Wi[c * B + e];
          Wi[c * B + e] = Wi[pr * B + e];
          Wi[pr * B + e] = t;
        }
      const double rp = 1.0 / W[c * B + c];
      for (int e = 0; e < B; ++e) {
        W[c * B + e] *= rp;
        Wi[c * B + e] *= rp;
      }
      for (int r = 0; r < B; ++r)
        if (r != c) {
          const double f = W[r * B + c];
          for (int e = 0; e < B; ++e) {
            W[r * B + e] -= f * W[c * B + e];
            Wi[r * B + e] -= f * Wi[c * B + e];
          }
        }
    }
    for (int e = 0; e < BB; ++e) dinv[(int64_t)i * BB + e] = Wi[e];
    if (singular) {
      atomicOr(&status[0], 1);
      atomicMin(&status[1], i);
    }
  }
  for (int e = l; e < len * BB; e += kWave) F[(int64_t)beg * BB + e] = Ai[e];
}

// y_i = d_i - sum_{k < i} L_ik y_k for the rows of one level (y != d)
template <int B, typename T>
__global__ __launch_bounds__(256) void k_ilu_lower(const int32_t *__restrict__ rows, int nr,
                                                   const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ colind,
                                                   const int32_t *__restrict__ idiag,
                                                   const T *__restrict__ F,
                                                   const T *__restrict__ d, T *__restrict__ y) {
  constexpr int BB = B * B;
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (wv >= nr) return;
  const int i = rows[wv];
  const int p1 = idiag[i];
  T acc[B];
#pragma unroll
  for (int r = 0; r < B; ++r) acc[r] = T(0);
  for (int p = rowptr[i] + l; p < p1; p += kWave) {
    const int k = colind[p];
    const T *f = F + (int64_t)p * BB;
    T yk[B];
#pragma unroll
    for (int c = 0; c < B; ++c) yk[c] = y[(int64_t)k * B + c];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) acc[r] += f[r * B + c] * yk[c];
  }
#pragma unroll
  for (int r = 0; r < B; ++r) acc[r] = wave_sum_t(acc[r]);
  if (l == 0)
#pragma unroll
    for (int r = 0; r < B; ++r) y[(int64_t)i * B + r] = d[(int64_t)i * B + r] - acc[r];
}

// z_i = U_ii^{-1} (y_i - sum_{j > i} U_ij z_j) in place of y for the rows of
// one level
template <int B, typename T>
__global__ __launch_bounds__(256) void k_ilu_upper(const int32_t *__restrict__ rows, int nr,
                                                   const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ colind,
                                                   const int32_t *__restrict__ idiag,
                                                   const T *__restrict__ F,
                                                   const T *__restrict__ dinv,
                                                   T *__restrict__ y) {
  constexpr int BB = B * B;
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (wv >= nr) return;
  const int i = rows[wv];
  const int p1 = rowptr[i + 1];
  T acc[B];
#pragma unroll
  for (int r = 0; r < B; ++r) acc[r] = T(0);
  for (int p = idiag[i] + 1 + l; p < p1; p += kWave) {
    const int j = colind[p];
    const T *f = F + (int64_t)p * BB;
    T zj[B];
#pragma unroll
    for (int c = 0; c < B; ++c) zj[c] = y[(int64_t)j * B + c];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) acc[r] += f[r * B + c] * zj[c];
  }
#pragma unroll
  for (int r = 0; r < B; ++r) acc[r] = wave_sum_t(acc[r]);
  if (l == 0) {
    T s[B];
#pragma unroll
    for (int r = 0; r < B; ++r) s[r] = y[(int64_t)i * B + r] - acc[r];
    const T *di = dinv + (int64_t)i * BB;
#pragma unroll
    for (int r = 0; r < B; ++r) {
      T z = T(0);
#pragma unroll
      for (int c = 0; c < B; ++c) z += di[r * B + c] * s[c];
      y[(int64_t)i * B + r] = z;
    }
  }
}

// x (+)= omega z at the non-identity dofs (identity dofs: kept, or 0 when
// assigning)
template <typename T>
__global__ __launch_bounds__(256) void k_ilu_axpy(int64_t n, const T *__restrict__ z,
                                                  const uint8_t *__restrict__ mask, T omega,
                                                  int assign, T *__restrict__ x) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  if (mask[o]) {
    if (assign) x[o] = T(0);
  } else {
    x[o] = assign ? omega * z[o] : x[o] + omega * z[o];
  }
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

void launch_ilu_factor(const DevLevel &L, int *status, hipStream_t s) {
  const int bb = L.b * L.b;
  const size_t lds = (size_t)L.ilu_maxrow * (bb * 8 + 4) + (size_t)2 * bb * 8 + 16;
  for (size_t lv = 0; lv + 1 < L.lptr.size(); ++lv) {
    const int64_t r0 = L.lptr[lv], cnt = L.lptr[lv + 1] - r0;
    if (cnt == 0) continue;
#define FSIMG_ILUF(BV)                                                                           \
  case BV:                                                                                       \
    hipLaunchKernelGGL(k_ilu_factor<BV>, dim3((unsigned)cnt), dim3(64), lds, s, L.lorder + r0,   \
                       L.rowptr, L.colind, L.idiag, L.ilu64, L.dinv64, status);                  \
    break;
    switch (L.b) {
      FSIMG_ILUF(1) FSIMG_ILUF(2) FSIMG_ILUF(3) FSIMG_ILUF(4)
      default: break;
    }
#undef FSIMG_ILUF
  }
}

template <typename T>
void launch_ilu_solve(const DevLevel &L, const T *F, const T *dinv, const T *d, T *work,
                      hipStream_t s) {
  for (size_t lv = 0; lv + 1 < L.lptr.size(); ++lv) {
    const int64_t r0 = L.lptr[lv], cnt = L.lptr[lv + 1] - r0;
    if (cnt == 0) continue;
#define FSIMG_ILUL(BV)                                                                           \
  case BV:                                                                                       \
    hipLaunchKernelGGL((k_ilu_lower<BV, T>), dim3(blocks_for(cnt, 4)), dim3(256), 0, s,         \
                       L.lorder + r0, (int)cnt, L.rowptr, L.colind, L.idiag, F, d, work);        \
    break;
    switch (L.b) {
      FSIMG_ILUL(1) FSIMG_ILUL(2) FSIMG_ILUL(3) FSIMG_ILUL(4)
      default: break;
    }
#undef FSIMG_ILUL
  }
  for (size_t lv = 0; lv + 1 < L.uptr.size(); ++lv) {
    const int64_t r0 = L.uptr[lv], cnt = L.uptr[lv + 1] - r0;
    if (cnt == 0) continue;
#define FSIMG_ILUU(BV)                                                                           \
  case BV:                                                                                       \
    hipLaunchKernelGGL((k_ilu_upper<BV, T>), dim3(blocks_for(cnt, 4)), dim3(256), 0, s,         \
                       L.uorder + r0, (int)cnt, L.rowptr, L.colind, L.idiag, F, dinv, work);     \
    break;
    switch (L.b) {
      FSIMG_ILUU(1) FSIMG_ILUU(2) FSIMG_ILUU(3) FSIMG_ILUU(4)
      default: break;
    }
#undef FSIMG_ILUU
  }
}

template <typename T>
void launch_ilu_axpy(const DevLevel &L, const T *z, T omega, bool assign, T *x, hipStream_t s) {
  hipLaunchKernelGGL((k_ilu_axpy<T>), dim3(blocks_for(L.n, 256)), dim3(256), 0, s, L.n, z, L.mask,
                     omega, assign ? 1 : 0, x);
}

#define FSIMG_ILUI(T)                                                                             \
  template void launch_ilu_solve<T>(const DevLevel &, const T *, const T *, const T *, T *,       \
                                    hipStream_t);                                                 \
  template void launch_ilu_axpy<T>(const DevLevel &, const T *, T, bool, T *, hipStream_t);
FSIMG_ILUI(double)
FSIMG_ILUI(float)
#undef FSIMG_ILUI

}  // namespace fsimg
