// Krylov vector kernels (FP64), patch / coarse factorisation and the
// deformation update.
#include <algorithm>
#include <cfloat>

#include "fsimg_internal.h"

namespace fsimg {

namespace {

constexpr int kWave = 64;

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int m = kWave / 2; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Block sum of one value per thread (256 threads), result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += red[i];
  __syncthreads();
  return t;
}

// ----------------------------------------------------------- Krylov kernels
// V is row-major (nvec x n).  Every thread keeps NV accumulators in registers
// (compile-time bound, runtime count nvec <= NV), one pass over V and w.
template <int NV>
__global__ __launch_bounds__(256) void k_multidot(const double *__restrict__ V, int nvec, int64_t n,
                                                  const double *__restrict__ w,
                                                  double *__restrict__ partial) {
  __shared__ double red[4];
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double wi = w[i];
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nvec) acc[k] += V[(int64_t)k * n + i] * wi;
  }
#pragma unroll
  for (int k = 0; k < NV; ++k)
    if (k < nvec) {
      const double t = block_sum(acc[k], red);
      if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * nvec + k] = t;
    }
}

// w -= V h, then per-block partials of V^T w (MODE 0) or of w.w (MODE 1)
template <int NV, int MODE>
__global__ __launch_bounds__(256) void k_axpy_red(const double *__restrict__ V, int nvec, int64_t n,
                                                  const double *__restrict__ h,
                                                  double *__restrict__ w,
                                                  double *__restrict__ partial) {
  __shared__ double red[4];
  __shared__ double hs[NV];
  if (threadIdx.x < NV) hs[threadIdx.x] = threadIdx.x < nvec ? h[threadIdx.x] : 0.0;
  __syncthreads();
  double acc[MODE == 0 ? NV : 1];
#pragma unroll
  for (int k = 0; k < (MODE == 0 ? NV : 1); ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double v[NV];
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nvec) {
        v[k] = V[(int64_t)k * n + i];
        wi -= hs[k] * v[k];
      }
    w[i] = wi;
    if (MODE == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k)
        if (k < nvec) acc[k] += v[k] * wi;
    } else {
      acc[0] += wi * wi;
    }
  }
  if (MODE == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nvec) {
        const double t = block_sum(acc[k], red);
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * nvec + k] = t;
      }
  } else {
    const double t = block_sum(acc[0], red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
  }
}

// one block per output: sum of kRedBlocks partials in a fixed order
__global__ __launch_bounds__(256) void k_reduce_partials(const double *__restrict__ partial, int nvec,
                                                         double *__restrict__ out) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  double t = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) t += partial[(int64_t)i * nvec + k];
  t = block_sum(t, red);
  if (threadIdx.x == 0) out[k] = t;
}

__global__ void k_add_small(const double *a, const double *b, double *out, int n) {
  const int i = threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

__global__ __launch_bounds__(256) void k_scale_by_rsqrt(const double *__restrict__ w,
                                                        const double *__restrict__ ss,
                                                        double *__restrict__ v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = w[i] / sqrt(ss[0]);
}

template <int NV>
__global__ __launch_bounds__(256) void k_combine(const double *__restrict__ Z, int k, int64_t n,
                                                 const double *__restrict__ y,
                                                 double *__restrict__ x) {
  __shared__ double ys[NV];
  if (threadIdx.x < NV) ys[threadIdx.x] = threadIdx.x < k ? y[threadIdx.x] : 0.0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < NV; ++j)
    if (j < k) s += ys[j] * Z[(int64_t)j * n + i];
  x[i] += s;
}

__global__ void k_nonfinite(const double *__restrict__ x, int64_t n, int *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) atomicOr(flag, 1);
}

// -------------------------------------------------- patch factorisation
// One workgroup per patch: extract A_i = R_i A R_i^T from the block-CSR
// matrix into LDS (row stride np+1), invert it in place by Gauss-Jordan
// elimination with partial (row) pivoting in FP64, undo the row interchanges
// as column interchanges, and store the inverse in the column-group-major
// layout read by the Vanka apply kernel.
__device__ __forceinline__ int64_t find_block(const int32_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ colind, int64_t row,
                                              int32_t col) {
  int64_t lo = rowptr[row], hi = rowptr[row + 1] - 1;
  while (lo <= hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int32_t c = colind[mid];
    if (c == col) return mid;
    if (c < col) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

template <typename Tout>
__global__ __launch_bounds__(256) void k_patch_factor(int64_t npatch, int b, int nl, int np, int npc,
                                                      const int32_t *__restrict__ pnodes,
                                                      const int32_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ colind,
                                                      const double *__restrict__ vals,
                                                      Tout *__restrict__ inv,
                                                      int *__restrict__ status) {
  extern __shared__ double sm[];
  const int ld = np + 1;
  double *a = sm;
  double *rowk = a + (size_t)np * ld;
  double *colk = rowk + np;
  int *perm = reinterpret_cast<int *>(colk + np);
  int *colmap = perm + np;
  __shared__ double red[4];
  __shared__ int s_piv;
  const int tid = threadIdx.x;
  const int64_t p = blockIdx.x;
  if (p >= npatch) return;
  const int32_t *pn = pnodes + p * nl;
  const int bb = b * b;
  for (int pr = tid; pr < nl * nl; pr += blockDim.x) {
    const int l1 = pr / nl, l2 = pr - l1 * nl;
    const int64_t pos = find_block(rowptr, colind, pn[l1], pn[l2]);
    for (int c1 = 0; c1 < b; ++c1)
      for (int c2 = 0; c2 < b; ++c2)
        a[(l1 * b + c1) * ld + l2 * b + c2] = pos >= 0 ? vals[pos * bb + c1 * b + c2] : 0.0;
  }
  __syncthreads();
  // scale for the singularity test: max |a_ij|
  double m = 0.0;
  for (int idx = tid; idx < np * np; idx += blockDim.x) {
    const int i = idx / np, j = idx - i * np;
    m = fmax(m, fabs(a[i * ld + j]));
  }
  for (int o = kWave / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((tid & (kWave - 1)) == 0) red[tid / kWave] = m;
  __syncthreads();
  const double amax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const double thr = 1e-15 * amax;
  const int rg = blockDim.x / np;              // row groups
  const int my_j = tid % np, my_i0 = tid / np;  // column owned in the elimination
  bool singular = false;
  for (int k = 0; k < np; ++k) {
    if (tid < kWave) {  // pivot search in column k, ties to the lowest row
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < np; i += kWave) {
        const double v = fabs(a[i * ld + k]);
        if (v > best) { best = v; bi = i; }
      }
      for (int o = kWave / 2; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) { s_piv = bi; perm[k] = bi; }
    }
    __syncthreads();
    const int pk = s_piv;
    if (pk != k)
      for (int j = tid; j < np; j += blockDim.x) {
        const double t = a[k * ld + j];
        a[k * ld + j] = a[pk * ld + j];
        a[pk * ld + j] = t;
      }
    __syncthreads();
    const double pv = a[k * ld + k];
    if (!(fabs(pv) > thr)) singular = true;
    for (int j = tid; j < np; j += blockDim.x) rowk[j] = (j == k ? 1.0 : a[k * ld + j]) / pv;
    for (int i = tid; i < np; i += blockDim.x) colk[i] = a[i * ld + k];
    __syncthreads();
    if (my_i0 < rg) {
      const double rj = rowk[my_j];
      for (int i = my_i0; i < np; i += rg) {
        if (i == k) a[i * ld + my_j] = rj;
        else a[i * ld + my_j] = (my_j == k ? 0.0 : a[i * ld + my_j]) - colk[i] * rj;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int j = 0; j < np; ++j) colmap[j] = j;
    for (int k = np - 1; k >= 0; --k) {
      const int t = colmap[k];
      colmap[k] = colmap[perm[k]];
      colmap[perm[k]] = t;
    }
    if (singular) {
      atomicOr(&status[0], 1);
      atomicMin(&status[1], (int)p);
    }
  }
  __syncthreads();
  constexpr int G = 16 / sizeof(Tout);
  Tout *out = inv + p * (int64_t)np * npc;
  for (int idx = tid; idx < np * npc; idx += blockDim.x) {
    const int g = idx / (np * G);
    const int rem = idx - g * np * G;
    const int r = rem / G, q = rem - r * G;
    const int c = g * G + q;
    out[idx] = c < np ? (Tout)a[r * ld + colmap[c]] : Tout(0);
  }
}

// ------------------------------------------- patch factorisation (MFMA)
// Blocked Gauss-Jordan inversion with partial pivoting in FP64, in exchange
// form: rows are never interchanged.  The pivot of column k is the largest
// |a_ik| over the rows not yet used as pivots (ties to the lowest row), and
// the in-place result M holds the inverse with rows and columns permuted:
// A^{-1}[k][r_j] = M[r_k][j], r_k the pivot row of column k.
// The matrix, padded with an identity block to N = 16*NT rows, lives in the
// registers of NT update waves in the accumulator layout of
// v_mfma_f64_16x16x4f64 (wave w owns rows 16w..16w+15; per tile-column tj
// lane l holds (16w + 4v + l/16, 16tj + l%16), v = 0..3).  One more wave,
// the panel wave, eliminates each panel of 8 columns in its registers (lane
// l holds rows l and l+64; the pivot search is a DPP / lane-read maximum of
// a key packing |a_ik| and the row) and publishes the processed columns G
// and the pivot rows.  Per panel P:
//   1. the panel wave eliminates P (its columns were published before);
//   2. the owners of P's pivot rows (set R) publish those rows;
//   3. the update waves apply A[:,Q] += (G - E_R) A[R,Q] (two MFMAs with
//      K = 4 per 16x16 tile; P's own columns become G) to the tile column of
//      panel P+1 first and publish P+1's columns, so that the panel wave
//      eliminates P+1 while they update the other tile columns.
// Occupancy: six waves per SIMD (at most 80 VGPRs; at n_p = 108 three are
// spilled, in the write-out) lets three 8-wave workgroups share a CU, which
// hides one patch's panel chain behind the others' MFMA work.
typedef double fsimg_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double d4get(const fsimg_d4 &a, int v) {
  return v == 0 ? a[0] : (v == 1 ? a[1] : (v == 2 ? a[2] : a[3]));
}

__device__ __forceinline__ double readlane_d(double x, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// maximum over the 64 lanes: within each row of 16 lanes by DPP (two quad
// permutations, the half-row and row mirrors), then across the four rows
__device__ __forceinline__ unsigned wave_max_u32(unsigned x) {
  x = max(x, (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false));
  x = max(x, (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false));
  x = max(x, (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x141, 0xF, 0xF, false));
  x = max(x, (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x140, 0xF, 0xF, false));
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)x, 0);
  const unsigned b = (unsigned)__builtin_amdgcn_readlane((int)x, 16);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)x, 32);
  const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)x, 48);
  return max(max(a, b), max(c, d));
}
// pivot key of row i (< 128): the high word of |a| (exponent and 20 mantissa
// bits) with its 8 low bits replaced by 255 - i, so that the maximum takes
// the largest |a| to a relative 2^-12 and then the lowest row; 0 for rows
// that may not pivot.  NaN entries have the largest keys, so a NaN pivot is
// found and reported.
__device__ __forceinline__ unsigned pivot_key(double a, int i, bool allowed) {
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(a) >> 32) & 0x7FFFFFFFu;
  return allowed ? ((hi & ~0xFFu) | (unsigned)(255 - i)) : 0u;
}
// 1/x for normal x with 1/x normal: hardware reciprocal estimate and two
// Newton steps y <- y + y (1 - x y)
__device__ __forceinline__ double recip_newton(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

template <int NT, typename Tout>
__global__ __launch_bounds__((NT + 1) * 64) __attribute__((amdgpu_waves_per_eu(NT >= 8 ? 5 : 6))) void
k_patch_factor_mfma(
    int64_t npatch, int b, int nl, int np, int npc, const int32_t *__restrict__ pnodes,
    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
    const double *__restrict__ vals, Tout *__restrict__ inv, int *__restrict__ status) {
  constexpr int N = NT * 16;
  constexpr int NW = NT + 1;
  constexpr int NTH = NW * 64;
  constexpr int PW = 8;               // panel width
  constexpr int NSM = 3 * N * PW;     // doubles of pan[2][N][PW] and rowbuf[PW][N]
  constexpr int CAP = 2 * NSM;        // int32 slots for the patch's column lists
  __shared__ double smem[NSM];
  __shared__ int bpos[27 * 27];
  __shared__ int sp[27], sbeg[27], soff[28];
  __shared__ int piv[N];              // pivot row of every column
  __shared__ int rinv[N];             // column whose pivot a row is
  __shared__ double red[NW];
  // pan: panel columns, then G (alternating buffers); rowbuf: the panel's
  // pivot rows before its update; both alias the column lists of the
  // extraction, which are dead by then
  double(*pan)[N][PW] = reinterpret_cast<double(*)[N][PW]>(smem);
  double(*rowbuf)[N] = reinterpret_cast<double(*)[N]>(smem + 2 * N * PW);
  int32_t *cols = reinterpret_cast<int32_t *>(smem);
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int lr = l >> 4, lc = l & 15;
  const int64_t p = blockIdx.x;
  if (p >= npatch) return;
  // extraction: the block rows of the patch nodes go to LDS, then every
  // (node, node) block is found by binary search there
  const int32_t *pn = pnodes + p * nl;
  if (tid < nl) {
    const int32_t node = pn[tid];
    const int32_t beg = rowptr[node];
    sp[tid] = node;
    sbeg[tid] = beg;
    soff[tid + 1] = rowptr[node + 1] - beg;
  }
  __syncthreads();
  if (tid == 0) {
    soff[0] = 0;
    for (int t = 0; t < nl; ++t) soff[t + 1] += soff[t];
  }
  __syncthreads();
  const bool staged = soff[nl] <= CAP;
  if (staged)
    for (int l1 = w; l1 < nl; l1 += NW) {
      const int beg = sbeg[l1], o = soff[l1], len = soff[l1 + 1] - o;
      for (int j = l; j < len; j += 64) cols[o + j] = colind[beg + j];
    }
  __syncthreads();
  const unsigned mnl = (65536u + nl - 1) / nl;  // q = (x * mnl) >> 16 is x / nl for x < 729
  for (int pr = tid; pr < nl * nl; pr += NTH) {
    const int l1 = (int)(((unsigned)pr * mnl) >> 16), l2 = pr - l1 * nl;
    int pos = -1;
    if (staged) {
      const int32_t col = sp[l2];
      int lo = soff[l1], hi = soff[l1 + 1] - 1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int32_t c = cols[mid];
        if (c == col) {
          pos = sbeg[l1] + (mid - soff[l1]);
          break;
        }
        if (c < col) lo = mid + 1;
        else hi = mid - 1;
      }
    } else {
      pos = (int)find_block(rowptr, colind, sp[l1], sp[l2]);
    }
    bpos[pr] = pos;
  }
  // the padding block is the identity and stays untouched: panels past np
  // are skipped and their columns pivot on their own rows
  const int kend = (np + PW - 1) & ~(PW - 1);
  for (int k = tid; k < N; k += NTH) {
    rinv[k] = N;
    if (k >= kend) piv[k] = k;
  }
  __syncthreads();
  constexpr int G = 16 / sizeof(Tout);
  Tout *out = inv + p * (int64_t)np * npc;
  // Wave-specialised from here on: the panel wave and the update waves run
  // loops of their own with the same sequence of barriers (three per panel,
  // two after the last), on a branch that is uniform per wave.
  if (__builtin_amdgcn_readfirstlane(w) == NT) {
    __syncthreads();  // the update waves have loaded A and published panel 0
    double thr = 0.0;
    for (int i = 0; i < NT; ++i) thr = fmax(thr, red[i]);
    thr *= 1e-15;
    // rows i0 = l and i1 = l + 64 (where < N), whether they pivoted yet
    const int i0 = l, i1 = l + 64;
    const bool ok0 = i0 < N, ok1 = i1 < N;
    bool used0 = !ok0, used1 = !ok1, singular = false;
    for (int k0 = 0, buf = 0; k0 < kend; k0 += PW, buf ^= 1) {
      double a0[PW], a1[PW];
#pragma unroll
      for (int c = 0; c < PW; ++c) {
        a0[c] = ok0 ? pan[buf][i0][c] : 0.0;
        a1[c] = ok1 ? pan[buf][i1][c] : 0.0;
      }
#pragma unroll
      for (int jj = 0; jj < PW; ++jj) {
        const unsigned key =
            wave_max_u32(max(pivot_key(a0[jj], i0, !used0), pivot_key(a1[jj], i1, !used1)));
        const int r = 255 - (int)(key & 0xFFu);  // uniform
        const int rl = r & 63;
        double vp[PW];
        if (r >= 64) {
#pragma unroll
          for (int c = 0; c < PW; ++c) vp[c] = readlane_d(a1[c], rl);
        } else {
#pragma unroll
          for (int c = 0; c < PW; ++c) vp[c] = readlane_d(a0[c], rl);
        }
        used0 = used0 || i0 == r;
        used1 = used1 || i1 == r;
        const double pv = vp[jj];
        if (!(fabs(pv) > thr)) singular = true;
        const double rp = recip_newton(pv);
        const double f0 = a0[jj], f1 = a1[jj];
#pragma unroll
        for (int c = 0; c < PW; ++c) {
          if (c == jj) {
            a0[c] = -f0 * rp;
            a1[c] = -f1 * rp;
          } else {
            const double rj = vp[c] * rp;
            a0[c] = fma(-f0, rj, a0[c]);
            a1[c] = fma(-f1, rj, a1[c]);
          }
        }
        // the pivot row itself becomes row r / pivot, with 1 / pivot in column jj
        if (r >= 64) {
          if (l == rl)
#pragma unroll
            for (int c = 0; c < PW; ++c) a1[c] = c == jj ? rp : vp[c] * rp;
        } else {
          if (l == rl)
#pragma unroll
            for (int c = 0; c < PW; ++c) a0[c] = c == jj ? rp : vp[c] * rp;
        }
        if (l == 0) piv[k0 + jj] = r;
      }
#pragma unroll
      for (int c = 0; c < PW; ++c) {
        if (ok0) pan[buf][i0][c] = a0[c];
        if (ok1) pan[buf][i1][c] = a1[c];
      }
      __syncthreads();  // G and the pivots are out
      __syncthreads();  // the pivot rows are out
      __syncthreads();  // the next panel's columns are out
    }
    __syncthreads();
    for (int k = tid; k < N; k += NTH) rinv[piv[k]] = k;
    if (l == 0 && singular) {
      atomicOr(&status[0], 1);
      atomicMin(&status[1], (int)p);
    }
    __syncthreads();
  } else {
    fsimg_d4 acc[NT];
    double amax = 0.0;
    const int bb = b * b;
    const unsigned mb = (65536u + b - 1) / b;  // x / b for x < 128
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * w + 4 * v + lr;
      const int rq = (int)(((unsigned)r * mb) >> 16), rr = r - rq * b;
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
        const int c = 16 * tj + lc;
        const int cq = (int)(((unsigned)c * mb) >> 16), cr = c - cq * b;
        double val;
        if (r < np && c < np) {
          const int pos = bpos[rq * nl + cq];
          val = pos >= 0 ? vals[(int64_t)pos * bb + rr * b + cr] : 0.0;
          amax = fmax(amax, fabs(val));
        } else {
          val = r == c ? 1.0 : 0.0;
        }
        acc[tj][v] = val;
      }
    }
    for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o));
    if (l == 0) red[w] = amax;
    if (lc < PW)  // panel 0's columns
#pragma unroll
      for (int v = 0; v < 4; ++v) pan[0][16 * w + 4 * v + lr][lc] = acc[0][v];
    __syncthreads();
    for (int k0 = 0, buf = 0; k0 < kend; k0 += PW, buf ^= 1) {
      const int tp = k0 >> 4, cp = k0 & 15;
      const int k1 = k0 + PW, tn = k1 >> 4, cn = k1 & 15;
      const bool more = k1 < kend;
      __syncthreads();  // G and the pivots of this panel
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int x = piv[k0 + q];
        if ((x >> 4) == w && (x & 3) == lr) {
          const int v = (x & 15) >> 2;
#pragma unroll
          for (int tj = 0; tj < NT; ++tj) rowbuf[q][16 * tj + lc] = d4get(acc[tj], v);
        }
      }
      __syncthreads();  // the pivot rows
      double aw[PW / 4];
      const int ra = 16 * w + lc;
#pragma unroll
      for (int h = 0; h < PW / 4; ++h) {
        const int q = 4 * h + lr;
        aw[h] = pan[buf][ra][q] - (ra == piv[k0 + q] ? 1.0 : 0.0);
      }
      // the next panel's tile column first
      if (more)
#pragma unroll
        for (int tj = 0; tj < NT; ++tj)
          if (tj == tn) {
#pragma unroll
            for (int h = 0; h < PW / 4; ++h)
              acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[h], rowbuf[4 * h + lr][16 * tj + lc],
                                                             acc[tj], 0, 0, 0);
            if (tj == tp && lc >= cp && lc < cp + PW)
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[tj][v] = pan[buf][16 * w + 4 * v + lr][lc - cp];
            if (lc >= cn && lc < cn + PW)
#pragma unroll
              for (int v = 0; v < 4; ++v) pan[buf ^ 1][16 * w + 4 * v + lr][lc - cn] = acc[tj][v];
          }
      __syncthreads();  // the next panel's columns
#pragma unroll
      for (int tj = 0; tj < NT; ++tj)
        if (!(more && tj == tn)) {
#pragma unroll
          for (int h = 0; h < PW / 4; ++h)
            acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[h], rowbuf[4 * h + lr][16 * tj + lc],
                                                           acc[tj], 0, 0, 0);
          if (tj == tp && lc >= cp && lc < cp + PW)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[tj][v] = pan[buf][16 * w + 4 * v + lr][lc - cp];
        }
    }
    __syncthreads();
    for (int k = tid; k < N; k += NTH) rinv[piv[k]] = k;
    __syncthreads();
    // M[i][j] = A^{-1}[rinv[i]][piv[j]], written in the column-group-major
    // layout of the Vanka apply (groups of G columns, n_p rows each)
    int cj[NT];
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) cj[tj] = piv[16 * tj + lc];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ro = rinv[16 * w + 4 * v + lr];
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
        const int c = cj[tj];
        if (ro < np && c < np) out[((int64_t)(c / G) * np + ro) * G + c % G] = (Tout)acc[tj][v];
      }
    }
  }
  for (int idx = tid; idx < np * (npc - np); idx += NTH) {
    const int r = idx / (npc - np), c = np + idx % (npc - np);
    out[((int64_t)(c / G) * np + r) * G + c % G] = Tout(0);
  }
}

// -------------------------------------------------- large patches
// Patches with more than 128 dofs (the 500-dof solid blocks of 3D) are
// inverted by Gauss-Jordan with partial pivoting in FP64: A_i is assembled
// into a per-patch n_p x n_p work matrix, which the coarse level's blocked
// exchange-form kernels (panels of 32 columns, below) factor for every patch
// of a launch at once (batch index blockIdx.z); the inverse is then written
// in the apply kernel's column-group-major layout.
__global__ __launch_bounds__(256) void k_big_load(int64_t npatch, int b, int nl, int np,
                                                  const int32_t *__restrict__ pnodes,
                                                  const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colind,
                                                  const double *__restrict__ vals,
                                                  double *__restrict__ work,
                                                  double *__restrict__ amax) {
  __shared__ double red[4];
  const int64_t p = blockIdx.x;
  if (p >= npatch) return;
  const int32_t *pn = pnodes + p * nl;
  double *a = work + p * (int64_t)np * np;
  const int bb = b * b;
  double m = 0.0;
  for (int pr = threadIdx.x; pr < nl * nl; pr += blockDim.x) {
    const int l1 = pr / nl, l2 = pr - l1 * nl;
    const int64_t pos = find_block(rowptr, colind, pn[l1], pn[l2]);
    for (int bi = 0; bi < b; ++bi)
      for (int bj = 0; bj < b; ++bj) {
        const double v = pos >= 0 ? vals[pos * bb + bi * b + bj] : 0.0;
        a[(int64_t)(l1 * b + bi) * np + l2 * b + bj] = v;
        m = fmax(m, fabs(v));
      }
  }
  for (int o = kWave / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) amax[p] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// the inverse of patch blockIdx.x from its blocked Gauss-Jordan result
// (coarse convention: A^{-1}[r][c] = a[rinv[r] np + piv[c]]), written in the
// apply kernel's column-group-major layout with zero columns up to npc
template <typename Tout>
__global__ __launch_bounds__(256) void k_bgj_out(int np, int npc, const double *__restrict__ work,
                                                 const int *__restrict__ piv,
                                                 const int *__restrict__ rinv,
                                                 Tout *__restrict__ inv) {
  const int64_t p = blockIdx.x;
  constexpr int G = 16 / sizeof(Tout);
  const double *a = work + p * (int64_t)np * np;
  const int *pv = piv + p * np, *ri = rinv + p * np;
  Tout *out = inv + p * (int64_t)np * npc;
  for (int e = threadIdx.x; e < np * npc; e += blockDim.x) {
    const int r = e / npc, c = e - r * npc;
    const double v = c < np ? a[(int64_t)ri[r] * np + pv[c]] : 0.0;
    out[((int64_t)(c / G) * np + r) * G + (c % G)] = (Tout)v;
  }
}


// ------------------------------------------------------- coarse level
// dense block of the free (non-identity) dofs: dense[cidx[i]][cidx[j]] = A[i][j]
__global__ __launch_bounds__(256) void k_densify(int64_t nrows, int b, int64_t nf,
                                                 const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ colind,
                                                 const double *__restrict__ vals,
                                                 const int32_t *__restrict__ cidx,
                                                 double *__restrict__ dense) {
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  if (row >= nrows) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int bb = b * b;
  for (int64_t j = rowptr[row]; j < rowptr[row + 1]; ++j) {
    const int64_t col = colind[j];
    if (lane < bb) {
      const int r = lane / b, c = lane - r * b;
      const int fi = cidx[row * b + r], fj = cidx[col * b + c];
      if (fi >= 0 && fj >= 0) dense[(int64_t)fi * nf + fj] = vals[j * bb + lane];
    }
  }
}

// pivot search + row swap + pivot row / column copies for column k (one block)
__global__ __launch_bounds__(1024) void k_gj_pivot(int64_t n, int64_t k, double *__restrict__ a,
                                                   int *__restrict__ piv, double *__restrict__ rowk,
                                                   double *__restrict__ colk, double thr,
                                                   int *__restrict__ status) {
  __shared__ double sb[16];
  __shared__ int si[16];
  __shared__ int s_p;
  double best = -1.0;
  int64_t bi = k;
  for (int64_t i = k + threadIdx.x; i < n; i += blockDim.x) {
    const double v = fabs(a[i * n + k]);
    if (v > best) { best = v; bi = i; }
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o);
    const int64_t oi = __shfl_xor(bi, o);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) { sb[w] = best; si[w] = (int)bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = sb[0];
    int bix = si[0];
    for (int i = 1; i < (int)(blockDim.x / kWave); ++i)
      if (sb[i] > bv || (sb[i] == bv && si[i] < bix)) { bv = sb[i]; bix = si[i]; }
    s_p = bix;
    piv[k] = bix;
  }
  __syncthreads();
  const int64_t p = s_p;
  if (p != k)
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
      const double t = a[k * n + j];
      a[k * n + j] = a[p * n + j];
      a[p * n + j] = t;
    }
  __syncthreads();
  const double pv = a[k * n + k];
  if (threadIdx.x == 0 && !(fabs(pv) > thr)) {
    atomicOr(&status[0], 1);
    atomicMin(&status[1], (int)k);
  }
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) rowk[j] = (j == k ? 1.0 : a[k * n + j]) / pv;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) colk[i] = a[i * n + k];
}

__global__ __launch_bounds__(256) void k_gj_update(int64_t n, int64_t k, double *__restrict__ a,
                                                   const double *__restrict__ rowk,
                                                   const double *__restrict__ colk) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= n) return;
  const int64_t o = i * n + j;
  if (i == k) a[o] = rowk[j];
  else a[o] = (j == k ? 0.0 : a[o]) - colk[i] * rowk[j];
}

__global__ void k_gj_colmap(int64_t n, const int *__restrict__ piv, int *__restrict__ colmap) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int64_t j = 0; j < n; ++j) colmap[j] = (int)j;
  for (int64_t k = n - 1; k >= 0; --k) {
    const int t = colmap[k];
    colmap[k] = colmap[piv[k]];
    colmap[piv[k]] = t;
  }
}

__global__ __launch_bounds__(256) void k_gj_out(int64_t n, const double *__restrict__ a,
                                                const int *__restrict__ colmap,
                                                double *__restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j < n) out[i * n + j] = a[i * n + colmap[j]];
}

// ------------------------------- coarse inverse: blocked Gauss-Jordan (n <= 4096)
// The kernels factor B = A^T, whose column-major storage is the row-major
// array of A, so that a thread's accesses to its rows of a panel column are
// contiguous across threads: B(i, j) = a[j n + i].  Exchange form, as for
// the patches: the pivot of column k is the largest |b_ik| over the rows not
// yet used (ties to the lowest row), no rows move, and B^{-1}[k][r_j] =
// M[r_k][j] at the end, i.e. A^{-1}[x][y] = M[r_y][rinv(x)].  Panels of
// kCoarsePB columns, each made of sub-panels t of PW columns with pivot rows
// R_t (ub, U column-major: U(i, q) = ub[q n + i]):
//   k_cgj_panel (one workgroup of 1024 threads, thread t owning rows
//     t + 1024 s, s < RPT), per sub-panel: bring its columns up to date with
//     the panel's earlier sub-panels (left-looking), eliminate them in
//     registers and keep U_t = G_t - E_{R_t} (G_t: the processed columns,
//     left in the matrix);
//   k_cgj_stage stages the pivot rows as they stood at their own sub-panel,
//     rb_t = A[R_t] + sum_{t' < t} U_t'[R_t] rb_t' for the columns outside
//     the panel; for a column of sub-panel s it starts from G_s and takes
//     only the later sub-panels (rb_t = 0 for t <= s);
//   k_cgj_update applies A += sum_t U_t rb_t to every column, which also
//     brings each sub-panel's columns G_s up to the panel's end.
constexpr int kCoarsePB = kCoarseStage;

// pivot key of row i (< 65536): |a| with its 16 low mantissa bits replaced by
// 65535 - i (largest |a| to a relative 2^-36, then the lowest row); 0 for
// rows that may not pivot
__device__ __forceinline__ unsigned long long coarse_key(double a, int i, bool allowed) {
  const unsigned long long m = (unsigned long long)__double_as_longlong(fabs(a));
  return allowed ? ((m & ~0xFFFFull) | (unsigned long long)(65535 - i)) : 0ull;
}
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)x, CTRL, 0xF, 0xF, false);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(x >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long x, int lane) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
  auto mx = [](unsigned long long a, unsigned long long b) { return a > b ? a : b; };
  x = mx(x, dpp_u64<0xB1>(x));
  x = mx(x, dpp_u64<0x4E>(x));
  x = mx(x, dpp_u64<0x141>(x));
  x = mx(x, dpp_u64<0x140>(x));
  return mx(mx(readlane_u64(x, 0), readlane_u64(x, 16)), mx(readlane_u64(x, 32), readlane_u64(x, 48)));
}

// Batched use (many matrices of one size n, e.g. the large Vanka patches):
// matrix z = blockIdx.z of a launch owns a[z n^2 ..], piv / used_g[z n ..],
// ub / rb[z PB n ..]; with amax != nullptr its pivot threshold is
// thr * amax[z] and a singular matrix reports its index zbase + z in
// status[1] (else the first singular column).  A launch of depth 1 is the
// single coarse matrix.
template <int RPT, int PW>
__global__ __launch_bounds__(1024) void k_cgj_panel(int64_t n, int64_t k0, double *__restrict__ a,
                                                    int *__restrict__ piv, int *__restrict__ used_g,
                                                    double *__restrict__ ub, double thr,
                                                    int *__restrict__ status,
                                                    const double *__restrict__ amax, int zbase) {
  constexpr int PB = kCoarsePB, NSUB = PB / PW;
  __shared__ unsigned long long skey[2][16];
  __shared__ double srow[2][16][PW];
  __shared__ double rbs[PW][PW];
  __shared__ int ptv[PB];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int64_t z = blockIdx.z;
  a += z * n * n;
  piv += z * n;
  used_g += z * n;
  ub += z * (int64_t)PB * n;
  if (amax) thr *= amax[z];
  const int64_t kend = min(k0 + (int64_t)PB, n);
  const int npb = (int)(kend - k0);
  int row[RPT];
  bool ok[RPT], used[RPT];
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    row[s] = t + 1024 * s;
    ok[s] = row[s] < n;
    used[s] = ok[s] ? used_g[row[s]] != 0 : true;
  }
  bool singular = false;
  int sing_k = (int)n;
  for (int sub = 0; sub < NSUB; ++sub) {
    const int64_t c0 = k0 + (int64_t)sub * PW;
    if (c0 >= kend) break;
    const int nc = (int)min<int64_t>(PW, kend - c0);
    double x[RPT][PW];
#pragma unroll
    for (int s = 0; s < RPT; ++s)
#pragma unroll
      for (int c = 0; c < PW; ++c)
        x[s][c] = (ok[s] && c < nc) ? a[(c0 + c) * n + row[s]] : 0.0;
    // left-looking: the panel's earlier sub-panels, in order, each with its
    // pivot rows as they stand at that point
    for (int tt = 0; tt < sub; ++tt) {
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int r = ptv[tt * PW + q];
#pragma unroll
        for (int s = 0; s < RPT; ++s)
          if (ok[s] && row[s] == r)
#pragma unroll
            for (int c = 0; c < PW; ++c) rbs[q][c] = x[s][c];
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < RPT; ++s)
        if (ok[s])
#pragma unroll
          for (int q = 0; q < PW; ++q) {
            const double u = ub[(int64_t)(tt * PW + q) * n + row[s]];
#pragma unroll
            for (int c = 0; c < PW; ++c) x[s][c] = fma(u, rbs[q][c], x[s][c]);
          }
      __syncthreads();
    }
#pragma unroll
    for (int jj = 0; jj < PW; ++jj) {
      if (jj >= nc) break;
      // one barrier per step: every wave publishes its best candidate's key
      // and row (double-buffered by step), every thread then picks the best
      const int bsel = jj & 1;
      unsigned long long key = 0;
      int bs = 0;
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const unsigned long long ks = coarse_key(x[s][jj], row[s], !used[s]);
        if (ks > key) {
          key = ks;
          bs = s;
        }
      }
      const unsigned long long wkey = wave_max_u64(key);
      if (wkey != 0 && key == wkey)
#pragma unroll
        for (int s = 0; s < RPT; ++s)
          if (s == bs)
#pragma unroll
            for (int c = 0; c < PW; ++c) srow[bsel][w][c] = x[s][c];
      if (l == 0) skey[bsel][w] = wkey;
      __syncthreads();
      int wb = 0;
      key = skey[bsel][0];
      for (int i = 1; i < 16; ++i)
        if (skey[bsel][i] > key) {
          key = skey[bsel][i];
          wb = i;
        }
      const int r = 65535 - (int)(key & 0xFFFFull);
      double prow[PW];
#pragma unroll
      for (int c = 0; c < PW; ++c) prow[c] = srow[bsel][wb][c];
      const double pv = prow[jj];
      if (!(fabs(pv) > thr) && !singular) {
        singular = true;
        sing_k = (int)(c0 + jj);
      }
      const double rp = 1.0 / pv;
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const double f = x[s][jj];
#pragma unroll
        for (int c = 0; c < PW; ++c) x[s][c] = c == jj ? -f * rp : fma(-f, prow[c] * rp, x[s][c]);
        if (ok[s] && row[s] == r) {
#pragma unroll
          for (int c = 0; c < PW; ++c) x[s][c] = c == jj ? rp : prow[c] * rp;
          used[s] = true;
        }
      }
      if (t == 0) ptv[sub * PW + jj] = r;  // LDS only: a global store here would
                                           // hold up every following barrier
    }
    // G_t to the matrix, U_t = G_t - E_{R_t} kept in ub
#pragma unroll
    for (int s = 0; s < RPT; ++s)
      if (ok[s])
#pragma unroll
        for (int c = 0; c < PW; ++c)
          if (c < nc) a[(c0 + c) * n + row[s]] = x[s][c];
    __syncthreads();  // the sub-panel's pivots are complete
#pragma unroll
    for (int s = 0; s < RPT; ++s)
      if (ok[s])
#pragma unroll
        for (int c = 0; c < PW; ++c)
          if (c < nc) {
            if (row[s] == ptv[sub * PW + c]) x[s][c] -= 1.0;
            ub[(int64_t)(sub * PW + c) * n + row[s]] = x[s][c];
          }
  }
  if (t < npb) piv[k0 + t] = ptv[t];
#pragma unroll
  for (int s = 0; s < RPT; ++s)
    if (ok[s]) used_g[row[s]] = used[s] ? 1 : 0;
  if (t == 0 && singular) {
    atomicOr(&status[0], 1);
    atomicMin(&status[1], amax ? zbase + (int)z : sing_k);
  }
}

// The panel's pivot rows as they stood at their own sub-panel: rb_p = A[r_p]
// + sum over the earlier sub-panels' rows q of U[r_p][q] rb_q (for a column
// of the panel's sub-panel s: from G_s, later sub-panels only).  A block
// takes 8 columns; thread (p, column) holds row p, and the sub-panels' rows
// are final, and published, one sub-panel at a time.
template <int PW>
__global__ __launch_bounds__(256) void k_cgj_stage(int64_t n, int64_t k0, int npb,
                                                   const double *__restrict__ a,
                                                   const int *__restrict__ piv,
                                                   const double *__restrict__ ub,
                                                   double *__restrict__ rb) {
  constexpr int PB = kCoarsePB, JW = 256 / PB, NSUB = PB / PW;
  __shared__ double ured[PB][PB + 1];
  __shared__ double rbl[PB][JW];
  const int64_t z = blockIdx.z;
  a += z * n * n;
  piv += z * n;
  ub += z * (int64_t)PB * n;
  rb += z * (int64_t)PB * n;
  for (int idx = threadIdx.x; idx < PB * PB; idx += 256) {
    const int p = idx / PB, q = idx - p * PB;
    ured[p][q] = (p < npb && q < npb) ? ub[(int64_t)q * n + piv[k0 + p]] : 0.0;
  }
  const int p = threadIdx.x / JW, jl = threadIdx.x - p * JW;
  const int64_t j = (int64_t)blockIdx.x * JW + jl;
  const int tp = p / PW;
  // sub-panel of column j (-1 outside the panel): rows of it and of earlier
  // sub-panels contribute nothing there
  const int tj = (j >= k0 && j < k0 + npb) ? (int)(j - k0) / PW : -1;
  const bool act = p < npb && j < n;
  double v = (act && tp > tj) ? a[j * n + piv[k0 + p]] : 0.0;
  __syncthreads();
  for (int t = 0; t < NSUB; ++t) {
    if (tp == t) rbl[p][jl] = v;
    __syncthreads();
    if (tp > t)
#pragma unroll
      for (int q = 0; q < PW; ++q) v = fma(ured[p][t * PW + q], rbl[t * PW + q][jl], v);
  }
  if (act) rb[(int64_t)p * n + j] = v;
}

// B(i, j) += sum_q U(i, q) rb[q][j] for every column j; a block takes 256
// rows (one per thread, U(i, :) in registers) and kCgjCols columns
constexpr int kCgjCols = 16;
__global__ __launch_bounds__(256) void k_cgj_update(int64_t n, int npb, double *__restrict__ a,
                                                    const double *__restrict__ ub,
                                                    const double *__restrict__ rb) {
  constexpr int PB = kCoarsePB, TC = kCgjCols;
  __shared__ double rbs[TC][PB];
  const int64_t z = blockIdx.z;
  a += z * n * n;
  ub += z * (int64_t)PB * n;
  rb += z * (int64_t)PB * n;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.y * TC;
  for (int idx = threadIdx.x; idx < TC * PB; idx += 256) {
    const int c = idx / PB, q = idx - c * PB;
    rbs[c][q] = (j0 + c < n && q < npb) ? rb[(int64_t)q * n + j0 + c] : 0.0;
  }
  __syncthreads();
  if (i >= n) return;
  double u[PB];
#pragma unroll
  for (int q = 0; q < PB; ++q) u[q] = q < npb ? ub[(int64_t)q * n + i] : 0.0;
  const int cols = (int)min<int64_t>(TC, n - j0);
  int c = 0;
  for (; c + 4 <= cols; c += 4) {
    double v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = a[(j0 + c + e) * n + i];
#pragma unroll
    for (int q = 0; q < PB; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = fma(u[q], rbs[c + e][q], v[e]);
#pragma unroll
    for (int e = 0; e < 4; ++e) a[(j0 + c + e) * n + i] = v[e];
  }
  for (; c < cols; ++c) {
    double v = a[(j0 + c) * n + i];
#pragma unroll
    for (int q = 0; q < PB; ++q) v = fma(u[q], rbs[c][q], v);
    a[(j0 + c) * n + i] = v;
  }
}

__global__ void k_cgj_zero(int64_t n, int *__restrict__ v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) v[(int64_t)blockIdx.z * n + k] = 0;
}

__global__ void k_cgj_rinv(int64_t n, const int *__restrict__ piv, int *__restrict__ rinv) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t z = (int64_t)blockIdx.z * n;
  if (k < n) rinv[z + piv[z + k]] = (int)k;
}

// out[x][y] = A^{-1}[x][y] = M(r_y, rinv(x)) = a[rinv(x) n + r_y]
__global__ __launch_bounds__(256) void k_cgj_out(int64_t n, const double *__restrict__ a,
                                                 const int *__restrict__ piv,
                                                 const int *__restrict__ rinv,
                                                 double *__restrict__ out) {
  const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t x = blockIdx.y;
  if (y < n) out[x * n + y] = a[(int64_t)rinv[x] * n + piv[y]];
}

__global__ __launch_bounds__(256) void k_absmax(const double *__restrict__ a, int64_t n,
                                                double *__restrict__ partial) {
  __shared__ double red[4];
  double m = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    m = fmax(m, fabs(a[i]));
  for (int o = kWave / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// y[free[i]] = sum_j A[i][j] x[free[j]] for the dense FP64 coarse inverse,
// one wavefront per row; the identity dofs of y are zeroed separately
__global__ __launch_bounds__(256) void k_coarse_gemv(int64_t nf, const double *__restrict__ A,
                                                     const int32_t *__restrict__ cfree,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ y) {
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  if (row >= nf) return;
  const int lane = threadIdx.x & (kWave - 1);
  const double *ar = A + row * nf;
  double s = 0.0;
  for (int64_t j = lane; j < nf; j += kWave) s += ar[j] * x[cfree[j]];
  s = wave_sum(s);
  if (lane == 0) y[cfree[row]] = s;
}

__global__ void k_zero_masked(double *__restrict__ y, const uint8_t *__restrict__ mask, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && mask[i]) y[i] = 0.0;
}

__global__ __launch_bounds__(256) void k_deform(int64_t nnodes, int dim,
                                                const uint8_t *__restrict__ mask, double kth,
                                                double k1, const double *__restrict__ v_new,
                                                int v_stride, int v_offset,
                                                const double *__restrict__ u_old,
                                                const double *__restrict__ v_old,
                                                double *__restrict__ u_new) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnodes * dim) return;
  const int64_t node = i / dim;
  const int c = (int)(i - node * dim);
  double u = 0.0;
  if (mask[node]) {
    u = kth * v_new[node * v_stride + v_offset + c];
    if (u_old) u += u_old[i];
    if (v_old) u += k1 * v_old[i];
  }
  u_new[i] = u;
}

}  // namespace

// ------------------------------------------------------------- launchers
#define FSIMG_NV_DISPATCH(nvec, KER, ...)                         \
  do {                                                            \
    if ((nvec) <= 8) KER(8, __VA_ARGS__);                         \
    else if ((nvec) <= 16) KER(16, __VA_ARGS__);                  \
    else KER(32, __VA_ARGS__);                                    \
  } while (0)

void launch_multidot(const double *V, int nvec, int64_t n, const double *w, double *partial,
                     hipStream_t s) {
#define K(NV, dummy)                                                                            \
  hipLaunchKernelGGL((k_multidot<NV>), dim3(kRedBlocks), dim3(256), 0, s, V, nvec, n, w, partial)
  FSIMG_NV_DISPATCH(nvec, K, 0);
#undef K
}
void launch_axpy_dot(const double *V, int nvec, int64_t n, const double *h, double *w,
                     double *partial, hipStream_t s) {
#define K(NV, dummy)                                                                            \
  hipLaunchKernelGGL((k_axpy_red<NV, 0>), dim3(kRedBlocks), dim3(256), 0, s, V, nvec, n, h, w,  \
                     partial)
  FSIMG_NV_DISPATCH(nvec, K, 0);
#undef K
}
void launch_axpy_norm(const double *V, int nvec, int64_t n, const double *h, double *w,
                      double *partial, hipStream_t s) {
#define K(NV, dummy)                                                                            \
  hipLaunchKernelGGL((k_axpy_red<NV, 1>), dim3(kRedBlocks), dim3(256), 0, s, V, nvec, n, h, w,  \
                     partial)
  FSIMG_NV_DISPATCH(nvec, K, 0);
#undef K
}
void launch_reduce_partials(const double *partial, int nvec, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(nvec), dim3(256), 0, s, partial, nvec, out);
}
void launch_add_small(const double *a, const double *b, double *out, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_add_small, dim3(1), dim3(64), 0, s, a, b, out, n);
}
void launch_scale_by_rsqrt(const double *w, const double *ss, double *v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_by_rsqrt, dim3(grid_for(n, 256)), dim3(256), 0, s, w, ss, v, n);
}
void launch_combine(const double *Z, int k, int64_t n, const double *y, double *x, hipStream_t s) {
#define K(NV, dummy)                                                                            \
  hipLaunchKernelGGL((k_combine<NV>), dim3(grid_for(n, 256)), dim3(256), 0, s, Z, k, n, y, x)
  FSIMG_NV_DISPATCH(k, K, 0);
#undef K
}
void launch_nonfinite_count(const double *x, int64_t n, int *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite, dim3(grid_for(n, 256)), dim3(256), 0, s, x, n, flag);
}

size_t patch_factor_lds_bytes(int np) {
  return sizeof(double) * ((size_t)np * (np + 1) + 2 * (size_t)np) + 2 * sizeof(int) * (size_t)np;
}

// one patch group (npatch patches of nl nodes, np dofs) of level L's matrix
template <typename Tout>
void factor_group(const DevLevel &L, int64_t npatch, int nl, int np, const int32_t *pnodes,
                  Tout *inv, int npc, int *status, const PatchBlocks *big, hipStream_t s) {
  if (npatch == 0) return;
  if (np <= 128 && nl <= 27) {
    const int nt = (np + 15) / 16;
#define FSIMG_MF(NTV)                                                                            \
  case NTV:                                                                                      \
    hipLaunchKernelGGL((k_patch_factor_mfma<NTV, Tout>), dim3((unsigned)npatch), dim3((NTV + 1) * 64),   \
                       0, s, npatch, L.b, nl, np, npc, pnodes, L.rowptr, L.colind, L.vals64, inv,  \
                       status);                                                                  \
    return;
    switch (nt) {
      FSIMG_MF(1) FSIMG_MF(2) FSIMG_MF(3) FSIMG_MF(4)
      FSIMG_MF(5) FSIMG_MF(6) FSIMG_MF(7) FSIMG_MF(8)
      default: break;
    }
#undef FSIMG_MF
  }
  if (big && big->work && np <= 1024) {
    hipLaunchKernelGGL(k_big_load, dim3((unsigned)npatch), dim3(256), 0, s, npatch, L.b, nl, np,
                       pnodes, L.rowptr, L.colind, L.vals64, big->work, big->amax);
    constexpr int64_t kMaxZ = 65535;  // grid depth limit: patches per launch
    const int64_t n = np;
    for (int64_t c0 = 0; c0 < npatch; c0 += kMaxZ) {
      const unsigned nz = (unsigned)std::min<int64_t>(kMaxZ, npatch - c0);
      double *a = big->work + c0 * n * n;
      int *pv = big->piv + c0 * n, *iw = big->iwork + c0 * n;
      double *ub = big->ub + c0 * kCoarsePB * n, *rb = big->rb + c0 * kCoarsePB * n;
      hipLaunchKernelGGL(k_cgj_zero, dim3((unsigned)grid_for(n, 256), 1, nz), dim3(256), 0, s, n, iw);
      for (int64_t k0 = 0; k0 < n; k0 += kCoarsePB) {
        const int npb = (int)std::min<int64_t>(kCoarsePB, n - k0);
        hipLaunchKernelGGL((k_cgj_panel<1, 8>), dim3(1, 1, nz), dim3(1024), 0, s, n, k0, a, pv, iw, ub,
                           1e-15, status, big->amax + c0, (int)c0);
        hipLaunchKernelGGL((k_cgj_stage<8>), dim3((unsigned)grid_for(n, 8), 1, nz), dim3(256), 0, s, n, k0,
                           npb, a, pv, ub, rb);
        hipLaunchKernelGGL(k_cgj_update,
                           dim3((unsigned)grid_for(n, 256), (unsigned)grid_for(n, kCgjCols), nz), dim3(256),
                           0, s, n, npb, a, ub, rb);
      }
      hipLaunchKernelGGL(k_cgj_rinv, dim3((unsigned)grid_for(n, 256), 1, nz), dim3(256), 0, s, n, pv, iw);
      hipLaunchKernelGGL((k_bgj_out<Tout>), dim3(nz), dim3(256), 0, s, np, npc, a, pv, iw,
                         inv + c0 * n * npc);
    }
    return;
  }
  const size_t lds = patch_factor_lds_bytes(np);
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_patch_factor<Tout>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_patch_factor<Tout>), dim3((unsigned)npatch), dim3(256), lds, s, npatch,
                     L.b, nl, np, npc, pnodes, L.rowptr, L.colind, L.vals64, inv, status);
}

template <typename Tout>
void launch_patch_factor(const DevLevel &L, Tout *inv, int npc, int *status, hipStream_t s) {
  factor_group<Tout>(L, L.npatch, L.nl, L.np, L.pnodes, inv, npc, status, nullptr, s);
}

template <typename Tout>
void launch_patch_factor_blocks(const DevLevel &L, Tout *inv, int npc, int *status,
                                hipStream_t s) {
  factor_group<Tout>(L, L.blk.npatch, L.blk.nl, L.blk.np, L.blk.pnodes, inv, npc, status, &L.blk,
                     s);
}
template void launch_patch_factor_blocks<double>(const DevLevel &, double *, int, int *,
                                                 hipStream_t);
template void launch_patch_factor_blocks<float>(const DevLevel &, float *, int, int *, hipStream_t);
template void launch_patch_factor<double>(const DevLevel &, double *, int, int *, hipStream_t);
template void launch_patch_factor<float>(const DevLevel &, float *, int, int *, hipStream_t);

void launch_densify(const DevLevel &L, double *dense, hipStream_t s) {
  hipLaunchKernelGGL(k_densify, dim3(grid_for(L.nrows, 4)), dim3(256), 0, s, L.nrows, L.b, L.nfree,
                     L.rowptr, L.colind, L.vals64, L.cidx, dense);
}
void launch_gj_pivot(int64_t n, int64_t k, double *a, int *piv, double *rowk, double *colk,
                     double thr, int *status, hipStream_t s) {
  hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, s, n, k, a, piv, rowk, colk, thr, status);
}
void launch_gj_update(int64_t n, int64_t k, double *a, const double *rowk, const double *colk,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_gj_update, dim3(grid_for(n, 256), (unsigned)n), dim3(256), 0, s, n, k, a,
                     rowk, colk);
}
void launch_gj_finish(int64_t n, const double *a, const int *piv, int *colmap, double *out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_gj_colmap, dim3(1), dim3(64), 0, s, n, piv, colmap);
  hipLaunchKernelGGL(k_gj_out, dim3(grid_for(n, 256), (unsigned)n), dim3(256), 0, s, n, a, colmap,
                     out);
}
bool launch_coarse_gj_blocked(int64_t n, double *a, int *piv, int *iwork, double *ub, double *rb,
                              double thr, int *status, double *out, hipStream_t s) {
  const int rpt = (int)((n + 1023) / 1024);
  if (n < 1 || rpt > 4) return false;
  hipLaunchKernelGGL(k_cgj_zero, dim3(grid_for(n, 256)), dim3(256), 0, s, n, iwork);
  for (int64_t k0 = 0; k0 < n; k0 += kCoarsePB) {
    const int npb = (int)std::min<int64_t>(kCoarsePB, n - k0);
    // rows per thread 1 to 3: sub-panels of 8 columns; 4: of 4 (registers)
    if (rpt <= 3) {
      if (rpt == 1)
        hipLaunchKernelGGL((k_cgj_panel<1, 8>), dim3(1), dim3(1024), 0, s, n, k0, a, piv, iwork, ub, thr, status, nullptr, 0);
      else if (rpt == 2)
        hipLaunchKernelGGL((k_cgj_panel<2, 8>), dim3(1), dim3(1024), 0, s, n, k0, a, piv, iwork, ub, thr, status, nullptr, 0);
      else
        hipLaunchKernelGGL((k_cgj_panel<3, 8>), dim3(1), dim3(1024), 0, s, n, k0, a, piv, iwork, ub, thr, status, nullptr, 0);
      hipLaunchKernelGGL((k_cgj_stage<8>), dim3(grid_for(n, 8)), dim3(256), 0, s, n, k0, npb, a, piv, ub, rb);
    } else {
      hipLaunchKernelGGL((k_cgj_panel<4, 4>), dim3(1), dim3(1024), 0, s, n, k0, a, piv, iwork, ub, thr, status, nullptr, 0);
      hipLaunchKernelGGL((k_cgj_stage<4>), dim3(grid_for(n, 8)), dim3(256), 0, s, n, k0, npb, a, piv, ub, rb);
    }
    hipLaunchKernelGGL(k_cgj_update, dim3(grid_for(n, 256), (unsigned)grid_for(n, kCgjCols)),
                       dim3(256), 0, s, n, npb, a, ub, rb);
  }
  hipLaunchKernelGGL(k_cgj_rinv, dim3(grid_for(n, 256)), dim3(256), 0, s, n, piv, iwork);
  hipLaunchKernelGGL(k_cgj_out, dim3(grid_for(n, 256), (unsigned)n), dim3(256), 0, s, n, a, piv,
                     iwork, out);
  return true;
}
void launch_absmax(const double *a, int64_t n, double *partial, hipStream_t s) {
  hipLaunchKernelGGL(k_absmax, dim3(kRedBlocks), dim3(256), 0, s, a, n, partial);
}
void launch_coarse_gemv(const DevLevel &C, const double *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_masked, dim3(grid_for(C.n, 256)), dim3(256), 0, s, y, C.mask, C.n);
  if (C.nfree > 0)
    hipLaunchKernelGGL(k_coarse_gemv, dim3(grid_for(C.nfree, 4)), dim3(256), 0, s, C.nfree, C.cinv,
                       C.cfree, x, y);
}
void launch_deform(int64_t nnodes, int dim, const uint8_t *mask, double k, double theta,
                   const double *v_new, int v_stride, int v_offset, const double *u_old,
                   const double *v_old, double *u_new, hipStream_t s) {
  const int64_t n = nnodes * dim;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_deform, dim3(grid_for(n, 256)), dim3(256), 0, s, nnodes, dim, mask,
                     k * theta, k * (1.0 - theta), v_new, v_stride, v_offset, u_old, v_old, u_new);
}

}  // namespace fsimg
