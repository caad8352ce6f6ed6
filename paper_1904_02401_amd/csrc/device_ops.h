// Device bodies of the bandwidth-bound operations, shared by the
// single-hierarchy kernels and the batched (many-instance) kernels: one
// block-CSR row, one workgroup of Vanka patches, one dof of the patch
// gather, one node of the Q2 restriction / prolongation.
#pragma once
#include "fsimg_internal.h"

namespace fsimg {
namespace dev {

constexpr int kWave = 64;

// Pointers reach the batched kernels inside descriptor structs, where the
// compiler cannot see that they address global memory and would emit flat
// loads (which also count against the LDS counter, so every cross-lane
// shuffle would wait for them).  The bodies below therefore access memory
// through global-address-space views of their pointer arguments.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> glb(T *p) {
  return (gptr<T>)p;
}

// 16-byte vectors as clang native vector types (loadable through
// global-address-space pointers)
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <typename T> struct Vec16;
template <> struct Vec16<double> { using type = dvec2; static constexpr int G = 2; };
template <> struct Vec16<float> { using type = fvec4; static constexpr int G = 4; };

__device__ __forceinline__ double vget(const dvec2 &v, int q) { return q == 0 ? v.x : v.y; }
__device__ __forceinline__ float vget(const fvec4 &v, int q) {
  return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}

template <typename T>
__device__ __forceinline__ T dot16(const typename Vec16<T>::type &a, const typename Vec16<T>::type &b);
template <>
__device__ __forceinline__ double dot16<double>(const dvec2 &a, const dvec2 &b) {
  return a.x * b.x + a.y * b.y;
}
template <>
__device__ __forceinline__ float dot16<float>(const fvec4 &a, const fvec4 &b) {
  return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Renumbering them so that XCD k takes the k-th contiguous eighth of
// the logical block range keeps neighbouring rows (and the x entries they
// share) in one L2.  A bijection of [0, nblocks).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblocks) {
  const int64_t q = nblocks >> 3, r = nblocks & 7, xc = b & 7, j = b >> 3;
  return xc * q + (xc < r ? xc : r) + j;
}

// ------------------------------------------------------------ BSR SpMV
// One wavefront per R consecutive block rows.  The R + 1 row pointers come
// in with one load; each row's column indices (at most 128 blocks, the Q2
// maximum is 125) with one or two coalesced loads, broadcast by cross-lane
// shuffles.  Then every value / x load of all R rows is issued in one fully
// unrolled, predicated sweep, so a wave keeps R rows' bytes in flight after
// two dependent round trips.  Rows longer than 128 blocks take a plain loop
// with the same lane mapping and summation order.
//
// b = 4: each lane loads 16 bytes of a block (2 doubles / 4 floats) and the
// matching 16 bytes of x, so a wave covers 8 (FP64) or 16 (FP32) blocks per
// step with 1 KB coalesced value loads.  b = 1, 2, 3: each lane owns one
// block row (b values and the b entries of x), 64 / b blocks per step.
// Lane partials are summed across lanes in a fixed tree; lanes 0..b-1 write
// the b results of the row.  The result of a row does not depend on R.
//
// MODE 0: y = A x;  1: y = b - A x, 0 at identity rows;  2: y = A x, 0 at
// identity rows.
template <int B, typename T>
struct RowMap {
  static constexpr bool kVec = (B == 4);
  static constexpr int LPB = kVec ? 16 / Vec16<T>::G : B;  // lanes per block
  static constexpr int KB = kWave / LPB;                     // blocks per wave step
  static constexpr int ACT = KB * LPB;                       // lanes in use
  static constexpr int MAXT = (128 + KB - 1) / KB;           // steps covering 128 blocks
};

// lane partial of one block (index jj of the row, column col)
template <int B, typename T>
__device__ __forceinline__ T block_partial(gptr<const T> vals, gptr<const T> x, int64_t blk, int col,
                                           int q) {
  if constexpr (B == 4) {
    using V = typename Vec16<T>::type;
    constexpr int G = Vec16<T>::G;
    const V a = *reinterpret_cast<gptr<const V>>(vals + blk * 16 + q * G);
    const V xv = *reinterpret_cast<gptr<const V>>(x + (int64_t)col * 4 + ((q * G) & 3));
    return dot16<T>(a, xv);
  } else {
    gptr<const T> v = vals + blk * (B * B) + q * B;
    gptr<const T> xv = x + (int64_t)col * B;
    T s = v[0] * xv[0];
#pragma unroll
    for (int c = 1; c < B; ++c) s += v[c] * xv[c];
    return s;
  }
}

// sum the lane partials of a row; lanes 0..B-1 receive the B results
template <int B, typename T>
__device__ __forceinline__ T row_total(T acc, int lane) {
  if constexpr (B == 4) {
    constexpr int G = Vec16<T>::G;
    constexpr int LPB = 16 / G;
    // lanes holding block row r: q * G / 4 == r; sum over them and over blocks
    for (int m = 1; m < 4 / G; m <<= 1) acc += __shfl_xor(acc, m);
    for (int m = LPB; m < kWave; m <<= 1) acc += __shfl_xor(acc, m);
    return __shfl(acc, (lane & 3) * (4 / G));
  } else if constexpr ((B & (B - 1)) == 0) {
    for (int m = B; m < kWave; m <<= 1) acc += __shfl_xor(acc, m);
    return acc;
  } else {
    // B = 3: 21 block groups of 3 lanes; tree over groups (absent ones are 0)
    constexpr int ACT = RowMap<B, T>::ACT;
#pragma unroll
    for (int sft = 16; sft >= 1; sft >>= 1) {
      const int src = lane + B * sft;
      const T o = __shfl(acc, src & (kWave - 1));
      if (src < ACT) acc += o;
    }
    return acc;
  }
}

// NS wave steps over R rows with no branch inside: indices past the end of
// a row are clamped to its last block (a cached re-read) and their products
// masked out, so the compiler can issue every value / x load of the R rows
// before the first use.  acc starts at +0 and masked steps add +0, so the
// sums equal those of a loop over the row's blocks only.
template <int B, typename T, int NS, int R>
__device__ __forceinline__ void sweep_rows(const int (&rs)[R], const int (&nb)[R],
                                           const int (&c0)[R], const int (&c1)[R], int k0, int q,
                                           bool on, gptr<const T> vals, gptr<const T> x,
                                           T (&acc)[R]) {
  using M = RowMap<B, T>;
  int col[R][NS];
  int64_t blk[R][NS];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int jj = t * M::KB + k0;
      const int jc = nb[r] > 0 ? min(jj, nb[r] - 1) : 0;
      const int ca = __shfl(c0[r], jc & (kWave - 1));
      int cv = ca;
      if (t * M::KB + M::KB > kWave) {
        const int cb = __shfl(c1[r], jc & (kWave - 1));
        cv = jc < kWave ? ca : cb;
      }
      col[r][t] = cv;
      blk[r][t] = nb[r] > 0 ? (int64_t)rs[r] + jc : 0;
    }
  T p[R][NS];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int t = 0; t < NS; ++t) p[r][t] = block_partial<B, T>(vals, x, blk[r][t], col[r][t], q);
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int t = 0; t < NS; ++t) acc[r] += (on && t * M::KB + k0 < nb[r]) ? p[r][t] : T(0);
}

template <int B, typename T, int MODE, int R>
__device__ __forceinline__ void spmv_rows_wave(int64_t row0, int64_t nrows, int lane,
                                          const int32_t *rowptr_, const int32_t *colind_,
                                          const T *vals_, const T *x_, const T *b_,
                                          const uint8_t *mask_, T *y_) {
  using M = RowMap<B, T>;
  const gptr<const int32_t> rowptr = glb(rowptr_), colind = glb(colind_);
  const gptr<const T> vals = glb(vals_), x = glb(x_), b = glb(b_);
  const gptr<const uint8_t> mask = glb(mask_);
  const gptr<T> y = glb(y_);
  const int k0 = lane / M::LPB, q = lane - k0 * M::LPB;
  const bool on = lane < M::ACT;
  int rp = 0;
  if (lane <= R) rp = rowptr[row0 + lane <= nrows ? row0 + lane : nrows];
  int rs[R], nb[R];
  int nbmax = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    rs[r] = __shfl(rp, r);
    nb[r] = __shfl(rp, r + 1) - rs[r];
    nbmax = max(nbmax, nb[r]);
  }
  // the row's identity flags and right-hand side, fetched now so that
  // their latency overlaps the sweep instead of following the reduction
  uint8_t mrow[R];
  T brow[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    mrow[r] = 0;
    brow[r] = T(0);
    if (lane < B && row0 + r < nrows) {
      const int64_t dof = (row0 + r) * B + lane;
      if (MODE != 0) mrow[r] = mask[dof];
      if (MODE == 1) brow[r] = b[dof];
    }
  }
  T acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = T(0);
  if (nbmax <= 128) {
    int c0[R], c1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      c0[r] = lane < nb[r] ? colind[rs[r] + lane] : 0;
      c1[r] = lane + kWave < nb[r] ? colind[rs[r] + kWave + lane] : 0;
    }
    // steps in use, rounded up to a quarter of the 128-block maximum
    constexpr int S1 = (M::MAXT + 3) / 4, S2 = (M::MAXT + 1) / 2, S3 = (3 * M::MAXT + 3) / 4;
    const int steps = (nbmax + M::KB - 1) / M::KB;
    if (steps <= S1)
      sweep_rows<B, T, S1, R>(rs, nb, c0, c1, k0, q, on, vals, x, acc);
    else if (steps <= S2)
      sweep_rows<B, T, S2, R>(rs, nb, c0, c1, k0, q, on, vals, x, acc);
    else if (steps <= S3)
      sweep_rows<B, T, S3, R>(rs, nb, c0, c1, k0, q, on, vals, x, acc);
    else
      sweep_rows<B, T, M::MAXT, R>(rs, nb, c0, c1, k0, q, on, vals, x, acc);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (on)
        for (int jj = k0; jj < nb[r]; jj += M::KB)
          acc[r] += block_partial<B, T>(vals, x, (int64_t)rs[r] + jj, colind[rs[r] + jj], q);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const T tot = row_total<B, T>(acc[r], lane);
    const int64_t row = row0 + r;
    if (lane < B && row < nrows) {
      const int64_t dof = row * B + lane;
      if (MODE == 1)
        y[dof] = mrow[r] ? T(0) : brow[r] - tot;
      else if (MODE == 2)
        y[dof] = mrow[r] ? T(0) : tot;
      else
        y[dof] = tot;
    }
  }
}

// FP32 (and b <= 2): 64 / LR rows per wavefront, LR lanes per row, one lane
// per block (its b x b values and the b entries of x); a lane takes blocks
// li, li + LR, ... of its row.  For the short FP32 rows this keeps more rows
// in flight per wave than the whole-wave mapping above.  Lane partials are
// summed by an xor tree inside the row's lane group.
template <int B, typename T, int MODE, int LR>
__device__ __forceinline__ void spmv_group(int64_t row0, int64_t nrows, int lane,
                                           gptr<const int32_t> rowptr, gptr<const int32_t> colind,
                                           gptr<const T> vals, gptr<const T> x, gptr<const T> b,
                                           gptr<const uint8_t> mask, gptr<T> y) {
  constexpr int RPW = kWave / LR;  // rows of this group
  constexpr int NI = 128 / LR;     // blocks per lane at most
  const int li = lane % LR, rsub = lane / LR;
  const int rp = lane <= RPW ? rowptr[min(row0 + lane, nrows)] : 0;
  const int64_t row = row0 + rsub;
  const bool live = row < nrows;
  const int rs = __shfl(rp, rsub);
  const int nb = live ? __shfl(rp, rsub + 1) - rs : 0;
  int nbmax = nb;
  for (int m = LR; m < kWave; m <<= 1) nbmax = max(nbmax, __shfl_xor(nbmax, m));
  uint8_t mv = 0;
  T bv = T(0);
  if (li < B && live) {
    if (MODE != 0) mv = mask[row * B + li];
    if (MODE == 1) bv = b[row * B + li];
  }
  T acc[B];
#pragma unroll
  for (int r = 0; r < B; ++r) acc[r] = T(0);
  if (nbmax <= 128) {
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      if (it * LR < nbmax) {
        const int jj = it * LR + li;
        const bool ok = jj < nb;
        const int64_t blk = nb > 0 ? (int64_t)rs + (ok ? jj : nb - 1) : 0;
        const int col = colind[blk];
        gptr<const T> v = vals + blk * (B * B);
        gptr<const T> xv = x + (int64_t)col * B;
        T xr[B], vv[B * B];
#pragma unroll
        for (int c = 0; c < B; ++c) xr[c] = xv[c];
#pragma unroll
        for (int e = 0; e < B * B; ++e) vv[e] = v[e];
#pragma unroll
        for (int r = 0; r < B; ++r) {
          T p = vv[r * B] * xr[0];
#pragma unroll
          for (int c = 1; c < B; ++c) p += vv[r * B + c] * xr[c];
          acc[r] += ok ? p : T(0);
        }
      }
    }
  } else {
    for (int jj = li; jj < nb; jj += LR) {
      const int64_t blk = (int64_t)rs + jj;
      gptr<const T> v = vals + blk * (B * B);
      gptr<const T> xv = x + (int64_t)colind[blk] * B;
#pragma unroll
      for (int r = 0; r < B; ++r) {
        T p = v[r * B] * xv[0];
#pragma unroll
        for (int c = 1; c < B; ++c) p += v[r * B + c] * xv[c];
        acc[r] += p;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < B; ++r)
    for (int m = LR / 2; m > 0; m >>= 1) acc[r] += __shfl_xor(acc[r], m);
  T tot = acc[0];
#pragma unroll
  for (int r = 1; r < B; ++r) tot = li == r ? acc[r] : tot;
  if (li < B && live) {
    const int64_t dof = row * B + li;
    if (MODE == 1)
      y[dof] = mv ? T(0) : bv - tot;
    else if (MODE == 2)
      y[dof] = mv ? T(0) : tot;
    else
      y[dof] = tot;
  }
}

// R row groups per wavefront (a group = 64 / lanes-per-row rows), starting
// at row0; the result of a row does not depend on R.
template <int B, typename T, int MODE, int R>
__device__ __forceinline__ void spmv_rows(int64_t row0, int64_t nrows, int lane,
                                          const int32_t *rowptr_, const int32_t *colind_,
                                          const T *vals_, const T *x_, const T *b_,
                                          const uint8_t *mask_, T *y_) {
  constexpr int LR = kWave / spmv_group_rows(B, (int)sizeof(T));
  if constexpr (LR == kWave) {
    spmv_rows_wave<B, T, MODE, R>(row0, nrows, lane, rowptr_, colind_, vals_, x_, b_, mask_, y_);
  } else {
    constexpr int RPW = kWave / LR;
#pragma unroll
    for (int g = 0; g < R; ++g)
      if (row0 + g * RPW < nrows)
        spmv_group<B, T, MODE, LR>(row0 + g * RPW, nrows, lane, glb(rowptr_), glb(colind_),
                                   glb(vals_), glb(x_), glb(b_), glb(mask_), glb(y_));
  }
}

// ------------------------------------------------------------ Vanka apply
// Each active patch i computes y_i = A_i^{-1} d_i, d_i = R_i d (eq. vanka).
// A workgroup holds ppw patches (e.g. 7 patches of 108 rows in 768 threads,
// 98% of the lanes busy); thread r of a patch owns row r.  The inverse is
// stored "column-group-major": entry (r, c) at ((c / G) * np + r) * G + c % G
// with G = 16 bytes / sizeof(T), so at each step the np threads of a patch
// read one contiguous np*16-byte segment with 16-byte loads.  d_i is gathered
// once into LDS (dl: ppw * npc entries).  Must be called by every thread of
// the workgroup.
template <typename T>
__device__ __forceinline__ void vanka_patch_wg(int64_t pfirst, int64_t pend, int np, int npc, int b,
                                               int nl, int ppw, const int32_t *pnodes_,
                                               const T *inv_, const T *d_, T *Y_, int scatter,
                                               T *x_, const T *scale_, const uint8_t *mask_,
                                               T omega, T *dl) {
  using V = typename Vec16<T>::type;
  const gptr<const int32_t> pnodes = glb(pnodes_);
  const gptr<const T> inv = glb(inv_), d = glb(d_), scale = glb(scale_);
  const gptr<const uint8_t> mask = glb(mask_);
  const gptr<T> Y = glb(Y_), x = glb(x_);
  constexpr int G = Vec16<T>::G;
  const int t = threadIdx.x;
  const int s = t / np;
  const int r = t - s * np;
  const int64_t p = pfirst + s;
  const bool act = (s < ppw) && (p < pend);
  int node = 0, c = 0;
  if (act) {
    const int ln = r / b;
    c = r - ln * b;
    node = pnodes[p * nl + ln];
    dl[s * npc + r] = d[(int64_t)node * b + c];
  }
  if (s < ppw && r < npc - np) dl[s * npc + np + r] = T(0);
  // the first column groups of the inverse do not depend on d: fetch them
  // before the barrier so that their latency overlaps the gather
  constexpr int PF = 6;
  const int ng = npc / G;
  gptr<const V> A = reinterpret_cast<gptr<const V>>(inv + (act ? p : 0) * (int64_t)np * npc) + r;
  V pre[PF];
#pragma unroll
  for (int k = 0; k < PF; ++k) pre[k] = (act && k < ng) ? A[(int64_t)k * np] : V{};
  __syncthreads();
  if (!act) return;
  const T *dv = dl + s * npc;
  T acc = 0;
#pragma unroll
  for (int k = 0; k < PF; ++k)
    if (k < ng) {
#pragma unroll
      for (int q = 0; q < G; ++q) acc += vget(pre[k], q) * dv[k * G + q];
    }
#pragma unroll 6
  for (int g = PF; g < ng; ++g) {
    const V v = A[(int64_t)g * np];
#pragma unroll
    for (int q = 0; q < G; ++q) acc += vget(v, q) * dv[g * G + q];
  }
  if (!scatter) {
    Y[p * np + r] = acc;
  } else {
    const int64_t dof = (int64_t)node * b + c;
    if (!mask[dof]) x[dof] += omega * scale[node] * acc;
  }
}

// Sum, per dof, the corrections of all patches containing its node, in
// patch order: x += omega * w(node) * sum_i (R_i^T y_i); identity dofs keep x
// (assign: x starts from 0).
template <typename T>
__device__ __forceinline__ void vanka_gather_dof(int64_t dof, int b, const int32_t *gptr_,
                                                 const int32_t *gidx_, const T *Y_, const T *scale_,
                                                 const uint8_t *mask_, T omega, int assign, T *x_) {
  const gptr<const int32_t> gp = glb(gptr_), gidx = glb(gidx_);
  const gptr<const T> Y = glb(Y_), scale = glb(scale_);
  const gptr<const uint8_t> mask = glb(mask_);
  const gptr<T> x = glb(x_);
  const int64_t node = dof / b;
  const int c = (int)(dof - node * b);
  T s = 0;
  const int e1 = gp[node + 1];
  for (int e = gp[node]; e < e1; ++e) s += Y[(int64_t)gidx[e] * b + c];
  const T xv = assign ? T(0) : x[dof];
  x[dof] = mask[dof] ? xv : xv + omega * scale[node] * s;
}

// ------------------------------------------------------------ Q2 transfers
// 1D canonical Q2 interpolation between a coarse axis with nc cells and its
// bisection: fine node i takes coarse node i/2 (i even), else the quadratic
// Lagrange values at the quarter points of coarse cell i/4.
template <typename T>
__device__ __forceinline__ int prolong_1d(int i, int *idx, T *w) {
  if ((i & 1) == 0) { idx[0] = i >> 1; w[0] = T(1); return 1; }
  const int e = i >> 2;
  idx[0] = 2 * e; idx[1] = 2 * e + 1; idx[2] = 2 * e + 2;
  if ((i & 3) == 1) { w[0] = T(0.375); w[1] = T(0.75); w[2] = T(-0.125); }
  else { w[0] = T(-0.125); w[1] = T(0.75); w[2] = T(0.375); }
  return 3;
}
// transpose: the fine nodes that coarse node I interpolates into
template <typename T>
__device__ __forceinline__ int restrict_1d(int I, int nc, int *idx, T *w) {
  int k = 0;
  idx[k] = 2 * I; w[k++] = T(1);
  if ((I & 1) == 0) {
    const int e = I >> 1;
    if (e < nc) { idx[k] = 4 * e + 1; w[k++] = T(0.375); idx[k] = 4 * e + 3; w[k++] = T(-0.125); }
    if (e >= 1) { idx[k] = 4 * e - 3; w[k++] = T(-0.125); idx[k] = 4 * e - 1; w[k++] = T(0.375); }
  } else {
    const int e = (I - 1) >> 1;
    idx[k] = 4 * e + 1; w[k++] = T(0.75); idx[k] = 4 * e + 3; w[k++] = T(0.75);
  }
  return k;
}

// r_c(node) = sum over the fine nodes it interpolates into; 0 at identity rows
template <int B, int DIM, typename T>
__device__ __forceinline__ void restrict_node(int64_t node, int cx, int cy, int cz,
                                              const T *rf_, T *rc_, const uint8_t *maskc_) {
  const gptr<const T> rf = glb(rf_);
  const gptr<T> rc = glb(rc_);
  const gptr<const uint8_t> maskc = glb(maskc_);
  const int NX = 2 * cx + 1, NY = 2 * cy + 1;
  const int FX = 4 * cx + 1, FY = 4 * cy + 1;
  const int I = (int)(node % NX), J = (int)((node / NX) % NY), K = (int)(node / ((int64_t)NX * NY));
  int ix[5], iy[5], iz[5];
  T wx[5], wy[5], wz[5];
  const int nx = restrict_1d<T>(I, cx, ix, wx), ny = restrict_1d<T>(J, cy, iy, wy);
  int nz = 1;
  iz[0] = 0; wz[0] = T(1);
  if (DIM == 3) nz = restrict_1d<T>(K, cz, iz, wz);
  T acc[B];
#pragma unroll
  for (int c = 0; c < B; ++c) acc[c] = 0;
  for (int a = 0; a < nz; ++a)
    for (int bb = 0; bb < ny; ++bb) {
      const T wyz = wy[bb] * wz[a];
      const int64_t base = ((int64_t)iz[a] * FY + iy[bb]) * FX;
      for (int q = 0; q < nx; ++q) {
        const T w = wyz * wx[q];
        gptr<const T> src = rf + (base + ix[q]) * B;
#pragma unroll
        for (int c = 0; c < B; ++c) acc[c] += w * src[c];
      }
    }
#pragma unroll
  for (int c = 0; c < B; ++c) {
    const int64_t dof = node * B + c;
    rc[dof] = maskc[dof] ? T(0) : acc[c];
  }
}

// x_f(node) += interpolated coarse correction; 0 at identity rows
template <int B, int DIM, typename T>
__device__ __forceinline__ void prolong_node(int64_t node, int cx, int cy, int cz,
                                             const T *xc_, T *xf_, const uint8_t *maskf_) {
  const gptr<const T> xc = glb(xc_);
  const gptr<T> xf = glb(xf_);
  const gptr<const uint8_t> maskf = glb(maskf_);
  const int NX = 2 * cx + 1, NY = 2 * cy + 1;
  const int FX = 4 * cx + 1, FY = 4 * cy + 1;
  const int i = (int)(node % FX), j = (int)((node / FX) % FY), k = (int)(node / ((int64_t)FX * FY));
  int ix[3], iy[3], iz[3];
  T wx[3], wy[3], wz[3];
  const int nx = prolong_1d<T>(i, ix, wx), ny = prolong_1d<T>(j, iy, wy);
  int nz = 1;
  iz[0] = 0; wz[0] = T(1);
  if (DIM == 3) nz = prolong_1d<T>(k, iz, wz);
  T acc[B];
#pragma unroll
  for (int c = 0; c < B; ++c) acc[c] = 0;
  for (int a = 0; a < nz; ++a)
    for (int bb = 0; bb < ny; ++bb) {
      const T wyz = wy[bb] * wz[a];
      const int64_t base = ((int64_t)iz[a] * NY + iy[bb]) * NX;
      for (int q = 0; q < nx; ++q) {
        const T w = wyz * wx[q];
        gptr<const T> src = xc + (base + ix[q]) * B;
#pragma unroll
        for (int c = 0; c < B; ++c) acc[c] += w * src[c];
      }
    }
#pragma unroll
  for (int c = 0; c < B; ++c) {
    const int64_t dof = node * B + c;
    xf[dof] = maskf[dof] ? T(0) : xf[dof] + acc[c];
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int m = kWave / 2; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Block sum of one value per thread, result valid in thread 0.
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

}  // namespace dev
}  // namespace fsimg
