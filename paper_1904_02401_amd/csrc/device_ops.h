// Device bodies of the bandwidth-bound operations, shared by the
// single-hierarchy kernels and the batched (many-instance) kernels: one
// block-CSR row, one workgroup of Vanka patches, one dof of the patch
// gather, one node of the Q2 restriction / prolongation.
#pragma once
#include "fsimg_internal.h"

namespace fsimg {
namespace dev {

constexpr int kWave = 64;

template <typename T> struct Vec16;
template <> struct Vec16<double> { using type = double2; static constexpr int G = 2; };
template <> struct Vec16<float> { using type = float4; static constexpr int G = 4; };

__device__ __forceinline__ double vget(const double2 &v, int q) { return q == 0 ? v.x : v.y; }
__device__ __forceinline__ float vget(const float4 &v, int q) {
  return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}

template <typename T>
__device__ __forceinline__ T dot16(const typename Vec16<T>::type &a, const typename Vec16<T>::type &b);
template <>
__device__ __forceinline__ double dot16<double>(const double2 &a, const double2 &b) {
  return a.x * b.x + a.y * b.y;
}
template <>
__device__ __forceinline__ float dot16<float>(const float4 &a, const float4 &b) {
  return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
}

// ------------------------------------------------------------ BSR SpMV
// One wavefront per block row.  The row's column indices (at most 128
// blocks, the Q2 maximum is 125) are loaded once with one coalesced load and
// broadcast by cross-lane shuffles, so no global load depends on another
// inside the row: every value / x load of the row is issued in one fully
// unrolled, predicated sweep.  Rows longer than 128 blocks take a plain loop.
//
// b = 4: each lane loads 16 bytes of a block (2 doubles / 4 floats) and the
// matching 16 bytes of x, so a wave covers 8 (FP64) or 16 (FP32) blocks per
// step with 1 KB coalesced value loads.  Other b: one entry per lane,
// 64 / b^2 blocks per step.  Partial products are summed across lanes with
// xor-shuffles; lanes 0..b-1 write the b results of the row.
//
// MODE 0: y = A x;  1: y = b - A x, 0 at identity rows;  2: y = A x, 0 at
// identity rows.
template <int B, typename T>
__device__ __forceinline__ T row_reduce(T acc, int lane) {
  constexpr int BB = B * B;
  if constexpr ((B & (B - 1)) == 0) {
    for (int m = 1; m < B; m <<= 1) acc += __shfl_xor(acc, m);
    for (int m = BB; m < kWave; m <<= 1) acc += __shfl_xor(acc, m);
    return __shfl(acc, (lane % B) * B);
  } else {
    constexpr int KB = kWave / BB;
    T s = 0;
#pragma unroll
    for (int k0 = 0; k0 < KB; ++k0)
#pragma unroll
      for (int c = 0; c < B; ++c) s += __shfl(acc, k0 * BB + (lane % B) * B + c);
    return s;
  }
}

template <int B, typename T, int MODE>
__device__ __forceinline__ void spmv_row(int64_t row, int lane, const int32_t *__restrict__ rowptr,
                                         const int32_t *__restrict__ colind,
                                         const T *__restrict__ vals, const T *__restrict__ x,
                                         const T *__restrict__ b, const uint8_t *__restrict__ mask,
                                         T *__restrict__ y) {
  const int64_t rs = rowptr[row];
  const int nb = (int)(rowptr[row + 1] - rs);
  T tot;
  if constexpr (B == 4) {
    using V = typename Vec16<T>::type;
    constexpr int G = Vec16<T>::G;   // entries per 16-byte load
    constexpr int LPB = 16 / G;      // lanes per 4x4 block
    constexpr int KB = kWave / LPB;  // blocks per wave step
    constexpr int MAXT = 128 / KB;
    const int k0 = lane / LPB, q = lane - k0 * LPB;
    const int cofs = (q * G) & 3;
    const T *vrow = vals + rs * 16 + q * G;
    T acc = 0;
    if (nb <= 128) {
      const int c0 = lane < nb ? colind[rs + lane] : 0;
      const int c1 = lane + kWave < nb ? colind[rs + kWave + lane] : 0;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        const int jj = t * KB + k0;
        const int col = __shfl(t * KB < kWave ? c0 : c1, jj & (kWave - 1));
        if (jj < nb) {
          const V a = *reinterpret_cast<const V *>(vrow + (int64_t)jj * 16);
          const V xv = *reinterpret_cast<const V *>(x + (int64_t)col * 4 + cofs);
          acc += dot16<T>(a, xv);
        }
      }
    } else {
      for (int jj = k0; jj < nb; jj += KB) {
        const int col = colind[rs + jj];
        const V a = *reinterpret_cast<const V *>(vrow + (int64_t)jj * 16);
        const V xv = *reinterpret_cast<const V *>(x + (int64_t)col * 4 + cofs);
        acc += dot16<T>(a, xv);
      }
    }
    // lanes holding block row r: q * G / 4 == r; sum over them and over k0
    for (int m = 1; m < 4 / G; m <<= 1) acc += __shfl_xor(acc, m);
    for (int m = LPB; m < kWave; m <<= 1) acc += __shfl_xor(acc, m);
    tot = __shfl(acc, (lane & 3) * (4 / G));
  } else {
    constexpr int BB = B * B;
    constexpr int KB = kWave / BB;
    constexpr int ACT = KB * BB;
    constexpr int MAXT = (128 + KB - 1) / KB;
    const int k0 = lane / BB, e = lane - k0 * BB, c = e % B;
    const bool on = lane < ACT;
    T acc = 0;
    if (nb <= 128) {
      const int c0 = lane < nb ? colind[rs + lane] : 0;
      const int c1 = lane + kWave < nb ? colind[rs + kWave + lane] : 0;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        const int jj = t * KB + k0;
        const int ca = __shfl(c0, jj & (kWave - 1));
        const int cb = __shfl(c1, jj & (kWave - 1));
        const int col = jj < kWave ? ca : cb;
        if (on && jj < nb) acc += vals[(rs + jj) * BB + e] * x[(int64_t)col * B + c];
      }
    } else if (on) {
      for (int jj = k0; jj < nb; jj += KB)
        acc += vals[(rs + jj) * BB + e] * x[(int64_t)colind[rs + jj] * B + c];
    }
    tot = row_reduce<B, T>(acc, lane);
  }
  if (lane < B) {
    const int64_t dof = row * B + lane;
    if (MODE == 1)
      y[dof] = mask[dof] ? T(0) : b[dof] - tot;
    else if (MODE == 2)
      y[dof] = mask[dof] ? T(0) : tot;
    else
      y[dof] = tot;
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
                                               int nl, int ppw, const int32_t *__restrict__ pnodes,
                                               const T *__restrict__ inv, const T *__restrict__ d,
                                               T *__restrict__ Y, int scatter, T *__restrict__ x,
                                               const T *__restrict__ scale,
                                               const uint8_t *__restrict__ mask, T omega, T *dl) {
  using V = typename Vec16<T>::type;
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
  __syncthreads();
  if (!act) return;
  const V *A = reinterpret_cast<const V *>(inv + p * (int64_t)np * npc) + r;
  const T *dv = dl + s * npc;
  T acc = 0;
  const int ng = npc / G;
#pragma unroll 6
  for (int g = 0; g < ng; ++g) {
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
__device__ __forceinline__ void vanka_gather_dof(int64_t dof, int b, const int32_t *__restrict__ gptr,
                                                 const int32_t *__restrict__ gidx,
                                                 const T *__restrict__ Y, const T *__restrict__ scale,
                                                 const uint8_t *__restrict__ mask, T omega, int assign,
                                                 T *__restrict__ x) {
  const int64_t node = dof / b;
  const int c = (int)(dof - node * b);
  T s = 0;
  const int e1 = gptr[node + 1];
  for (int e = gptr[node]; e < e1; ++e) s += Y[(int64_t)gidx[e] * b + c];
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
                                              const T *__restrict__ rf, T *__restrict__ rc,
                                              const uint8_t *__restrict__ maskc) {
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
        const T *src = rf + (base + ix[q]) * B;
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
                                             const T *__restrict__ xc, T *__restrict__ xf,
                                             const uint8_t *__restrict__ maskf) {
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
        const T *src = xc + (base + ix[q]) * B;
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
