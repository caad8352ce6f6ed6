// Element assembly of the condensed ALE fluid-structure system on tensor Q2
// meshes (Sec. 2 eq. aletime:2, Sec. 3.1 eq. defgrad, Sec. 4.2 eq.
// problem:1): the nonlinear residual of the theta time step and its
// approximate Jacobian (every derivative with respect to the ALE deformation
// dropped), plus the small vector kernels of the Newton loop (eq. newton).
//
// One workgroup per element.  Elements are launched by parity colour (the
// parity of the cell index per axis): two cells of one colour share no node,
// so each launch adds into the global arrays without conflicts and the sum
// order is fixed (colours in order, Gauss points in order).  The element's
// nodal fields, the basis values at the 3^d Gauss points, the fields at the
// Gauss points and the per-point material data are staged in LDS; for the
// Jacobian each thread owns one row node and (in 3D) two column nodes and
// keeps their (d+1) x (d+1) blocks in registers while it sums over the Gauss
// points (the row node's basis data are loaded once for both).
#include "fsimg_internal.h"

namespace fsimg {
namespace {

inline unsigned grid_for(int64_t n, int per_block) { return (unsigned)((n + per_block - 1) / per_block); }

// 3-point Gauss rule on [0, 1] and the quadratic Lagrange basis on the nodes
// 0, 1/2, 1 (Sec. 3.2: equal-order Q2 elements)
__device__ __forceinline__ double gauss_point(int q) {
  return q == 0 ? 0.1127016653792583115 : (q == 1 ? 0.5 : 0.8872983346207416885);
}
__device__ __forceinline__ double gauss_weight(int q) {
  return q == 1 ? 8.0 / 18.0 : 5.0 / 18.0;
}
__device__ __forceinline__ double lag(int l, double x) {
  return l == 0 ? 2.0 * (x - 0.5) * (x - 1.0) : (l == 1 ? 4.0 * x * (1.0 - x) : 2.0 * x * (x - 0.5));
}
__device__ __forceinline__ double dlag(int l, double x) {
  return l == 0 ? 4.0 * x - 3.0 : (l == 1 ? 4.0 - 8.0 * x : 4.0 * x - 1.0);
}

template <int D>
__device__ __forceinline__ double det_d(const double (&A)[D][D]) {
  if constexpr (D == 2) {
    return A[0][0] * A[1][1] - A[0][1] * A[1][0];
  } else {
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  }
}
// inverse by the adjugate
template <int D>
__device__ __forceinline__ void inv_d(const double (&A)[D][D], double det, double (&B)[D][D]) {
  const double r = 1.0 / det;
  if constexpr (D == 2) {
    B[0][0] = A[1][1] * r; B[0][1] = -A[0][1] * r;
    B[1][0] = -A[1][0] * r; B[1][1] = A[0][0] * r;
  } else {
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const int r0 = (b + 1) % 3, r1 = (b + 2) % 3, c0 = (a + 1) % 3, c1 = (a + 2) % 3;
        B[a][b] = (A[r0][c0] * A[r1][c1] - A[r0][c1] * A[r1][c0]) * r;
      }
  }
}

// cell coordinates of the blk-th element of a parity colour
template <int D>
__device__ __forceinline__ void colour_cell(const AsmLevel &L, int colour, int64_t blk, int (&e)[3]) {
  e[0] = e[1] = e[2] = 0;
  int64_t r = blk;
  for (int a = 0; a < D; ++a) {
    const int pa = (colour >> a) & 1;
    const int cnt = (L.cells[a] - pa + 1) / 2;
    e[a] = 2 * (int)(r % cnt) + pa;
    r /= cnt;
  }
}

template <int D>
__device__ __forceinline__ int64_t local_node(const AsmLevel &L, const int (&e)[3], int i) {
  int64_t g = 0, stride = 1;
  for (int a = 0; a < D; ++a) {
    const int la = (i / (a == 0 ? 1 : (a == 1 ? 3 : 9))) % 3;
    g += stride * (2 * e[a] + la);
    stride *= L.nnode[a];
  }
  return g;
}

// position of block (row, col) in the block-CSR pattern, -1 if absent
__device__ __forceinline__ int64_t find_block(const int32_t *rowptr, const int32_t *colind, int64_t row,
                                              int64_t col) {
  int64_t lo = rowptr[row], hi = rowptr[row + 1] - 1;
  while (lo <= hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int64_t c = colind[mid];
    if (c == col) return mid;
    if (c < col) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

// the node range of row node g's stencil along one axis (n nodes): a
// mid-cell node couples with its own cell only, a vertex with both neighbours
__device__ __forceinline__ void stencil_range(int g, int n, int &lo, int &hi) {
  if (g & 1) {
    lo = g - 1;
    hi = g + 1;
  } else {
    lo = g - 2 < 0 ? 0 : g - 2;
    hi = g + 2 > n - 1 ? n - 1 : g + 2;
  }
}

// position of block (row, col) in a full Q2 stencil pattern: the row's columns
// are its stencil box, lexicographic with x fastest
__device__ __forceinline__ int64_t stencil_block(const AsmLevel &L, int64_t row, int64_t col) {
  int64_t off = 0, span = 1, r = row, c = col;
  for (int a = 0; a < 3; ++a) {
    const int n = L.nnode[a];
    const int gr = (int)(r % n), gc = (int)(c % n);
    r /= n;
    c /= n;
    int lo, hi;
    stencil_range(gr, n, lo, hi);
    off += span * (gc - lo);
    span *= hi - lo + 1;
  }
  return L.rowptr[row] + off;
}

__device__ __forceinline__ int64_t block_position(const AsmLevel &L, int64_t row, int64_t col) {
  return L.structured ? stencil_block(L, row, col) : find_block(L.rowptr, L.colind, row, col);
}

template <int D>
struct ElemGeom {
  double h[D];
  double vol, hK;
  bool solid;
  bool iso;  // isoparametric cell (node positions): dx/dxi per Gauss point
};

template <int D>
__device__ __forceinline__ int64_t local_node(const AsmLevel &L, const int (&e)[3], int i);

// the cell's sizes: rectilinear h per axis (volume, h_K = the longest side);
// isoparametric cells: h_K = the longest edge from the first corner (local
// nodes 2, 6, 18), the volume per Gauss point from det(dx/dxi)
template <int D>
__device__ __forceinline__ ElemGeom<D> elem_geom(const AsmLevel &L, const int (&e)[3]) {
  ElemGeom<D> g;
  g.vol = 1.0;
  g.hK = 0.0;
  g.iso = L.xyz != nullptr;
  if (g.iso) {
    const int64_t g0 = local_node<D>(L, e, 0);
    for (int a = 0; a < D; ++a) {
      g.h[a] = 1.0;  // reference cell: the basis is staged in reference coordinates
      const int64_t gc = local_node<D>(L, e, 2 * (a == 0 ? 1 : (a == 1 ? 3 : 9)));
      double s = 0.0;
      for (int c = 0; c < D; ++c) {
        const double dx = L.xyz[gc * D + c] - L.xyz[g0 * D + c];
        s += dx * dx;
      }
      g.hK = fmax(g.hK, sqrt(s));
    }
  } else {
    for (int a = 0; a < D; ++a) {
      g.h[a] = L.coord[a][2 * e[a] + 2] - L.coord[a][2 * e[a]];
      g.vol *= g.h[a];
      g.hK = fmax(g.hK, g.h[a]);
    }
  }
  int64_t cell = 0, stride = 1;
  for (int a = 0; a < D; ++a) {
    cell += stride * e[a];
    stride *= L.cells[a];
  }
  g.solid = L.solid[cell] != 0;
  return g;
}

// N[q][i] and physical dN[m][q][i] at the Gauss points
template <int D, int NN>
__device__ __forceinline__ void basis_at(int q, int i, const double (&h)[D], double &N, double (&dN)[D]) {
  double L[D], dL[D];
  for (int a = 0; a < D; ++a) {
    const int p = a == 0 ? 1 : (a == 1 ? 3 : 9);
    const double x = gauss_point((q / p) % 3);
    const int l = (i / p) % 3;
    L[a] = lag(l, x);
    dL[a] = dlag(l, x);
  }
  N = 1.0;
  for (int a = 0; a < D; ++a) N *= L[a];
  for (int m = 0; m < D; ++m) {
    double v = 1.0;
    for (int a = 0; a < D; ++a) v *= (a == m) ? dL[a] : L[a];
    dN[m] = v / h[m];
  }
}

// Isoparametric cells: with the reference gradients s_dN[m][q][i] (h = 1)
// and the node positions s_x staged, compute per Gauss point q the Jacobian
// dx/dxi = sum_i x_i grad_xi N_i, its determinant (into s_det[q]) and its
// inverse, then turn s_dN into physical gradients in place:
// dN/dx_c = sum_k dN/dxi_k dxi_k/dx_c.  Called by the whole workgroup
// between barriers; flag[0] = 1 if det(dx/dxi) <= 0 (an inverted cell).
template <int D, int NN>
__device__ __forceinline__ void map_gradients(const double (&s_x)[NN][D], double (&s_dN)[D][NN][NN],
                                              double (&s_ji)[NN][D * D], double (&s_det)[NN],
                                              int *flag) {
  const int t = threadIdx.x;
  if (t < NN) {
    const int q = t;
    double Jg[D][D], Ji[D][D];
    for (int c = 0; c < D; ++c)
      for (int m = 0; m < D; ++m) Jg[c][m] = 0.0;
#pragma unroll 1
    for (int i = 0; i < NN; ++i)
      for (int c = 0; c < D; ++c) {
        const double xc = s_x[i][c];
        for (int m = 0; m < D; ++m) Jg[c][m] += xc * s_dN[m][q][i];
      }
    const double det = det_d<D>(Jg);
    if (!(det > 0.0)) flag[0] = 1;
    inv_d<D>(Jg, det, Ji);  // Ji[k][c] = dxi_k / dx_c
    for (int k = 0; k < D; ++k)
      for (int c = 0; c < D; ++c) s_ji[q][k * D + c] = Ji[k][c];
    s_det[q] = det;
  }
  __syncthreads();
#pragma unroll 1
  for (int it = t; it < NN * NN; it += blockDim.x) {
    const int q = it / NN, i = it % NN;
    double r[D];
    for (int k = 0; k < D; ++k) r[k] = s_dN[k][q][i];
    for (int c = 0; c < D; ++c) {
      double s = 0.0;
      for (int k = 0; k < D; ++k) s += r[k] * s_ji[q][k * D + c];
      s_dN[c][q][i] = s;
    }
  }
  __syncthreads();
}

template <int D>
__device__ __forceinline__ double qweight(int q) {
  double w = 1.0;
  for (int a = 0; a < D; ++a) w *= gauss_weight((q / (a == 0 ? 1 : (a == 1 ? 3 : 9))) % 3);
  return w;
}

// ---------------------------------------------------------------- Jacobian
// The approximate Jacobian of eq. problem:1 for one element, added into the
// block-CSR values with the identity rows and columns of `mask` left out.
//
//   fluid (deformation frozen): rho_f Jbar (dv, phi) - rho_f theta ((w.grad) dv, phi)
//     + k theta rho_f [(J (F^-1 v.grad) dv, phi) + (J (F^-1 dv.grad) v, phi)]
//     + k theta rho_f nu_f (J (grad dv F^-1 + F^-T grad dv^T) F^-T, grad phi)
//     - k (J dp F^-T, grad phi) + k (J tr(grad dv F^-1), xi) + s_h(dp, xi),
//     w = Jbar Fbar^-1 (u_n - u_{n-1});
//   solid (deformation condensed, dF = k theta grad dv):
//     rho_s (dv, phi) + k theta (dF Sigma + F dSigma, grad phi).
template <int D>
constexpr int jac_threads() { return D == 3 ? 384 : 128; }

template <int D>
__global__ __launch_bounds__(jac_threads<D>()) void k_asm_jac(AsmLevel L, AsmPhys P, AsmState S,
                                                            double *__restrict__ vals, int colour,
                                                            int *__restrict__ flag) {
  constexpr int NN = D == 3 ? 27 : 9, B = D + 1, NF = 3 * D * (D + 1), NQS = 32;
  constexpr int JT = D == 3 ? 2 : 1, NJ = (NN + JT - 1) / JT;  // column nodes per thread
  static_assert(NN * NJ <= jac_threads<D>(), "one thread per (row node, column group)");
  __shared__ double s_nod[4][NN][D];  // v, v_old, u (condensed in solid cells), u_old
  __shared__ double s_N[NN][NN];      // [q][i]
  __shared__ double s_dN[D][NN][NN];  // [m][q][i], physical
  __shared__ double s_qf[NN][NF];     // per point: (v, u, u_old) x comp x (value, d/dx_m)
  __shared__ double s_qs[NN][NQS];    // per point material data
  __shared__ double s_tf[D + 1][NN][NN];  // [c][q][i]: F^-T grad N_i (fluid) or F grad N_i
                                          // (solid); [D]: transport a.grad N_i (fluid)
  __shared__ double s_x[NN][D];           // node positions (isoparametric cells)
  __shared__ double s_ji[NN][D * D];      // per point: (dx/dxi)^-1
  __shared__ double s_det[NN];            // per point: det(dx/dxi)
  const int t = threadIdx.x;
  int e[3];
  colour_cell<D>(L, colour, blockIdx.x, e);
  const ElemGeom<D> G = elem_geom<D>(L, e);
  const double k = P.k, th = P.theta, kt = k * th;

  if (t < NN) {
    const int64_t g = local_node<D>(L, e, t);
    for (int c = 0; c < D; ++c) {
      const double v = S.x[g * B + 1 + c], vo = S.xo[g * B + 1 + c], uo = S.uo[g * D + c];
      s_nod[0][t][c] = v;
      s_nod[1][t][c] = vo;
      s_nod[2][t][c] = G.solid ? uo + kt * v + k * (1.0 - th) * vo : S.u[g * D + c];
      s_nod[3][t][c] = uo;
      if (G.iso) s_x[t][c] = L.xyz[g * D + c];
    }
  }
  for (int it = t; it < NN * NN; it += blockDim.x) {
    const int q = it / NN, i = it % NN;
    double N, dN[D];
    basis_at<D, NN>(q, i, G.h, N, dN);
    s_N[q][i] = N;
    for (int m = 0; m < D; ++m) s_dN[m][q][i] = dN[m];
  }
  __syncthreads();
  if (G.iso) map_gradients<D, NN>(s_x, s_dN, s_ji, s_det, flag);
  // fields at the Gauss points: item (q, f), f = field * D(D+1) + c (D+1) + w
  for (int it = t; it < NN * NF; it += blockDim.x) {
    const int q = it / NF, f = it % NF;
    const int fld = f / (D * (D + 1)), rem = f % (D * (D + 1));
    const int c = rem / (D + 1), w = rem % (D + 1);
    const int src = fld == 0 ? 0 : (fld == 1 ? 2 : 3);
    double s = 0.0;
    for (int i = 0; i < NN; ++i) s += (w == 0 ? s_N[q][i] : s_dN[w - 1][q][i]) * s_nod[src][i][c];
    s_qf[q][f] = s;
  }
  __syncthreads();
  if (t < NN) {
    const int q = t;
    const double *qf = s_qf[q];
    constexpr int FB = D * (D + 1);
    auto val = [&](int fld, int c) { return qf[fld * FB + c * (D + 1)]; };
    auto grd = [&](int fld, int c, int m) { return qf[fld * FB + c * (D + 1) + 1 + m]; };
    double F[D][D], Fi[D][D];
    for (int a = 0; a < D; ++a)
      for (int m = 0; m < D; ++m) F[a][m] = (a == m ? 1.0 : 0.0) + grd(1, a, m);
    const double J = det_d<D>(F);
    if (!(J > 0.0)) flag[0] = 1;
    inv_d<D>(F, J, Fi);
    double *qs = s_qs[q];
    qs[0] = qweight<D>(q) * (G.iso ? s_det[q] : G.vol);
    if (!G.solid) {
      double Fo[D][D], Fb[D][D], Fbi[D][D];
      for (int a = 0; a < D; ++a)
        for (int m = 0; m < D; ++m) {
          Fo[a][m] = (a == m ? 1.0 : 0.0) + grd(2, a, m);
          Fb[a][m] = 0.5 * (F[a][m] + Fo[a][m]);
        }
      const double Jo = det_d<D>(Fo), Jb = 0.5 * (J + Jo);
      inv_d<D>(Fb, det_d<D>(Fb), Fbi);
      qs[1] = P.rho_f * Jb;                  // inertia
      qs[2] = kt * P.rho_f * P.nu_f * J;     // viscosity
      qs[3] = k * J;                         // pressure / divergence coupling
      for (int a = 0; a < D; ++a) {
        double wv = 0.0, tv = 0.0;
        for (int m = 0; m < D; ++m) {
          wv += Fbi[a][m] * (val(1, m) - val(2, m));
          tv += Fi[a][m] * val(0, m);
        }
        qs[4 + a] = kt * P.rho_f * J * tv - P.rho_f * th * Jb * wv;   // transport velocity
      }
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
          double s = 0.0;
          for (int m = 0; m < D; ++m) s += grd(0, a, m) * Fi[m][b];
          qs[4 + D + a * D + b] = kt * P.rho_f * J * s;               // (F^-1 dv.grad) v
        }
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) qs[4 + D + D * D + a * D + b] = Fi[a][b];
    } else {
      double E[D][D], trE = 0.0;
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
          double s = 0.0;
          for (int m = 0; m < D; ++m) s += F[m][a] * F[m][b];
          E[a][b] = 0.5 * (s - (a == b ? 1.0 : 0.0));
        }
      for (int a = 0; a < D; ++a) trE += E[a][a];
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
          double fft = 0.0;
          for (int m = 0; m < D; ++m) fft += F[a][m] * F[b][m];
          qs[1 + a * D + b] = 2.0 * P.mu_s * E[a][b] + (a == b ? P.lambda_s * trE : 0.0);  // Sigma
          qs[1 + D * D + a * D + b] = fft;                                                   // F F^T
          qs[1 + 2 * D * D + a * D + b] = F[a][b];
        }
    }
  }
  __syncthreads();
  for (int it = t; it < NN * NN; it += blockDim.x) {
    const int q = it / NN, i = it % NN;
    const double *qs = s_qs[q];
    double dN[D];
    for (int m = 0; m < D; ++m) dN[m] = s_dN[m][q][i];
    if (!G.solid) {
      double adn = 0.0;
      for (int c = 0; c < D; ++c) {
        double s = 0.0;
        for (int m = 0; m < D; ++m) s += qs[4 + D + D * D + m * D + c] * dN[m];   // (F^-T grad N)_c
        s_tf[c][q][i] = s;
        adn += qs[4 + c] * dN[c];
      }
      s_tf[D][q][i] = adn;
    } else {
      for (int a = 0; a < D; ++a) {
        double s = 0.0;
        for (int m = 0; m < D; ++m) s += qs[1 + 2 * D * D + a * D + m] * dN[m];   // (F grad N)_a
        s_tf[a][q][i] = s;
      }
    }
  }
  __syncthreads();
  // each thread: row node i and JT column nodes j = jb + jj * NJ (the i-side
  // loads are shared by the JT blocks)
  if (t >= NN * NJ) return;
  const int i = t / NJ, jb = t % NJ;
  int js[JT];
  bool jok[JT];
  for (int jj = 0; jj < JT; ++jj) {
    const int j = jb + jj * NJ;
    jok[jj] = j < NN;
    js[jj] = jok[jj] ? j : NN - 1;
  }
  double K[JT][B][B];
  for (int jj = 0; jj < JT; ++jj)
    for (int a = 0; a < B; ++a)
      for (int c = 0; c < B; ++c) K[jj][a][c] = 0.0;
  const double dK = P.alpha0 * k * k * G.hK * G.hK / (P.rho_f * (G.hK * G.hK + kt * P.nu_f));
  const double kt2 = kt * kt;
  for (int q = 0; q < NN; ++q) {
    const double *qs = s_qs[q];
    const double wq = qs[0];
    const double Ni = s_N[q][i];
    double dNi[D];
    for (int m = 0; m < D; ++m) dNi[m] = s_dN[m][q][i];
    if (!G.solid) {
      double gi[D];
      for (int c = 0; c < D; ++c) gi[c] = s_tf[c][q][i];
      const double visc = qs[2], kJ = qs[3], cm = qs[1];
      double R[D][D];
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) R[a][b] = qs[4 + D + a * D + b];
      for (int jj = 0; jj < JT; ++jj) {
        const int j = js[jj];
        const double Nj = s_N[q][j], NNij = Ni * Nj;
        double dd = 0.0, gg = 0.0, gj[D];
        for (int m = 0; m < D; ++m) dd += dNi[m] * s_dN[m][q][j];
        for (int c = 0; c < D; ++c) {
          gj[c] = s_tf[c][q][j];
          gg += gi[c] * gj[c];
        }
        const double diag = cm * NNij + Ni * s_tf[D][q][j] + visc * gg;
        K[jj][0][0] += wq * dK * dd;
        for (int b = 0; b < D; ++b) K[jj][0][1 + b] += wq * kJ * Ni * gj[b];
        for (int a = 0; a < D; ++a) {
          K[jj][1 + a][0] -= wq * kJ * Nj * gi[a];
          for (int b = 0; b < D; ++b)
            K[jj][1 + a][1 + b] += wq * (NNij * R[a][b] + visc * gj[a] * gi[b] + (a == b ? diag : 0.0));
        }
      }
    } else {
      double fi[D], Sd[D];
      for (int a = 0; a < D; ++a) fi[a] = s_tf[a][q][i];
      for (int m = 0; m < D; ++m) {
        double s = 0.0;
        for (int n2 = 0; n2 < D; ++n2) s += qs[1 + m * D + n2] * dNi[n2];
        Sd[m] = s;  // (Sigma grad N_i)_m
      }
      for (int jj = 0; jj < JT; ++jj) {
        const int j = js[jj];
        const double NNij = Ni * s_N[q][j];
        double fj[D], dd = 0.0, cS = 0.0;
        for (int m = 0; m < D; ++m) {
          const double dnj = s_dN[m][q][j];
          dd += dNi[m] * dnj;
          cS += dnj * Sd[m];
          fj[m] = s_tf[m][q][j];
        }
        for (int a = 0; a < D; ++a)
          for (int b = 0; b < D; ++b)
            K[jj][1 + a][1 + b] += wq * (kt2 * (P.mu_s * (fj[a] * fi[b] + qs[1 + D * D + a * D + b] * dd) +
                                                P.lambda_s * fj[b] * fi[a]) +
                                         (a == b ? P.rho_s * NNij + kt2 * cS : 0.0));
      }
    }
  }
  const int64_t gr = local_node<D>(L, e, i);
  for (int jj = 0; jj < JT; ++jj) {
    if (!jok[jj]) continue;
    const int64_t gc = local_node<D>(L, e, js[jj]);
    const int64_t pos = block_position(L, gr, gc);
    if (pos < 0) {
      flag[1] = 1;
      continue;
    }
    double *blk = vals + pos * (B * B);
    for (int a = 0; a < B; ++a) {
      if (L.mask[gr * B + a]) continue;
      for (int c = 0; c < B; ++c)
        if (!L.mask[gc * B + c]) blk[a * B + c] += K[jj][a][c];
    }
  }
}

// identity rows: diagonal entry one (rows and columns were left out above)
__global__ __launch_bounds__(256) void k_asm_identity(const int32_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ colind,
                                                      const uint8_t *__restrict__ mask, int64_t nrows,
                                                      int b, double *__restrict__ vals,
                                                      int *__restrict__ flag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  bool any = false;
  for (int a = 0; a < b; ++a) any |= mask[r * b + a] != 0;
  if (!any) return;
  const int64_t pos = find_block(rowptr, colind, r, r);
  if (pos < 0) {
    flag[1] = 1;
    return;
  }
  for (int a = 0; a < b; ++a)
    if (mask[r * b + a]) vals[pos * b * b + a * b + a] = 1.0;
}

// ---------------------------------------------------------------- residual
// A(U) of eq. aletime:2 moved to the left-hand side (solid deformation
// condensed, fluid deformation u), tested with every local basis function;
// res -= A(U) at the rows that are not identity rows.
template <int D>
__global__ __launch_bounds__(D == 3 ? 256 : 128) void k_asm_res(AsmLevel L, AsmPhys P, AsmState S,
                                                              double *__restrict__ res, int colour,
                                                              int *__restrict__ flag) {
  constexpr int NN = D == 3 ? 27 : 9, B = D + 1, FB = D * (D + 1), NF = 4 * FB + D + 1;
  constexpr int NO = 1 + D + D * D + D;  // per point: w vec, w ten, w div, w dK grad p
  __shared__ double s_nod[4][NN][D];     // v, v_old, u (condensed in solid cells), u_old
  __shared__ double s_p[NN];
  __shared__ double s_N[NN][NN];
  __shared__ double s_dN[D][NN][NN];
  __shared__ double s_qf[NN][NF];        // (v, v_old, u, u_old) x comp x (value, grad); p, grad p
  __shared__ double s_qo[NN][NO];
  __shared__ double s_x[NN][D];          // node positions (isoparametric cells)
  __shared__ double s_ji[NN][D * D];     // per point: (dx/dxi)^-1
  __shared__ double s_det[NN];           // per point: det(dx/dxi)
  const int t = threadIdx.x;
  int e[3];
  colour_cell<D>(L, colour, blockIdx.x, e);
  const ElemGeom<D> G = elem_geom<D>(L, e);
  const double k = P.k, th = P.theta, kt = k * th;
  if (t < NN) {
    const int64_t g = local_node<D>(L, e, t);
    for (int c = 0; c < D; ++c) {
      const double v = S.x[g * B + 1 + c], vo = S.xo[g * B + 1 + c], uo = S.uo[g * D + c];
      s_nod[0][t][c] = v;
      s_nod[1][t][c] = vo;
      s_nod[2][t][c] = G.solid ? uo + kt * v + k * (1.0 - th) * vo : S.u[g * D + c];
      s_nod[3][t][c] = uo;
      if (G.iso) s_x[t][c] = L.xyz[g * D + c];
    }
    s_p[t] = S.x[g * B];
  }
  for (int it = t; it < NN * NN; it += blockDim.x) {
    const int q = it / NN, i = it % NN;
    double N, dN[D];
    basis_at<D, NN>(q, i, G.h, N, dN);
    s_N[q][i] = N;
    for (int m = 0; m < D; ++m) s_dN[m][q][i] = dN[m];
  }
  __syncthreads();
  if (G.iso) map_gradients<D, NN>(s_x, s_dN, s_ji, s_det, flag);
  for (int it = t; it < NN * NF; it += blockDim.x) {
    const int q = it / NF, f = it % NF;
    double s = 0.0;
    if (f < 4 * FB) {
      const int fld = f / FB, rem = f % FB, c = rem / (D + 1), w = rem % (D + 1);
      for (int i = 0; i < NN; ++i) s += (w == 0 ? s_N[q][i] : s_dN[w - 1][q][i]) * s_nod[fld][i][c];
    } else {
      const int w = f - 4 * FB;
      for (int i = 0; i < NN; ++i) s += (w == 0 ? s_N[q][i] : s_dN[w - 1][q][i]) * s_p[i];
    }
    s_qf[q][f] = s;
  }
  __syncthreads();
  if (t < NN) {
    const int q = t;
    const double *qf = s_qf[q];
    auto val = [&](int fld, int c) { return qf[fld * FB + c * (D + 1)]; };
    auto grd = [&](int fld, int c, int m) { return qf[fld * FB + c * (D + 1) + 1 + m]; };
    const double pq = qf[4 * FB];
    double F[D][D], Fo[D][D], Fi[D][D], Foi[D][D];
    for (int a = 0; a < D; ++a)
      for (int m = 0; m < D; ++m) {
        F[a][m] = (a == m ? 1.0 : 0.0) + grd(2, a, m);
        Fo[a][m] = (a == m ? 1.0 : 0.0) + grd(3, a, m);
      }
    const double J = det_d<D>(F), Jo = det_d<D>(Fo);
    if (!(J > 0.0)) flag[0] = 1;
    double vec[D], ten[D][D], div = 0.0;
    if (!G.solid) {
      inv_d<D>(F, J, Fi);
      inv_d<D>(Fo, Jo, Foi);
      double Fb[D][D], Fbi[D][D];
      for (int a = 0; a < D; ++a)
        for (int m = 0; m < D; ++m) Fb[a][m] = 0.5 * (F[a][m] + Fo[a][m]);
      inv_d<D>(Fb, det_d<D>(Fb), Fbi);
      const double Jb = 0.5 * (J + Jo);
      double w[D], tv[D], to[D];
      for (int a = 0; a < D; ++a) {
        double s = 0.0, s1 = 0.0, s2 = 0.0;
        for (int m = 0; m < D; ++m) {
          s += Fbi[a][m] * (val(2, m) - val(3, m));
          s1 += Fi[a][m] * val(0, m);
          s2 += Foi[a][m] * val(1, m);
        }
        w[a] = Jb * s;
        tv[a] = s1;
        to[a] = s2;
      }
      for (int a = 0; a < D; ++a) {
        double tr = 0.0, cv = 0.0, co = 0.0;
        for (int m = 0; m < D; ++m) {
          tr += (th * grd(0, a, m) + (1.0 - th) * grd(1, a, m)) * w[m];
          cv += grd(0, a, m) * tv[m];
          co += grd(1, a, m) * to[m];
        }
        vec[a] = P.rho_f * Jb * (val(0, a) - val(1, a)) - P.rho_f * tr + kt * P.rho_f * J * cv +
                 k * (1.0 - th) * P.rho_f * Jo * co;
      }
      // viscous stress rho nu J (G + G^T) F^-T, G = grad v F^-1, now and at t_{n-1}
      double Gn[D][D], Go[D][D];
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
          double s = 0.0, so = 0.0;
          for (int m = 0; m < D; ++m) {
            s += grd(0, a, m) * Fi[m][b];
            so += grd(1, a, m) * Foi[m][b];
          }
          Gn[a][b] = s;
          Go[a][b] = so;
        }
      for (int a = 0; a < D; ++a) div += Gn[a][a];
      div *= k * J;
      const double cn = kt * P.rho_f * P.nu_f * J, co = k * (1.0 - th) * P.rho_f * P.nu_f * Jo;
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
          double s = 0.0, so = 0.0;
          for (int m = 0; m < D; ++m) {
            s += (Gn[a][m] + Gn[m][a]) * Fi[b][m];
            so += (Go[a][m] + Go[m][a]) * Foi[b][m];
          }
          ten[a][b] = cn * s + co * so - k * J * pq * Fi[b][a];
        }
    } else {
      // first Piola stress F Sigma(E), E = (F^T F - I) / 2, now and at t_{n-1}
      for (int a = 0; a < D; ++a) {
        vec[a] = P.rho_s * (val(0, a) - val(1, a));
        for (int b = 0; b < D; ++b) ten[a][b] = 0.0;
      }
      for (int pass = 0; pass < 2; ++pass) {
        const double(&Fx)[D][D] = pass == 0 ? F : Fo;
        const double wt = pass == 0 ? kt : k * (1.0 - th);
        double E[D][D], Sg[D][D], trE = 0.0;
        for (int a = 0; a < D; ++a)
          for (int b = 0; b < D; ++b) {
            double s = 0.0;
            for (int m = 0; m < D; ++m) s += Fx[m][a] * Fx[m][b];
            E[a][b] = 0.5 * (s - (a == b ? 1.0 : 0.0));
          }
        for (int a = 0; a < D; ++a) trE += E[a][a];
        for (int a = 0; a < D; ++a)
          for (int b = 0; b < D; ++b) Sg[a][b] = 2.0 * P.mu_s * E[a][b] + (a == b ? P.lambda_s * trE : 0.0);
        for (int a = 0; a < D; ++a)
          for (int b = 0; b < D; ++b) {
            double s = 0.0;
            for (int m = 0; m < D; ++m) s += Fx[a][m] * Sg[m][b];
            ten[a][b] += wt * s;
          }
      }
    }
    const double wq = qweight<D>(q) * (G.iso ? s_det[q] : G.vol);
    double *qo = s_qo[q];
    for (int a = 0; a < D; ++a) qo[a] = wq * vec[a];
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) qo[D + a * D + b] = wq * ten[a][b];
    qo[D + D * D] = wq * div;
    const double dK = G.solid ? 0.0
                              : P.alpha0 * k * k * G.hK * G.hK / (P.rho_f * (G.hK * G.hK + kt * P.nu_f));
    for (int m = 0; m < D; ++m) qo[D + D * D + 1 + m] = wq * dK * qf[4 * FB + 1 + m];
  }
  __syncthreads();
  if (t >= NN * B) return;
  const int i = t / B, comp = t % B;
  double s = 0.0;
  for (int q = 0; q < NN; ++q) {
    const double *qo = s_qo[q];
    if (comp == 0) {
      s += qo[D + D * D] * s_N[q][i];
      for (int m = 0; m < D; ++m) s += qo[D + D * D + 1 + m] * s_dN[m][q][i];
    } else {
      const int a = comp - 1;
      s += qo[a] * s_N[q][i];
      for (int b = 0; b < D; ++b) s += qo[D + a * D + b] * s_dN[b][q][i];
    }
  }
  const int64_t g = local_node<D>(L, e, i);
  if (!L.mask[g * B + comp]) res[g * B + comp] -= s;
}

// ---------------------------------------------------------------- helpers
__global__ __launch_bounds__(256) void k_asm_fill(double *__restrict__ x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// coarse nodal field from the fine one at the coincident nodes (node 2g)
__global__ __launch_bounds__(256) void k_inject(const double *__restrict__ f, double *__restrict__ c,
                                                int nfx, int nfy, int ncx, int ncy, int64_t nc, int comps) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nc) return;
  const int64_t gx = r % ncx, gy = (r / ncx) % ncy, gz = r / ((int64_t)ncx * ncy);
  const int64_t src = 2 * gx + (int64_t)nfx * (2 * gy + (int64_t)nfy * 2 * gz);
  for (int q = 0; q < comps; ++q) c[r * comps + q] = f[src * comps + q];
}

// y = x + omega z
__global__ __launch_bounds__(256) void k_axpy_to(const double *__restrict__ x, const double *__restrict__ z,
                                                 double omega, double *__restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] + omega * z[i];
}

// y = -y at rows that are not identity rows, 0 at identity rows
__global__ __launch_bounds__(256) void k_neg_free(double *__restrict__ y, const uint8_t *__restrict__ mask,
                                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = mask[i] ? 0.0 : -y[i];
}

// *bad = 1 unless every row's columns are exactly its Q2 stencil box
__global__ __launch_bounds__(256) void k_check_structured(AsmLevel L, int64_t nrows, int *__restrict__ bad) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int lo[3], hi[3], g[3];
  int64_t q = r;
  for (int a = 0; a < 3; ++a) {
    g[a] = (int)(q % L.nnode[a]);
    q /= L.nnode[a];
    stencil_range(g[a], L.nnode[a], lo[a], hi[a]);
  }
  const int64_t cnt = (int64_t)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
  const int64_t p0 = L.rowptr[r];
  if (L.rowptr[r + 1] - p0 != cnt) {
    bad[0] = 1;
    return;
  }
  int64_t p = p0;
  for (int z = lo[2]; z <= hi[2]; ++z)
    for (int y = lo[1]; y <= hi[1]; ++y)
      for (int x = lo[0]; x <= hi[0]; ++x, ++p) {
        const int64_t col = x + (int64_t)L.nnode[0] * (y + (int64_t)L.nnode[1] * z);
        if (L.colind[p] != col) {
          bad[0] = 1;
          return;
        }
      }
}

// residual of the condensation relation (deformation rows, mass matrix
// cancelled): r = u_old + k theta v + k (1 - theta) v_old - u at the nodes of
// solid cells, 0 elsewhere; v, v_old from the (p, v) vectors x, x_old
__global__ __launch_bounds__(256) void k_cond_residual(int64_t nnodes, int dim, const uint8_t *__restrict__ mask,
                                                       double kt, double k1, const double *__restrict__ x,
                                                       const double *__restrict__ xo,
                                                       const double *__restrict__ u,
                                                       const double *__restrict__ uo, double *__restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnodes) return;
  const bool on = mask[i] != 0;
  for (int c = 0; c < dim; ++c) {
    const int64_t q = i * dim + c, pv = i * (dim + 1) + 1 + c;
    r[q] = on ? uo[q] + kt * x[pv] + k1 * xo[pv] - u[q] : 0.0;
  }
}

// *out = max(*out, max_i |x_i|); the bit patterns of non-negative doubles
// order like the values, so an unsigned 64-bit atomic max is exact
__global__ __launch_bounds__(256) void k_absmax(const double *__restrict__ x, int64_t n,
                                                unsigned long long *__restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(x[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

inline int64_t colour_count(const AsmLevel &L, int dim, int colour) {
  int64_t n = 1;
  for (int a = 0; a < dim; ++a) n *= (L.cells[a] - ((colour >> a) & 1) + 1) / 2;
  return n;
}

}  // namespace

void launch_asm_jacobian(const AsmLevel &L, int dim, const AsmPhys &P, const AsmState &S, double *vals,
                         int64_t nrows, int64_t nnzb, int *flag, hipStream_t s, hipEvent_t *ev) {
  const int b = dim + 1;
  const int64_t nv = nnzb * b * b;
  hipLaunchKernelGGL(k_asm_fill, dim3(grid_for(nv, 256)), dim3(256), 0, s, vals, nv, 0.0);
  for (int c = 0; c < (1 << dim); ++c) {
    const int64_t ne = colour_count(L, dim, c);
    if (ev) (void)hipEventRecord(ev[2 * c], s);
    if (ne > 0) {
      if (dim == 3)
        hipLaunchKernelGGL(k_asm_jac<3>, dim3(ne), dim3(jac_threads<3>()), 0, s, L, P, S, vals, c, flag);
      else
        hipLaunchKernelGGL(k_asm_jac<2>, dim3(ne), dim3(jac_threads<2>()), 0, s, L, P, S, vals, c, flag);
    }
    if (ev) (void)hipEventRecord(ev[2 * c + 1], s);
  }
  hipLaunchKernelGGL(k_asm_identity, dim3(grid_for(nrows, 256)), dim3(256), 0, s, L.rowptr, L.colind,
                     L.mask, nrows, b, vals, flag);
}

void launch_asm_residual(const AsmLevel &L, int dim, const AsmPhys &P, const AsmState &S, double *res,
                         int64_t nrows, int *flag, hipStream_t s, hipEvent_t *ev) {
  const int64_t n = nrows * (dim + 1);
  hipLaunchKernelGGL(k_asm_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, res, n, 0.0);
  for (int c = 0; c < (1 << dim); ++c) {
    const int64_t ne = colour_count(L, dim, c);
    if (ev) (void)hipEventRecord(ev[2 * c], s);
    if (ne > 0) {
      if (dim == 3)
        hipLaunchKernelGGL(k_asm_res<3>, dim3(ne), dim3(256), 0, s, L, P, S, res, c, flag);
      else
        hipLaunchKernelGGL(k_asm_res<2>, dim3(ne), dim3(128), 0, s, L, P, S, res, c, flag);
    }
    if (ev) (void)hipEventRecord(ev[2 * c + 1], s);
  }
}

void launch_inject(const double *f, double *c, const int *nnode_f, const int *nnode_c, int comps,
                   hipStream_t s) {
  const int64_t nc = (int64_t)nnode_c[0] * nnode_c[1] * nnode_c[2];
  hipLaunchKernelGGL(k_inject, dim3(grid_for(nc, 256)), dim3(256), 0, s, f, c, nnode_f[0], nnode_f[1],
                     nnode_c[0], nnode_c[1], nc, comps);
}

void launch_axpy_to(const double *x, const double *z, double omega, double *y, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_axpy_to, dim3(grid_for(n, 256)), dim3(256), 0, s, x, z, omega, y, n);
}

void launch_neg_free(double *y, const uint8_t *mask, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_neg_free, dim3(grid_for(n, 256)), dim3(256), 0, s, y, mask, n);
}

void launch_cond_residual(int64_t nnodes, int dim, const uint8_t *mask, double k, double theta,
                          const double *x, const double *xo, const double *u, const double *uo, double *r,
                          hipStream_t s) {
  if (nnodes > 0)
    hipLaunchKernelGGL(k_cond_residual, dim3(grid_for(nnodes, 256)), dim3(256), 0, s, nnodes, dim, mask,
                       k * theta, k * (1.0 - theta), x, xo, u, uo, r);
}

void launch_check_structured(const AsmLevel &L, int dim, int64_t nrows, int *bad, hipStream_t s) {
  (void)dim;
  if (nrows > 0)
    hipLaunchKernelGGL(k_check_structured, dim3(grid_for(nrows, 256)), dim3(256), 0, s, L, nrows, bad);
}

void launch_absmax_u64(const double *x, int64_t n, unsigned long long *out, hipStream_t s) {
  if (n <= 0) return;
  const int64_t g = std::min<int64_t>(grid_for(n, 256), 2048);
  hipLaunchKernelGGL(k_absmax, dim3(g), dim3(256), 0, s, x, n, out);
}

}  // namespace fsimg
