/*
 * Input-fixture assembly for the synthetic FSI Newton-step systems.
 *
 * This file builds the matrices that the solver (GPU library) and the oracle
 * both receive as INPUT: it is neither of the two.  It evaluates the
 * linearised, condensed monolithic ALE fluid-structure system of the paper
 * (Sec. 3.1, eq. aletime:2 with the condensation eq. defgrad; Sec. 4.2,
 * eq. problem:1 with the ALE derivatives dropped; eq. problem:3 for the
 * harmonic mesh extension) with equal-order Q2 elements (Sec. 3.2) on a
 * graded tensor-product mesh of [0,1]^d, or on isoparametric Q2 cells when
 * node positions are given (the curved cylinder of Sec. 5: per Gauss point
 * the Jacobian dx/dxi of x(xi) = sum_i x_i N_i(xi), physical gradients by its
 * inverse transpose, weights by its determinant; h_K = the longest cell edge
 * from the first corner).
 *
 * Per element and Gauss point (3 points per axis):
 *   fluid cells  (u frozen: no derivatives w.r.t. the ALE deformation)
 *     rho_f Jbar (dv,phi) - rho_f theta ((Jbar Fbar^-1 (u-u_old)).grad dv, phi)
 *     + k theta rho_f [ (J (F^-1 v.grad) dv, phi) + (J (F^-1 dv.grad) v, phi) ]
 *     + k theta rho_f nu_f (J (grad dv F^-1 + F^-T grad dv^T) F^-T, grad phi)
 *     - k (J dp F^-T, grad phi) + k (J tr(grad dv F^-1), xi) + s_h(dp, xi)
 *   solid cells  (deformation condensed into the velocity, eq. defgrad)
 *     rho_s (dv,phi) + k theta (dF Sigma + F dSigma, grad phi),  dF = k theta grad dv
 *   s_h(p,xi) = sum_K delta_K (grad p, grad xi)_K,
 *     delta_K = alpha0 k^2 h_K^2 / (rho_f (h_K^2 + k theta nu_f))
 *   ALE  : (grad du, grad psi) on fluid cells (vector Laplacian)
 *   mass : (du, psi) on solid cells (the deformation update system, eq. problem:2)
 *   smass: scalar Q2 mass on all cells (used to smooth random right-hand sides)
 *
 * Node numbering: lexicographic, x fastest, 2*cells[a]+1 nodes per axis.
 * Momentum block order per node: (p, v_1, .., v_d).
 * All matrices are written into a caller-provided block-CSR pattern
 * (row-major b x b blocks); entries are accumulated (+=).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXD 3
#define MAXN 27 /* nodes per element */
#define MAXQ 27 /* quadrature points per element */

typedef struct {
  double rho_f, nu_f, rho_s, mu_s, lambda_s, k, theta, alpha0;
} phys_params;

/* 1D quadratic Lagrange basis on [0,1] with nodes 0, 1/2, 1 */
static double L1d(int l, double x) {
  if (l == 0) return 2.0 * (x - 0.5) * (x - 1.0);
  if (l == 1) return 4.0 * x * (1.0 - x);
  return 2.0 * x * (x - 0.5);
}
static double dL1d(int l, double x) {
  if (l == 0) return 4.0 * x - 3.0;
  if (l == 1) return 4.0 - 8.0 * x;
  return 4.0 * x - 1.0;
}

typedef struct {
  int dim, nn, nq;
  double N[MAXQ][MAXN];        /* basis values */
  double dN[MAXQ][MAXN][MAXD]; /* reference derivatives */
  double w[MAXQ];              /* reference weights (sum 1) */
} ref_tables;

static void make_tables(int dim, ref_tables *t) {
  const double g[3] = {0.5 - sqrt(0.15), 0.5, 0.5 + sqrt(0.15)};
  const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  t->dim = dim;
  t->nn = dim == 2 ? 9 : 27;
  t->nq = t->nn;
  for (int q = 0; q < t->nq; ++q) {
    int qa[3] = {q % 3, (q / 3) % 3, q / 9};
    double w = 1.0;
    for (int a = 0; a < dim; ++a) w *= gw[qa[a]];
    t->w[q] = w;
    for (int i = 0; i < t->nn; ++i) {
      int la[3] = {i % 3, (i / 3) % 3, i / 9};
      double v = 1.0;
      for (int a = 0; a < dim; ++a) v *= L1d(la[a], g[qa[a]]);
      t->N[q][i] = v;
      for (int m = 0; m < dim; ++m) {
        double d = 1.0;
        for (int a = 0; a < dim; ++a)
          d *= (a == m) ? dL1d(la[a], g[qa[a]]) : L1d(la[a], g[qa[a]]);
        t->dN[q][i][m] = d;
      }
    }
  }
}

static double det_d(int d, const double A[MAXD][MAXD]) {
  if (d == 2) return A[0][0] * A[1][1] - A[0][1] * A[1][0];
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
         A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}
static void inv_d(int d, const double A[MAXD][MAXD], double B[MAXD][MAXD]) {
  double det = det_d(d, A);
  if (d == 2) {
    B[0][0] = A[1][1] / det; B[0][1] = -A[0][1] / det;
    B[1][0] = -A[1][0] / det; B[1][1] = A[0][0] / det;
    return;
  }
  B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
  B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
  B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
  B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
  B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
  B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
  B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
  B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
  B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
}

typedef struct {
  int dim;
  int cells[3];
  int nnode[3];
  const double *coords[3];
  const double *xyz; /* NULL: node coordinates from the per-axis grid; else
                        [nnodes][dim] (isoparametric Q2 cells) */
} mesh_t;

/* Geometry of element (nodes) at reference point q: weight w_q det(dx/dxi)
   and the physical basis gradients dNp = (dx/dxi)^-T dN.  Rectilinear cells
   (xyz NULL): dx/dxi = diag(h). */
static int point_geometry(const mesh_t *m, const ref_tables *T, const int64_t *nodes,
                          const double *h, int q, double *wq, double dNp[MAXN][MAXD]) {
  const int d = m->dim, nn = T->nn;
  if (!m->xyz) {
    double vol = 1.0;
    for (int a = 0; a < d; ++a) vol *= h[a];
    *wq = T->w[q] * vol;
    for (int i = 0; i < nn; ++i)
      for (int k = 0; k < d; ++k) dNp[i][k] = T->dN[q][i][k] / h[k];
    return 0;
  }
  double Jg[MAXD][MAXD], Ji[MAXD][MAXD];
  for (int c = 0; c < d; ++c)
    for (int k = 0; k < d; ++k) {
      double s = 0.0;
      for (int i = 0; i < nn; ++i) s += m->xyz[nodes[i] * d + c] * T->dN[q][i][k];
      Jg[c][k] = s; /* d x_c / d xi_k */
    }
  const double det = det_d(d, Jg);
  inv_d(d, Jg, Ji); /* Ji[k][c] = d xi_k / d x_c */
  *wq = T->w[q] * det;
  for (int i = 0; i < nn; ++i)
    for (int c = 0; c < d; ++c) {
      double s = 0.0;
      for (int k = 0; k < d; ++k) s += T->dN[q][i][k] * Ji[k][c];
      dNp[i][c] = s;
    }
  return det > 0.0 ? 0 : -1;
}

/* h_K: the longest of the d cell edges from the first corner (rectilinear:
   the longest side) */
static double cell_size(const mesh_t *m, const int64_t *nodes, const double *h) {
  const int d = m->dim;
  double hK = 0.0;
  if (!m->xyz) {
    for (int a = 0; a < d; ++a) if (h[a] > hK) hK = h[a];
    return hK;
  }
  for (int a = 0; a < d; ++a) {
    const int corner = 2 * (a == 0 ? 1 : (a == 1 ? 3 : 9));
    double s = 0.0;
    for (int c = 0; c < d; ++c) {
      const double e = m->xyz[nodes[corner] * d + c] - m->xyz[nodes[0] * d + c];
      s += e * e;
    }
    s = sqrt(s);
    if (s > hK) hK = s;
  }
  return hK;
}

/* element e (lexicographic) -> its 3^d node indices, per-axis sizes h */
static void element_nodes(const mesh_t *m, int64_t e, int64_t *nodes, double *h) {
  int ea[3] = {0, 0, 0};
  int64_t r = e;
  for (int a = 0; a < m->dim; ++a) {
    ea[a] = (int)(r % m->cells[a]);
    r /= m->cells[a];
  }
  for (int a = 0; a < m->dim; ++a)
    h[a] = m->coords[a][2 * ea[a] + 2] - m->coords[a][2 * ea[a]];
  int nn = m->dim == 2 ? 9 : 27;
  for (int i = 0; i < nn; ++i) {
    int la[3] = {i % 3, (i / 3) % 3, i / 9};
    int64_t g = 0, stride = 1;
    for (int a = 0; a < m->dim; ++a) {
      g += stride * (2 * ea[a] + la[a]);
      stride *= m->nnode[a];
    }
    nodes[i] = g;
  }
}

/* value and gradient of a nodal vector field (dim components, node-major) */
static void field_at(int d, int nn, const double *N, const double (*dNp)[MAXD],
                     const double *fld, const int64_t *nodes, double *val,
                     double grad[MAXD][MAXD]) {
  for (int c = 0; c < d; ++c) {
    val[c] = 0.0;
    for (int m = 0; m < d; ++m) grad[c][m] = 0.0;
  }
  for (int i = 0; i < nn; ++i) {
    const double *f = fld + nodes[i] * d;
    for (int c = 0; c < d; ++c) {
      val[c] += N[i] * f[c];
      for (int m = 0; m < d; ++m) grad[c][m] += dNp[i][m] * f[c];
    }
  }
}

static int64_t find_block(const int32_t *rowptr, const int32_t *colind, int64_t row,
                          int64_t col) {
  int64_t lo = rowptr[row], hi = rowptr[row + 1] - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) >> 1;
    int64_t c = colind[mid];
    if (c == col) return mid;
    if (c < col) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/*
 * Full Q2 block pattern: node r couples with node c iff they share a cell.
 * Pass rowptr only (colind NULL) to get counts; then again with colind.
 */
int fsigen_pattern(int dim, const int *cells, int32_t *rowptr, int32_t *colind) {
  int nn[3] = {1, 1, 1};
  for (int a = 0; a < dim; ++a) nn[a] = 2 * cells[a] + 1;
  int64_t n = (int64_t)nn[0] * nn[1] * nn[2];
  /* 1D neighbour ranges */
  int *lo[3], *hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = (int *)malloc(sizeof(int) * nn[a]);
    hi[a] = (int *)malloc(sizeof(int) * nn[a]);
    for (int g = 0; g < nn[a]; ++g) {
      if (a >= dim) { lo[a][g] = 0; hi[a][g] = 0; continue; }
      if (g % 2 == 1) { lo[a][g] = g - 1; hi[a][g] = g + 1; }
      else {
        lo[a][g] = g - 2 < 0 ? 0 : g - 2;
        hi[a][g] = g + 2 > nn[a] - 1 ? nn[a] - 1 : g + 2;
      }
    }
  }
  int64_t pos = 0;
  rowptr[0] = 0;
  for (int64_t r = 0; r < n; ++r) {
    int gx = (int)(r % nn[0]), gy = (int)((r / nn[0]) % nn[1]), gz = (int)(r / ((int64_t)nn[0] * nn[1]));
    for (int z = lo[2][gz]; z <= hi[2][gz]; ++z)
      for (int y = lo[1][gy]; y <= hi[1][gy]; ++y)
        for (int x = lo[0][gx]; x <= hi[0][gx]; ++x) {
          if (colind) colind[pos] = (int32_t)(x + (int64_t)nn[0] * (y + (int64_t)nn[1] * z));
          ++pos;
        }
    rowptr[r + 1] = (int32_t)pos;
  }
  for (int a = 0; a < 3; ++a) { free(lo[a]); free(hi[a]); }
  return 0;
}

static void scatter_block(double *vals, int b, const int32_t *rowptr, const int32_t *colind,
                          const int64_t *nodes, int nn, int lb, const double *Ke) {
  /* Ke is (nn*lb) x (nn*lb), node-major; blocks of size lb <= b written to
     the top-left of the b x b block */
  int ld = nn * lb;
  for (int i = 0; i < nn; ++i)
    for (int j = 0; j < nn; ++j) {
      int64_t pos = find_block(rowptr, colind, nodes[i], nodes[j]);
      if (pos < 0) continue; /* cannot happen for the full pattern */
      double *blk = vals + pos * (int64_t)b * b;
      for (int a = 0; a < lb; ++a)
        for (int c = 0; c < lb; ++c) blk[a * b + c] += Ke[(i * lb + a) * ld + j * lb + c];
    }
}

/*
 * Assemble momentum (b = dim+1), ALE (b = dim), solid mass (b = dim) and the
 * scalar mass (b = 1) on one level.  Any of the value arrays may be NULL.
 * Returns 0, or -1 if det F <= 0 at some Gauss point.
 */
int fsigen_assemble(int dim, const int *cells, const double *cx, const double *cy,
                    const double *cz, const double *xyz, const uint8_t *cell_solid,
                    const double *v_old,
                    const double *u_old, const double *v_cur, const double *u_cur,
                    const double *params, const int32_t *rowptr, const int32_t *colind,
                    double *vals_mom, double *vals_ale, double *vals_mass,
                    double *vals_smass, int nthreads) {
  (void)v_old;
  phys_params P = {params[0], params[1], params[2], params[3],
                   params[4], params[5], params[6], params[7]};
  mesh_t M;
  M.dim = dim;
  M.coords[0] = cx; M.coords[1] = cy; M.coords[2] = cz;
  M.xyz = xyz;
  int64_t ncell = 1;
  for (int a = 0; a < 3; ++a) {
    M.cells[a] = a < dim ? cells[a] : 1;
    M.nnode[a] = a < dim ? 2 * cells[a] + 1 : 1;
    if (a < dim) ncell *= cells[a];
  }
  ref_tables T;
  make_tables(dim, &T);
  const int nn = T.nn, nq = T.nq, d = dim, bm = dim + 1;
  int bad = 0;
  const int ncolour = 1 << dim;
  for (int colour = 0; colour < ncolour; ++colour) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads) reduction(min : bad)
    for (int64_t e = 0; e < ncell; ++e) {
      int64_t r = e;
      int col = 0;
      for (int a = 0; a < dim; ++a) {
        col |= (int)((r % M.cells[a]) & 1) << a;
        r /= M.cells[a];
      }
      if (col != colour) continue;
      int64_t nodes[MAXN];
      double h[3];
      element_nodes(&M, e, nodes, h);
      const double hK = cell_size(&M, nodes, h);
      const int solid = cell_solid[e] != 0;
      double Km[MAXN * 4 * MAXN * 4];
      double Ka[MAXN * 3 * MAXN * 3];
      double Ks[MAXN * MAXN];
      memset(Km, 0, sizeof(double) * nn * bm * nn * bm);
      memset(Ka, 0, sizeof(double) * nn * d * nn * d);
      memset(Ks, 0, sizeof(double) * nn * nn);
      const int ldm = nn * bm, lda = nn * d;
      for (int q = 0; q < nq; ++q) {
        double wq, dNp[MAXN][MAXD];
        if (point_geometry(&M, &T, nodes, h, q, &wq, dNp)) bad = -1;
        const double *Nq = T.N[q];
        for (int i = 0; i < nn; ++i)
          for (int j = 0; j < nn; ++j) Ks[i * nn + j] += wq * Nq[i] * Nq[j];
        double v[MAXD], gv[MAXD][MAXD], u[MAXD], gu[MAXD][MAXD], uo[MAXD], guo[MAXD][MAXD];
        field_at(d, nn, Nq, (const double(*)[MAXD])dNp, v_cur, nodes, v, gv);
        field_at(d, nn, Nq, (const double(*)[MAXD])dNp, u_cur, nodes, u, gu);
        field_at(d, nn, Nq, (const double(*)[MAXD])dNp, u_old, nodes, uo, guo);
        double F[MAXD][MAXD], Fi[MAXD][MAXD];
        for (int a = 0; a < d; ++a)
          for (int m = 0; m < d; ++m) F[a][m] = (a == m ? 1.0 : 0.0) + gu[a][m];
        const double J = det_d(d, F);
        if (!(J > 0.0)) bad = -1;
        inv_d(d, F, Fi);
        if (!solid) {
          double Fo[MAXD][MAXD], Fb[MAXD][MAXD], Fbi[MAXD][MAXD];
          for (int a = 0; a < d; ++a)
            for (int m = 0; m < d; ++m) {
              Fo[a][m] = (a == m ? 1.0 : 0.0) + guo[a][m];
              Fb[a][m] = 0.5 * (F[a][m] + Fo[a][m]);
            }
          const double Jo = det_d(d, Fo);
          const double Jb = 0.5 * (J + Jo);
          inv_d(d, Fb, Fbi);
          const double kt = P.k * P.theta;
          double wv[MAXD], av[MAXD], R[MAXD][MAXD];
          for (int a = 0; a < d; ++a) {
            double s = 0.0, t = 0.0;
            for (int m = 0; m < d; ++m) {
              s += Fbi[a][m] * (u[m] - uo[m]);
              t += Fi[a][m] * v[m];
            }
            wv[a] = Jb * s;
            av[a] = kt * P.rho_f * J * t - P.rho_f * P.theta * wv[a];
          }
          for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
              double s = 0.0;
              for (int m = 0; m < d; ++m) s += gv[a][m] * Fi[m][b];
              R[a][b] = kt * P.rho_f * J * s;
            }
          const double visc = kt * P.rho_f * P.nu_f * J;
          const double cm = P.rho_f * Jb;
          const double dK = P.alpha0 * P.k * P.k * hK * hK / (P.rho_f * (hK * hK + kt * P.nu_f));
          double g[MAXN][MAXD], adn[MAXN];
          for (int i = 0; i < nn; ++i) {
            adn[i] = 0.0;
            for (int kk = 0; kk < d; ++kk) {
              double s = 0.0;
              for (int m = 0; m < d; ++m) s += Fi[m][kk] * dNp[i][m];
              g[i][kk] = s;
              adn[i] += av[kk] * dNp[i][kk];
            }
          }
          for (int i = 0; i < nn; ++i)
            for (int j = 0; j < nn; ++j) {
              double gg = 0.0, dd = 0.0;
              for (int m = 0; m < d; ++m) { gg += g[i][m] * g[j][m]; dd += dNp[i][m] * dNp[j][m]; }
              const double NN = Nq[i] * Nq[j];
              const double diag = cm * NN + Nq[i] * adn[j] + visc * gg;
              double *row0 = Km + (int64_t)(i * bm) * ldm + j * bm;
              /* pressure-pressure */
              row0[0] += wq * dK * dd;
              for (int b = 0; b < d; ++b) {
                /* divergence row: k J N_i (g_j)_b */
                row0[1 + b] += wq * P.k * J * Nq[i] * g[j][b];
              }
              for (int a = 0; a < d; ++a) {
                double *row = Km + (int64_t)(i * bm + 1 + a) * ldm + j * bm;
                row[0] += wq * (-P.k * J * Nq[j] * g[i][a]);
                for (int b = 0; b < d; ++b) {
                  double val = NN * R[a][b] + visc * g[j][a] * g[i][b];
                  if (a == b) val += diag;
                  row[1 + b] += wq * val;
                }
              }
              for (int a = 0; a < d; ++a) Ka[(i * d + a) * lda + j * d + a] += wq * dd;
            }
        } else {
          double E[MAXD][MAXD], S[MAXD][MAXD], FFt[MAXD][MAXD];
          double trE = 0.0;
          for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
              double s = 0.0, t = 0.0;
              for (int m = 0; m < d; ++m) { s += F[m][a] * F[m][b]; t += F[a][m] * F[b][m]; }
              E[a][b] = 0.5 * (s - (a == b ? 1.0 : 0.0));
              FFt[a][b] = t;
            }
          for (int a = 0; a < d; ++a) trE += E[a][a];
          for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b)
              S[a][b] = 2.0 * P.mu_s * E[a][b] + (a == b ? P.lambda_s * trE : 0.0);
          const double kt2 = P.k * P.theta * P.k * P.theta;
          double FdN[MAXN][MAXD];
          for (int i = 0; i < nn; ++i)
            for (int a = 0; a < d; ++a) {
              double s = 0.0;
              for (int m = 0; m < d; ++m) s += F[a][m] * dNp[i][m];
              FdN[i][a] = s;
            }
          for (int i = 0; i < nn; ++i)
            for (int j = 0; j < nn; ++j) {
              double cSa = 0.0, ca = 0.0;
              for (int m = 0; m < d; ++m) {
                ca += dNp[j][m] * dNp[i][m];
                for (int n2 = 0; n2 < d; ++n2) cSa += dNp[j][m] * S[m][n2] * dNp[i][n2];
              }
              const double NN = Nq[i] * Nq[j];
              for (int a = 0; a < d; ++a) {
                double *row = Km + (int64_t)(i * bm + 1 + a) * ldm + j * bm;
                for (int b = 0; b < d; ++b) {
                  double val = kt2 * (P.mu_s * (FdN[j][a] * FdN[i][b] + FFt[a][b] * ca) +
                                      P.lambda_s * FdN[j][b] * FdN[i][a]);
                  if (a == b) val += P.rho_s * NN + kt2 * cSa;
                  row[1 + b] += wq * val;
                }
              }
            }
        }
      }
      if (vals_mom) scatter_block(vals_mom, bm, rowptr, colind, nodes, nn, bm, Km);
      if (vals_ale && !solid) scatter_block(vals_ale, d, rowptr, colind, nodes, nn, d, Ka);
      if (vals_mass && solid) {
        double Kms[MAXN * 3 * MAXN * 3];
        memset(Kms, 0, sizeof(double) * lda * lda);
        for (int i = 0; i < nn; ++i)
          for (int j = 0; j < nn; ++j)
            for (int a = 0; a < d; ++a) Kms[(i * d + a) * lda + j * d + a] = Ks[i * nn + j];
        scatter_block(vals_mass, d, rowptr, colind, nodes, nn, d, Kms);
      }
      if (vals_smass) scatter_block(vals_smass, 1, rowptr, colind, nodes, nn, 1, Ks);
    }
  }
  return bad;
}

/*
 * Nonlinear momentum residual (rows (p, v) per node) used only to check the
 * assembled Jacobian by finite differences.  Fluid cells use the frozen
 * deformation u_frz; solid cells recompute u from the velocity through the
 * condensation u = u_old + k theta v + k (1-theta) v_old.
 */
int fsigen_residual(int dim, const int *cells, const double *cx, const double *cy,
                    const double *cz, const double *xyz, const uint8_t *cell_solid,
                    const double *v_old,
                    const double *u_old, const double *u_frz, const double *v,
                    const double *p, const double *params, double *res) {
  phys_params P = {params[0], params[1], params[2], params[3],
                   params[4], params[5], params[6], params[7]};
  mesh_t M;
  M.dim = dim;
  M.coords[0] = cx; M.coords[1] = cy; M.coords[2] = cz;
  M.xyz = xyz;
  int64_t ncell = 1, nnodes = 1;
  for (int a = 0; a < 3; ++a) {
    M.cells[a] = a < dim ? cells[a] : 1;
    M.nnode[a] = a < dim ? 2 * cells[a] + 1 : 1;
    if (a < dim) { ncell *= cells[a]; nnodes *= M.nnode[a]; }
  }
  ref_tables T;
  make_tables(dim, &T);
  const int nn = T.nn, d = dim, bm = dim + 1;
  const double kt = P.k * P.theta;
  memset(res, 0, sizeof(double) * nnodes * bm);
  double *us = (double *)malloc(sizeof(double) * nnodes * d);
  for (int64_t i = 0; i < nnodes * d; ++i)
    us[i] = u_old[i] + kt * v[i] + P.k * (1.0 - P.theta) * v_old[i];
  for (int64_t e = 0; e < ncell; ++e) {
    int64_t nodes[MAXN];
    double h[3];
    element_nodes(&M, e, nodes, h);
    const double hK = cell_size(&M, nodes, h);
    const int solid = cell_solid[e] != 0;
    for (int q = 0; q < T.nq; ++q) {
      double wq, dNp[MAXN][MAXD];
      (void)point_geometry(&M, &T, nodes, h, q, &wq, dNp);
      const double *Nq = T.N[q];
      double vv[MAXD], gv[MAXD][MAXD], vo[MAXD], gvo[MAXD][MAXD];
      double u[MAXD], gu[MAXD][MAXD], uo[MAXD], guo[MAXD][MAXD];
      field_at(d, nn, Nq, (const double(*)[MAXD])dNp, v, nodes, vv, gv);
      field_at(d, nn, Nq, (const double(*)[MAXD])dNp, v_old, nodes, vo, gvo);
      field_at(d, nn, Nq, (const double(*)[MAXD])dNp, solid ? us : u_frz, nodes, u, gu);
      field_at(d, nn, Nq, (const double(*)[MAXD])dNp, u_old, nodes, uo, guo);
      double pq = 0.0, gp[MAXD] = {0, 0, 0};
      for (int i = 0; i < nn; ++i) {
        pq += Nq[i] * p[nodes[i]];
        for (int m = 0; m < d; ++m) gp[m] += dNp[i][m] * p[nodes[i]];
      }
      double F[MAXD][MAXD], Fi[MAXD][MAXD];
      for (int a = 0; a < d; ++a)
        for (int m = 0; m < d; ++m) F[a][m] = (a == m ? 1.0 : 0.0) + gu[a][m];
      const double J = det_d(d, F);
      inv_d(d, F, Fi);
      if (!solid) {
        double Fo[MAXD][MAXD], Fb[MAXD][MAXD], Fbi[MAXD][MAXD];
        for (int a = 0; a < d; ++a)
          for (int m = 0; m < d; ++m) {
            Fo[a][m] = (a == m ? 1.0 : 0.0) + guo[a][m];
            Fb[a][m] = 0.5 * (F[a][m] + Fo[a][m]);
          }
        const double Jb = 0.5 * (J + det_d(d, Fo));
        inv_d(d, Fb, Fbi);
        /* vector pieces: inertia, mesh transport of vbar, convection */
        double wv[MAXD], a1[MAXD];
        for (int a = 0; a < d; ++a) {
          double s = 0.0, t = 0.0;
          for (int m = 0; m < d; ++m) { s += Fbi[a][m] * (u[m] - uo[m]); t += Fi[a][m] * vv[m]; }
          wv[a] = Jb * s;
          a1[a] = t;
        }
        double vec[MAXD];
        for (int a = 0; a < d; ++a) {
          double tr = 0.0, cv = 0.0;
          for (int m = 0; m < d; ++m) {
            double gvb = P.theta * gv[a][m] + (1.0 - P.theta) * gvo[a][m];
            tr += wv[m] * gvb;
            cv += a1[m] * gv[a][m];
          }
          vec[a] = P.rho_f * Jb * (vv[a] - vo[a]) - P.rho_f * tr + kt * P.rho_f * J * cv;
        }
        /* tensor: viscous + pressure, tested with grad phi */
        double G[MAXD][MAXD], S[MAXD][MAXD], T2[MAXD][MAXD];
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) {
            double s = 0.0;
            for (int m = 0; m < d; ++m) s += gv[a][m] * Fi[m][b];
            G[a][b] = s;
          }
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) S[a][b] = G[a][b] + G[b][a];
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) {
            double s = 0.0;
            for (int m = 0; m < d; ++m) s += S[a][m] * Fi[b][m];
            T2[a][b] = kt * P.rho_f * P.nu_f * J * s - P.k * J * pq * Fi[b][a];
          }
        double divv = 0.0;
        for (int a = 0; a < d; ++a) divv += G[a][a];
        const double dK = P.alpha0 * P.k * P.k * hK * hK / (P.rho_f * (hK * hK + kt * P.nu_f));
        for (int i = 0; i < nn; ++i) {
          double *r = res + nodes[i] * bm;
          double gg = 0.0;
          for (int m = 0; m < d; ++m) gg += gp[m] * dNp[i][m];
          r[0] += wq * (P.k * J * divv * Nq[i] + dK * gg);
          for (int a = 0; a < d; ++a) {
            double s = vec[a] * Nq[i];
            for (int m = 0; m < d; ++m) s += T2[a][m] * dNp[i][m];
            r[1 + a] += wq * s;
          }
        }
      } else {
        double E[MAXD][MAXD], S[MAXD][MAXD], FS[MAXD][MAXD];
        double trE = 0.0;
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) {
            double s = 0.0;
            for (int m = 0; m < d; ++m) s += F[m][a] * F[m][b];
            E[a][b] = 0.5 * (s - (a == b ? 1.0 : 0.0));
          }
        for (int a = 0; a < d; ++a) trE += E[a][a];
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b)
            S[a][b] = 2.0 * P.mu_s * E[a][b] + (a == b ? P.lambda_s * trE : 0.0);
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) {
            double s = 0.0;
            for (int m = 0; m < d; ++m) s += F[a][m] * S[m][b];
            FS[a][b] = s;
          }
        for (int i = 0; i < nn; ++i) {
          double *r = res + nodes[i] * bm;
          for (int a = 0; a < d; ++a) {
            double s = P.rho_s * (vv[a] - vo[a]) * Nq[i];
            for (int m = 0; m < d; ++m) s += kt * FS[a][m] * dNp[i][m];
            r[1 + a] += wq * s;
          }
        }
      }
    }
  }
  free(us);
  return 0;
}
