/* Plain-C client of the Newton-loop ABI (fsimg_newton.h; no Python, no torch):
 * reads a momentum and an ALE hierarchy, the mesh geometry, the material
 * parameters and a state written by tests/test_gpu_cabi.py, runs one Newton
 * time step on the GPU and writes the new state.
 *
 *   cabi_newton <dir> <precision 0|1>
 *
 * <dir>/meta.txt: nlev dim, then per level: cells0 cells1 cells2 nrows
 *   nnzb_mom nnzb_ale
 * <dir>/{M,A}<l>_{rowptr,colind,vals,dirichlet}.bin: the two systems' levels
 * <dir>/G<l>_c<a>.bin (float64, 2*cells[a]+1), G<l>_solid.bin (uint8)
 * <dir>/phys.bin: rho_f nu_f rho_s mu_s lambda_s k theta alpha0 (float64)
 * <dir>/{x,u,xo,uo}.bin (float64); writes <dir>/{x_out,u_out}.bin and prints
 * "status steps jacobians". */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "fsimg_newton.h"

static void *slurp(const char *dir, const char *name, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE *f = fopen(path, "rb");
  if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
  void *p = malloc(bytes ? bytes : 1);
  if (bytes && fread(p, 1, bytes, f) != bytes) { fprintf(stderr, "short read %s\n", path); exit(2); }
  fclose(f);
  return p;
}

static void read_system(const char *dir, char tag, int l, int dim, int block, const int *cells,
                        long long nrows, long long nnzb, fsimg_level_desc *d) {
  char name[64];
  memset(d, 0, sizeof *d);
  d->dim = dim;
  d->block = block;
  for (int a = 0; a < 3; ++a) d->cells[a] = cells[a];
  d->nrows = nrows;
  d->nnzb = nnzb;
  snprintf(name, sizeof name, "%c%d_rowptr.bin", tag, l);
  d->rowptr = slurp(dir, name, (size_t)(nrows + 1) * 4);
  snprintf(name, sizeof name, "%c%d_colind.bin", tag, l);
  d->colind = slurp(dir, name, (size_t)nnzb * 4);
  snprintf(name, sizeof name, "%c%d_vals.bin", tag, l);
  d->vals = slurp(dir, name, (size_t)nnzb * block * block * 8);
  snprintf(name, sizeof name, "%c%d_dirichlet.bin", tag, l);
  d->dirichlet = slurp(dir, name, (size_t)nrows * block);
}

static int put(const char *dir, const char *name, const double *dev, size_t n) {
  char path[4096];
  double *h = malloc(n * 8);
  if (hipMemcpy(h, dev, n * 8, hipMemcpyDeviceToHost) != hipSuccess) return 3;
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE *f = fopen(path, "wb");
  if (!f || fwrite(h, 8, n, f) != n) return 2;
  fclose(f);
  free(h);
  return 0;
}

int main(int argc, char **argv) {
  if (argc != 3) { fprintf(stderr, "usage: %s <dir> <precision>\n", argv[0]); return 2; }
  const char *dir = argv[1];
  char path[4096];
  snprintf(path, sizeof path, "%s/meta.txt", dir);
  FILE *m = fopen(path, "r");
  if (!m) { fprintf(stderr, "no meta\n"); return 2; }
  int nlev, dim;
  if (fscanf(m, "%d %d", &nlev, &dim) != 2 || nlev < 1 || nlev > 16 || dim < 2 || dim > 3) return 2;
  fsimg_level_desc mom[16], ale[16];
  fsimg_fsi_level geo[16];
  memset(geo, 0, sizeof geo);
  for (int l = 0; l < nlev; ++l) {
    int cells[3];
    long long nrows, nnzb_m, nnzb_a;
    if (fscanf(m, "%d %d %d %lld %lld %lld", &cells[0], &cells[1], &cells[2], &nrows, &nnzb_m, &nnzb_a) != 6)
      return 2;
    read_system(dir, 'M', l, dim, dim + 1, cells, nrows, nnzb_m, &mom[l]);
    read_system(dir, 'A', l, dim, dim, cells, nrows, nnzb_a, &ale[l]);
    char name[64];
    for (int a = 0; a < dim; ++a) {
      snprintf(name, sizeof name, "G%d_c%d.bin", l, a);
      geo[l].coords[a] = slurp(dir, name, (size_t)(2 * cells[a] + 1) * 8);
    }
    long long ncell = (long long)cells[0] * cells[1] * cells[2];
    snprintf(name, sizeof name, "G%d_solid.bin", l);
    geo[l].cell_solid = slurp(dir, name, (size_t)ncell);
  }
  fclose(m);
  double *ph = slurp(dir, "phys.bin", 8 * 8);
  fsimg_phys phys = {ph[0], ph[1], ph[2], ph[3], ph[4], ph[5], ph[6], ph[7]};
  const size_t nm = (size_t)mom[0].nrows * (dim + 1), na = (size_t)mom[0].nrows * dim;
  const char *names[4] = {"x.bin", "u.bin", "xo.bin", "uo.bin"};
  const size_t sizes[4] = {nm, na, nm, na};
  double *dev[4] = {NULL, NULL, NULL, NULL};
  for (int q = 0; q < 4; ++q) {
    double *hbuf = slurp(dir, names[q], sizes[q] * 8);
    if (hipMalloc((void **)&dev[q], sizes[q] * 8) != hipSuccess ||
        hipMemcpy(dev[q], hbuf, sizes[q] * 8, hipMemcpyHostToDevice) != hipSuccess) {
      fprintf(stderr, "HIP setup failed\n");
      return 3;
    }
    free(hbuf);
  }

  fsimg_ctx *ctx = NULL;
  fsimg_hier *hm = NULL, *ha = NULL;
  fsimg_fsi *f = NULL;
  fsimg_opts opts;
  fsimg_default_opts(&opts);
  opts.precision = atoi(argv[2]) ? FSIMG_MIXED : FSIMG_FP64;
  fsimg_newton_opts nopts;
  fsimg_default_newton_opts(&nopts);
  fsimg_newton_stats stats;
  memset(&stats, 0, sizeof stats);
  fsimg_status st = fsimg_ctx_create(0, 0, &ctx);
  if (st == FSIMG_OK) st = fsimg_hier_create(ctx, mom, nlev, &opts, NULL, &hm);
  if (st == FSIMG_OK) st = fsimg_hier_create(ctx, ale, nlev, &opts, NULL, &ha);
  if (st == FSIMG_OK) st = fsimg_fsi_create(hm, ha, geo, &phys, &f);
  if (st == FSIMG_OK) st = fsimg_fsi_newton(f, dev[0], dev[1], dev[2], dev[3], &nopts, &stats, NULL);
  if (st != FSIMG_OK) {
    fprintf(stderr, "fsimg error %d: %s\n", (int)st, fsimg_last_error());
    return 1;
  }
  int rc = put(dir, "x_out.bin", dev[0], nm);
  if (!rc) rc = put(dir, "u_out.bin", dev[1], na);
  if (rc) return rc;
  printf("%d %d %d\n", stats.status, stats.steps, stats.jacobians);
  for (int q = 0; q < 4; ++q) (void)hipFree(dev[q]);
  fsimg_fsi_destroy(f);
  fsimg_hier_destroy(hm);
  fsimg_hier_destroy(ha);
  fsimg_ctx_destroy(ctx);
  for (int l = 0; l < nlev; ++l) {
    fsimg_level_desc *ds[2] = {&mom[l], &ale[l]};
    for (int k = 0; k < 2; ++k) {
      free((void *)ds[k]->rowptr);
      free((void *)ds[k]->colind);
      free((void *)ds[k]->vals);
      free((void *)ds[k]->dirichlet);
    }
    for (int a = 0; a < dim; ++a) free((void *)geo[l].coords[a]);
    free((void *)geo[l].cell_solid);
  }
  free(ph);
  return 0;
}
