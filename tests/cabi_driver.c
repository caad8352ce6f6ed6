/* Plain-C client of the fsimg C ABI (no Python, no torch): reads a hierarchy
 * written by tests/test_gpu_cabi.py, solves it on the GPU and writes x.
 *
 *   cabi_driver <dir> <precision 0|1>
 *
 * <dir>/meta.txt: nlev dim block, then per level: cells0 cells1 cells2 nrows nnzb
 * <dir>/L<l>_{rowptr,colind,dirichlet,cellclass}.bin, L<l>_vals.bin (float64),
 * <dir>/rhs.bin (float64); writes <dir>/x.bin and prints "status iters rel_res". */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "fsimg.h"

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

int main(int argc, char **argv) {
  if (argc != 3) { fprintf(stderr, "usage: %s <dir> <precision>\n", argv[0]); return 2; }
  const char *dir = argv[1];
  char path[4096];
  snprintf(path, sizeof path, "%s/meta.txt", dir);
  FILE *m = fopen(path, "r");
  if (!m) { fprintf(stderr, "no meta\n"); return 2; }
  int nlev, dim, block;
  if (fscanf(m, "%d %d %d", &nlev, &dim, &block) != 3 || nlev < 1 || nlev > 16) return 2;
  fsimg_level_desc lv[16];
  memset(lv, 0, sizeof lv);
  for (int l = 0; l < nlev; ++l) {
    long long nrows, nnzb;
    if (fscanf(m, "%d %d %d %lld %lld", &lv[l].cells[0], &lv[l].cells[1], &lv[l].cells[2], &nrows,
               &nnzb) != 5)
      return 2;
    lv[l].dim = dim;
    lv[l].block = block;
    lv[l].nrows = nrows;
    lv[l].nnzb = nnzb;
    char name[64];
    long long ncell = (long long)lv[l].cells[0] * lv[l].cells[1] * lv[l].cells[2];
    snprintf(name, sizeof name, "L%d_rowptr.bin", l);
    lv[l].rowptr = slurp(dir, name, (size_t)(nrows + 1) * 4);
    snprintf(name, sizeof name, "L%d_colind.bin", l);
    lv[l].colind = slurp(dir, name, (size_t)nnzb * 4);
    snprintf(name, sizeof name, "L%d_vals.bin", l);
    lv[l].vals = slurp(dir, name, (size_t)nnzb * block * block * 8);
    snprintf(name, sizeof name, "L%d_dirichlet.bin", l);
    lv[l].dirichlet = slurp(dir, name, (size_t)nrows * block);
    snprintf(name, sizeof name, "L%d_cellclass.bin", l);
    lv[l].cell_class = slurp(dir, name, (size_t)ncell);
  }
  fclose(m);
  const size_t n = (size_t)lv[0].nrows * block;
  double *rhs = slurp(dir, "rhs.bin", n * 8);

  fsimg_ctx *ctx = NULL;
  fsimg_hier *h = NULL;
  fsimg_opts opts;
  fsimg_default_opts(&opts);
  opts.precision = atoi(argv[2]) ? FSIMG_MIXED : FSIMG_FP64;
  fsimg_status st = fsimg_ctx_create(0, 0, &ctx);
  if (st == FSIMG_OK) st = fsimg_hier_create(ctx, lv, nlev, &opts, NULL, &h);
  if (st == FSIMG_OK) st = fsimg_factor(h, NULL);
  double *b_dev = NULL, *x_dev = NULL;
  fsimg_stats stats;
  memset(&stats, 0, sizeof stats);
  if (st == FSIMG_OK) {
    double *zero = calloc(n, sizeof(double));
    if (hipMalloc((void **)&b_dev, n * 8) != hipSuccess || hipMalloc((void **)&x_dev, n * 8) != hipSuccess ||
        hipMemcpy(b_dev, rhs, n * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(x_dev, zero, n * 8, hipMemcpyHostToDevice) != hipSuccess) {
      fprintf(stderr, "HIP setup failed\n");
      return 3;
    }
    free(zero);
    st = fsimg_solve(h, b_dev, x_dev, &stats, NULL);
  }
  if (st != FSIMG_OK) {
    fprintf(stderr, "fsimg error %d: %s\n", (int)st, fsimg_last_error());
    return 1;
  }
  double *x = malloc(n * 8);
  if (hipMemcpy(x, x_dev, n * 8, hipMemcpyDeviceToHost) != hipSuccess) return 3;
  snprintf(path, sizeof path, "%s/x.bin", dir);
  FILE *f = fopen(path, "wb");
  if (!f || fwrite(x, 8, n, f) != n) return 2;
  fclose(f);
  printf("%d %d %.6e\n", stats.status, stats.iters, stats.rel_res);
  (void)hipFree(b_dev);
  (void)hipFree(x_dev);
  fsimg_hier_destroy(h);
  fsimg_ctx_destroy(ctx);
  for (int l = 0; l < nlev; ++l) {
    free((void *)lv[l].rowptr);
    free((void *)lv[l].colind);
    free((void *)lv[l].vals);
    free((void *)lv[l].dirichlet);
    free((void *)lv[l].cell_class);
  }
  free(rhs);
  free(x);
  return 0;
}
