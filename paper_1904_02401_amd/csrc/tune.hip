// Launch-shape table and its tuner.  Only shapes that cannot change a
// result bit are tuned: the SpMV rows per wavefront (every row is summed by
// the same lane mapping and tree whatever wave holds it) and the Vanka
// patches per workgroup (every patch is computed by the same row threads in
// the same order).  Keys never depend on a batch composition.
#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "hier.h"

using namespace fsimg;

namespace {

int bucket_of(int64_t size) {
  int k = 0;
  while (size > 1) {
    size >>= 1;
    ++k;
  }
  return k;
}

bool valid_value(int kind, int key, int value) {
  if (kind == FSIMG_TUNE_SPMV_ROWS) return value == 1 || value == 2 || value == 4;
  if (kind == FSIMG_TUNE_VANKA_PPW) return key > 0 && value >= 1 && (int64_t)value * key <= 1024;
  return false;
}

bool valid_key(int kind, int key, int word) {
  if (word != 4 && word != 8) return false;
  if (kind == FSIMG_TUNE_SPMV_ROWS) return key >= 1 && key <= 4;
  if (kind == FSIMG_TUNE_VANKA_PPW) return key >= 1 && key <= 1024;
  return false;
}

// built-in SpMV default: rows per wavefront by block size and word
int default_rows(int b, int word) {
  (void)b;
  (void)word;
  return 1;
}

int lookup(const TuneTable *t, int kind, int key, int word, int64_t size, int fallback) {
  if (!t) return fallback;
  auto it = t->entries.find({kind, key, word, bucket_of(size)});
  return it == t->entries.end() ? fallback : it->second;
}

std::string arch_name(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// average ms of `reps` launches after one warm-up launch
template <typename F>
double time_launches(F &&launch, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps) {
  launch();
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, s);
  if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
  return ms / reps;
}

// Vanka candidates: ppw with at least 75 % of the workgroup's lanes busy
std::vector<int> ppw_candidates(int np) {
  std::vector<int> c;
  for (int p = 1; (int64_t)p * np <= 1024; ++p)
    if ((double)(p * np) / vanka_threads(np, p) >= 0.75) c.push_back(p);
  return c;
}

template <typename T>
struct LevelVec;
template <>
struct LevelVec<double> {
  static const double *vals(const DevLevel &L) { return L.vals64; }
  static const double *inv(const DevLevel &L, int g) { return g ? L.blk.inv64 : L.inv64; }
  static int npc(const DevLevel &L, int g) { return g ? L.blk.npc64 : L.npc64; }
  static double *x(const DevLevel &L) { return L.x64; }
  static double *r(const DevLevel &L) { return L.r64; }
  static double *d(const DevLevel &L) { return L.d64; }
  static double *Y(const DevLevel &L) { return L.Y64; }
};
template <>
struct LevelVec<float> {
  static const float *vals(const DevLevel &L) { return L.vals32; }
  static const float *inv(const DevLevel &L, int g) { return g ? L.blk.inv32 : L.inv32; }
  static int npc(const DevLevel &L, int g) { return g ? L.blk.npc32 : L.npc32; }
  static float *x(const DevLevel &L) { return L.x32; }
  static float *r(const DevLevel &L) { return L.r32; }
  static float *d(const DevLevel &L) { return L.d32; }
  static float *Y(const DevLevel &L) { return L.Y32; }
};

struct Tuner {
  TuneTable &t;
  bool force;
  hipStream_t s;
  hipEvent_t e0, e1;
  bool changed = false;

  bool need(int kind, int key, int word, int64_t size) const {
    return force || !t.entries.count({kind, key, word, bucket_of(size)});
  }

  template <typename T>
  void spmv(const DevLevel &L, const T *vals, const T *x, const T *b, T *y) {
    const int word = (int)sizeof(T);
    if (L.nrows == 0 || !need(FSIMG_TUNE_SPMV_ROWS, L.b, word, L.nrows)) return;
    int best = 1;
    double best_ms = 1e300;
    for (int R : {1, 2, 4}) {
      const double ms = time_launches(
          [&] { launch_bsr_spmv_rpw<T>(L, vals, x, b, y, true, R, s); }, s, e0, e1, 5);
      if (ms >= 0.0 && ms < best_ms) { best_ms = ms; best = R; }
      if (ms > 1.5 * best_ms) break;  // more rows per wave only gets slower from here
    }
    t.entries[{FSIMG_TUNE_SPMV_ROWS, L.b, word, bucket_of(L.nrows)}] = best;
    changed = true;
  }

  template <typename T>
  void vanka(const DevLevel &L, int g) {
    const int word = (int)sizeof(T);
    const int64_t npatch = g ? L.blk.npatch : L.npatch;
    const int np = g ? L.blk.np : L.np;
    if (npatch == 0 || !need(FSIMG_TUNE_VANKA_PPW, np, word, npatch)) return;
    int best = vanka_default_ppw(np);
    double best_ms = 1e300;
    T *Y = LevelVec<T>::Y(L) + (g ? L.blk.yofs : 0);
    for (int p : ppw_candidates(np)) {
      const double ms = time_launches(
          [&] {
            launch_vanka_patch_ppw<T>(L, g, LevelVec<T>::inv(L, g), LevelVec<T>::npc(L, g),
                                      LevelVec<T>::r(L), Y, p, s);
          },
          s, e0, e1, 5);
      if (ms >= 0.0 && ms < best_ms) { best_ms = ms; best = p; }
    }
    t.entries[{FSIMG_TUNE_VANKA_PPW, np, word, bucket_of(npatch)}] = best;
    changed = true;
  }

  template <typename T>
  void levels(fsimg_hier *h) {
    const int nl = (int)h->lev.size();
    for (int l = 0; l + 1 < nl; ++l) {  // levels that smooth
      const DevLevel &L = h->lev[l];
      spmv<T>(L, LevelVec<T>::vals(L), LevelVec<T>::x(L), LevelVec<T>::r(L), LevelVec<T>::d(L));
      if (h->opts.smoother != FSIMG_SMOOTHER_VANKA) continue;  // no patch inverses to time
      vanka<T>(L, 0);
      vanka<T>(L, 1);
    }
  }
};

}  // namespace

namespace fsimg {

int spmv_rows_per_wave(const TuneTable *t, int b, int word, int64_t nrows) {
  return lookup(t, FSIMG_TUNE_SPMV_ROWS, b, word, nrows, default_rows(b, word));
}

int vanka_patches_per_wg(const TuneTable *t, int np, int word, int64_t npatch) {
  return lookup(t, FSIMG_TUNE_VANKA_PPW, np, word, npatch, vanka_default_ppw(np));
}

}  // namespace fsimg

extern "C" {

fsimg_status fsimg_hier_tune(fsimg_hier *h, int force, void *stream) {
  if (!h) return set_error(FSIMG_ERR_ARG, "null hierarchy");
  if (!h->factored) return set_error(FSIMG_ERR_STATE, "fsimg_factor must run before tuning");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return set_error(FSIMG_ERR_HIP, "event creation failed");
  }
  Tuner tu{h->ctx->tune, force != 0, s, e0, e1};
  if (h->opts.precision == FSIMG_MIXED) {
    tu.levels<float>(h);
    // the outer FP64 product on level 0, on the Krylov work vectors
    tu.spmv<double>(h->lev[0], h->lev[0].vals64, h->V, h->Z, h->w);
  } else {
    tu.levels<double>(h);
  }
  const hipError_t e = hipStreamSynchronize(s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return set_error(FSIMG_ERR_HIP, std::string("tuning: ") + hipGetErrorString(e));
  if (tu.changed) drop_plans(h->ctx);
  return FSIMG_OK;
}

fsimg_status fsimg_tune_set(fsimg_ctx *ctx, int kind, int key, int word, int64_t size, int value) {
  if (!ctx || !valid_key(kind, key, word) || size < 1 || !valid_value(kind, key, value))
    return set_error(FSIMG_ERR_ARG, "bad tuning key or value");
  ctx->tune.entries[{kind, key, word, bucket_of(size)}] = value;
  drop_plans(ctx);
  return FSIMG_OK;
}

fsimg_status fsimg_tune_get(const fsimg_ctx *ctx, int kind, int key, int word, int64_t size,
                            int *value) {
  if (!ctx || !value || !valid_key(kind, key, word) || size < 1)
    return set_error(FSIMG_ERR_ARG, "bad tuning key");
  *value = kind == FSIMG_TUNE_SPMV_ROWS ? spmv_rows_per_wave(&ctx->tune, key, word, size)
                                        : vanka_patches_per_wg(&ctx->tune, key, word, size);
  return FSIMG_OK;
}

fsimg_status fsimg_tune_save(const fsimg_ctx *ctx, const char *path) {
  if (!ctx || !path) return set_error(FSIMG_ERR_ARG, "null context or path");
  std::ofstream f(path);
  if (!f) return set_error(FSIMG_ERR_ARG, std::string("cannot write ") + path);
  f << "{\"arch\": \"" << arch_name(ctx->device) << "\", \"entries\": [";
  bool first = true;
  for (const auto &kv : ctx->tune.entries) {
    f << (first ? "\n  " : ",\n  ") << "{\"kind\": " << kv.first[0] << ", \"key\": " << kv.first[1]
      << ", \"word\": " << kv.first[2] << ", \"bucket\": " << kv.first[3]
      << ", \"value\": " << kv.second << "}";
    first = false;
  }
  f << "\n]}\n";
  return f.good() ? FSIMG_OK : set_error(FSIMG_ERR_ARG, std::string("write failed: ") + path);
}

fsimg_status fsimg_tune_load(fsimg_ctx *ctx, const char *path) {
  if (!ctx || !path) return set_error(FSIMG_ERR_ARG, "null context or path");
  std::ifstream f(path);
  if (!f) return set_error(FSIMG_ERR_ARG, std::string("cannot read ") + path);
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string txt = ss.str();
  auto fail = [&](const std::string &m) {
    return set_error(FSIMG_ERR_ARG, std::string(path) + ": " + m);
  };
  // "arch": "<name>"
  size_t p = txt.find("\"arch\"");
  if (p == std::string::npos) return fail("no arch");
  size_t q0 = txt.find('"', txt.find(':', p) + 1), q1 = txt.find('"', q0 + 1);
  if (q0 == std::string::npos || q1 == std::string::npos) return fail("bad arch");
  const std::string arch = txt.substr(q0 + 1, q1 - q0 - 1);
  if (arch != arch_name(ctx->device)) return fail("written for " + arch);
  size_t e = txt.find("\"entries\"");
  if (e == std::string::npos) return fail("no entries");
  e = txt.find('[', e);
  const size_t end = txt.find(']', e);
  if (e == std::string::npos || end == std::string::npos) return fail("bad entries");
  std::vector<std::pair<std::array<int, 4>, int>> got;
  for (size_t o = txt.find('{', e); o != std::string::npos && o < end; o = txt.find('{', o + 1)) {
    const size_t c = txt.find('}', o);
    if (c == std::string::npos || c > end) return fail("unterminated entry");
    const std::string obj = txt.substr(o, c - o);
    long v[5];
    const char *names[5] = {"\"kind\"", "\"key\"", "\"word\"", "\"bucket\"", "\"value\""};
    for (int k = 0; k < 5; ++k) {
      const size_t at = obj.find(names[k]);
      const size_t colon = at == std::string::npos ? at : obj.find(':', at);
      if (colon == std::string::npos) return fail(std::string("entry without ") + names[k]);
      errno = 0;
      char *stop = nullptr;
      v[k] = std::strtol(obj.c_str() + colon + 1, &stop, 10);
      if (errno || stop == obj.c_str() + colon + 1) return fail("bad number");
    }
    if (!valid_key((int)v[0], (int)v[1], (int)v[2]) || v[3] < 0 || v[3] > 62 ||
        !valid_value((int)v[0], (int)v[1], (int)v[4]))
      return fail("entry out of range");
    got.push_back({{(int)v[0], (int)v[1], (int)v[2], (int)v[3]}, (int)v[4]});
  }
  for (const auto &g : got) ctx->tune.entries[g.first] = g.second;
  drop_plans(ctx);
  return FSIMG_OK;
}

}  // extern "C"

// ---- Vanka schedule: measured, not result-invariant, so it is reported and
// left to the caller (the hierarchy's schedule is fixed when it is created)
extern "C" fsimg_status fsimg_tune_schedule(fsimg_ctx *ctx, const fsimg_level_desc *levels, int nlev,
                                            const fsimg_opts *opts, int reps, double *ms_out,
                                            int *best, void *stream) {
  if (!ctx || !levels || nlev < 1 || !opts || !ms_out || !best || reps < 1)
    return set_error(FSIMG_ERR_ARG, "bad schedule tuning arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int sched[3] = {FSIMG_VANKA_GATHER, FSIMG_VANKA_PARITY, FSIMG_VANKA_GREEDY};
  const bool f32 = opts->precision == FSIMG_MIXED;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return set_error(FSIMG_ERR_HIP, "event creation failed");
  }
  void *r = nullptr, *z = nullptr;
  fsimg_status ret = FSIMG_OK;
  *best = -1;
  for (int k = 0; k < 3 && ret == FSIMG_OK; ++k) {
    ms_out[k] = -1.0;
    fsimg_opts o = *opts;
    o.vanka_schedule = sched[k];
    o.profile = 0;
    fsimg_hier *h = nullptr;
    const fsimg_status st = fsimg_hier_create(ctx, levels, nlev, &o, stream, &h);
    if (st == FSIMG_ERR_ARG) continue;  // the schedule does not apply (e.g. block patches)
    if (st != FSIMG_OK) {
      ret = st;
      break;
    }
    ret = fsimg_factor(h, stream);
    const size_t bytes = (size_t)h->lev[0].n * (f32 ? sizeof(float) : sizeof(double));
    if (ret == FSIMG_OK && !r) {
      if (hipMalloc(&r, bytes) != hipSuccess || hipMalloc(&z, bytes) != hipSuccess)
        ret = set_error(FSIMG_ERR_OOM, "schedule tuning vectors");
    }
    if (ret == FSIMG_OK) {
      // a fixed non-zero right-hand side: the constant 1 in every dof
      if (f32) {
        std::vector<float> one(h->lev[0].n, 1.0f);
        if (hipMemcpyAsync(r, one.data(), bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          ret = set_error(FSIMG_ERR_HIP, "schedule tuning upload");
      } else {
        std::vector<double> one(h->lev[0].n, 1.0);
        if (hipMemcpyAsync(r, one.data(), bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          ret = set_error(FSIMG_ERR_HIP, "schedule tuning upload");
      }
    }
    if (ret == FSIMG_OK) ret = fsimg_vcycle(h, o.precision, r, z, stream);  // warm-up
    if (ret == FSIMG_OK) {
      (void)hipEventRecord(e0, s);
      for (int q = 0; q < reps && ret == FSIMG_OK; ++q) ret = fsimg_vcycle(h, o.precision, r, z, stream);
      (void)hipEventRecord(e1, s);
      float t = 0.0f;
      if (ret == FSIMG_OK && (hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        ret = set_error(FSIMG_ERR_HIP, "schedule tuning timing");
      if (ret == FSIMG_OK) {
        ms_out[k] = (double)t / reps;
        if (*best < 0 || ms_out[k] < ms_out[*best]) *best = k;
      }
    }
    fsimg_hier_destroy(h);
  }
  if (r) (void)hipFree(r);
  if (z) (void)hipFree(z);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ret == FSIMG_OK && *best >= 0) *best = sched[*best];
  return ret;
}
