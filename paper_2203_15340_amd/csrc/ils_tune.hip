// ils_tune.hip -- the autotuner: sweeps the Gram kernel's launch
// configurations (tile edge x workgroup target, hence the K-split) on the
// caller's matrix, keeps the fastest per (precision, log2 n, log2 K) bucket in
// the process-wide table that every Gram launch consults, and saves / loads
// that table as JSON.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ils_common.hpp"
#include "ils_runtime.hpp"

namespace ils {
std::vector<GramCfgEntry> gram_cfg_entries();
}

using namespace ils;

#define HIPCHK(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return ILS_ERR_HIP; \
  } while (0)

extern "C" int ils_tune_gram(ils_handle* h, int64_t K, int64_t n, const double* A, int64_t lda, int32_t precision,
                             int32_t reps, ils_tune_entry* best) {
  if (!h || !A || n < 1 || K < 1 || lda < K || reps < 1 || reps > 1000) return ILS_ERR_ARG;
  if (precision != ILS_PREC_FP64 && precision != ILS_PREC_MIXED) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  hipStream_t s = h->stream;
  const int tiles[2] = {64, 128};
  const int targets[10] = {256, 512, 1024, 1536, 2048, 3072, 4096, 5120, 6144, 8192};
  size_t part_max = 0;
  for (int t : tiles)
    for (int w : targets) part_max = std::max(part_max, gram_partials_size_cfg(n, K, GramCfg{t, w}));
  double *G, *part;
  int st;
  if ((st = h->need(kBufM, sizeof(double) * n * n, (void**)&G)) ||
      (st = h->need(kBufPart, sizeof(double) * part_max, (void**)&part)))
    return st;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  GramCfg win = gram_default_cfg(n);
  float win_ms = INFINITY;
  for (int t : tiles) {
    for (int w : targets) {
      const GramCfg c{t, w};
      launch_gram_cfg(s, precision, K, n, A, lda, part, G, n, c);  // warm-up
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r) launch_gram_cfg(s, precision, K, n, A, lda, part, G, n, c);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return ILS_ERR_HIP;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= (float)reps;
      if (ms < win_ms) {
        win_ms = ms;
        win = c;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipGetLastError());
  gram_set_cfg(precision, n, K, win);
  if (best) {
    best->kernel = ILS_TUNE_GRAM;
    best->precision = precision;
    best->n = n;
    best->K = K;
    best->tile = win.tile;
    best->workgroups = win.workgroups;
    best->ms = win_ms;
  }
  return ILS_OK;
}

extern "C" int ils_tune_clear(void) {
  gram_clear_cfg();
  return ILS_OK;
}

// One entry per line so that ils_tune_load can read the file back with a
// line scanner; the whole file is ordinary JSON.
extern "C" int ils_tune_save(const char* path) {
  if (!path) return ILS_ERR_ARG;
  FILE* f = fopen(path, "w");
  if (!f) return ILS_ERR_ARG;
  const std::vector<GramCfgEntry> es = gram_cfg_entries();
  fprintf(f, "{\"version\": 1, \"entries\": [\n");
  for (size_t i = 0; i < es.size(); ++i) {
    const GramCfgEntry& e = es[i];
    fprintf(f,
            "  {\"kernel\": \"gram\", \"precision\": %d, \"n_bucket\": %d, \"k_bucket\": %d, \"tile\": %d, "
            "\"workgroups\": %d}%s\n",
            e.precision, e.n_bucket, e.k_bucket, e.cfg.tile, e.cfg.workgroups, i + 1 < es.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  return fclose(f) == 0 ? ILS_OK : ILS_ERR_ARG;
}

extern "C" int ils_tune_load(const char* path) {
  if (!path) return ILS_ERR_ARG;
  FILE* f = fopen(path, "r");
  if (!f) return ILS_ERR_ARG;
  char line[512];
  std::vector<GramCfgEntry> es;
  bool ok = fgets(line, sizeof(line), f) && strstr(line, "\"version\": 1");
  while (ok && fgets(line, sizeof(line), f)) {
    if (!strstr(line, "\"kernel\": \"gram\"")) continue;
    GramCfgEntry e;
    if (sscanf(line,
               " {\"kernel\": \"gram\", \"precision\": %d, \"n_bucket\": %d, \"k_bucket\": %d, \"tile\": %d, "
               "\"workgroups\": %d}",
               &e.precision, &e.n_bucket, &e.k_bucket, &e.cfg.tile, &e.cfg.workgroups) != 5 ||
        (e.precision != ILS_PREC_FP64 && e.precision != ILS_PREC_MIXED) || (e.cfg.tile != 64 && e.cfg.tile != 128) ||
        e.cfg.workgroups < 8 || e.cfg.workgroups > (1 << 20) || e.n_bucket < 0 || e.n_bucket > 40 ||
        e.k_bucket < 0 || e.k_bucket > 62) {
      ok = false;
      break;
    }
    es.push_back(e);
  }
  fclose(f);
  if (!ok) return ILS_ERR_ARG;
  for (const GramCfgEntry& e : es) gram_set_cfg_bucket(e.precision, e.n_bucket, e.k_bucket, e.cfg);
  return ILS_OK;
}
