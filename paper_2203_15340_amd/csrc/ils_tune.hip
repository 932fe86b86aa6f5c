// ils_tune.hip -- the autotuner: sweeps the Gram kernel's launch
// configurations (split-K: tile edge x workgroup target, hence the K-split;
// FP64 also the resident kernel with direct global-to-LDS loads) on the
// caller's matrix, keeps the fastest per (precision, log2 n, log2 K) bucket in
// the process-wide table that every Gram launch consults, and saves / loads
// that table as JSON.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ils_common.hpp"
#include "ils_runtime.hpp"
#include "k_batched.hpp"

namespace ils {
std::vector<GramCfgEntry> gram_cfg_entries();
int batched_solve(ils_handle* h, int64_t batch, const ils_problem* probs, const ils_opts* o, ils_info* infos,
                  const BatchCfg* force);

// ---- launch tables of the batched solver and of the residual
// key (kernel, precision, form, log2 bucket of n, log2 bucket of the size),
// value (tile, workgroups, kind) with the meanings of ils_tune_entry
typedef std::tuple<int, int, int, int, int> TabKey;
static std::mutex g_tab_mu;
static std::map<TabKey, std::array<int, 3>> g_tab;

static int bucket_of(int64_t x) {
  int b = 0;
  while (((int64_t)1 << b) < x) ++b;
  return b;
}

BatchCfg batched_cfg(int precision, int form, int64_t nmax, int64_t batch) {
  BatchCfg c;
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto it = g_tab.find(TabKey{ILS_TUNE_BATCHED, precision, form, bucket_of(nmax), bucket_of(batch)});
  if (it != g_tab.end()) {
    c.stage_rows = it->second[0];
    c.wpc = it->second[1];
    c.order = it->second[2];
  }
  return c;
}

ResidCfg residual_cfg(int64_t n, int64_t m) {
  ResidCfg c;
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto it = g_tab.find(TabKey{ILS_TUNE_RESIDUAL, ILS_PREC_FP64, 0, bucket_of(n), bucket_of(m)});
  if (it != g_tab.end()) {
    c.wgs = it->second[1];
    c.path = it->second[2];
  }
  return c;
}

static void tab_set(int kernel, int precision, int form, int nb, int kb, int tile, int wg, int kind) {
  std::lock_guard<std::mutex> lk(g_tab_mu);
  g_tab[TabKey{kernel, precision, form, nb, kb}] = {tile, wg, kind};
}

static bool batched_entry_ok(int precision, int form, int tile, int wg, int kind) {
  return (precision == ILS_PREC_FP64 || precision == ILS_PREC_MIXED) &&
         (form == ILS_FORM_PAPER || form == ILS_FORM_CORRECTION) && (tile == 16 || tile == 32 || tile == 64) &&
         (wg == 1 || wg == 2) && (kind == kBatchOrderLargest || kind == kBatchOrderGiven);
}
static bool residual_entry_ok(int tile, int wg, int kind) {
  return tile == 16 && wg >= 64 && wg <= 2048 && (kind == kResidAuto || kind == kResidTwoPass);
}
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
  std::vector<GramCfg> cands;
  for (int t : tiles)
    for (int w : targets) cands.push_back(GramCfg{t, w, kGramSplitK});
  cands.push_back(GramCfg{64, kGramPersistentWpc, kGramPersistent});  // FP32: from a copy of the rows
  size_t part_max = 0;
  for (const GramCfg& c : cands) part_max = std::max(part_max, gram_partials_size_cfg(n, K, c));
  double *G, *part;
  float* a1f = nullptr;
  int st;
  if ((st = h->need(kBufM, sizeof(double) * n * n, (void**)&G)) ||
      (st = h->need(kBufPart, sizeof(double) * part_max, (void**)&part)) ||
      (precision == ILS_PREC_MIXED &&
       (st = h->need(kBufA1f32, sizeof(float) * gram_f32_copy_ld(K) * n, (void**)&a1f))))
    return st;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  GramCfg win = gram_default_cfg(n);
  float win_ms = INFINITY;
  {
    for (const GramCfg& c : cands) {
      launch_gram_cfg(s, precision, K, n, A, lda, part, G, n, c, a1f);  // warm-up
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r) launch_gram_cfg(s, precision, K, n, A, lda, part, G, n, c, a1f);
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
    best->kind = win.kind;
    best->reserved = 0;
    best->ms = win_ms;
  }
  return ILS_OK;
}

extern "C" int ils_tune_batched(ils_handle* h, int64_t batch, const ils_problem* probs, const ils_opts* o,
                                int32_t reps, ils_tune_entry* best) {
  if (!h || !probs || !o || batch < 1 || reps < 1 || reps > 1000) return ILS_ERR_ARG;
  std::vector<ils_info> infos(batch);
  int64_t nmax = 1;
  for (int64_t i = 0; i < batch; ++i) nmax = std::max(nmax, probs[i].n);
  BatchCfg win;
  double win_ms = INFINITY;
  int ref_rc = 0;
  bool first = true;
  for (int sr : {16, 32, 64})
    for (int wpc : {1, 2})
      for (int ord : {kBatchOrderLargest, kBatchOrderGiven}) {
        BatchCfg c;
        c.stage_rows = sr;
        c.wpc = wpc;
        c.order = ord;
        int rc = batched_solve(h, batch, probs, o, infos.data(), &c);  // warm-up (graph capture)
        if (rc == ILS_ERR_ARG || rc == ILS_ERR_HIP || rc == ILS_ERR_ALLOC) return rc;
        if (first) {
          ref_rc = rc;
          first = false;
        } else if (rc != ref_rc) {
          return ILS_ERR_HIP;  // the launch choice changed an outcome: never expected
        }
        double ms = 0.0;
        for (int r = 0; r < reps; ++r) {
          rc = batched_solve(h, batch, probs, o, infos.data(), &c);
          if (rc != ref_rc) return rc == ILS_OK ? ILS_ERR_HIP : rc;
          ms += infos[0].device_ms;
        }
        ms /= reps;
        if (ms < win_ms) {
          win_ms = ms;
          win = c;
        }
      }
  tab_set(ILS_TUNE_BATCHED, o->precision, o->form, bucket_of(nmax), bucket_of(batch), win.stage_rows, win.wpc,
          win.order);
  if (best) {
    best->kernel = ILS_TUNE_BATCHED;
    best->precision = o->precision;
    best->n = nmax;
    best->K = batch;
    best->tile = win.stage_rows;
    best->workgroups = win.wpc;
    best->ms = win_ms;
    best->kind = win.order;
    best->reserved = o->form;
  }
  return ILS_OK;
}

extern "C" int ils_tune_residual(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                                 const double* b, const double* x, int32_t reps, ils_tune_entry* best) {
  if (!h || !A || !b || !x || n < 1 || p < 0 || q < 0 || p + q < 1 || lda < p + q || reps < 1 || reps > 1000)
    return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  hipStream_t s = h->stream;
  const int64_t m = p + q;
  std::vector<ResidCfg> cands;
  for (int wg : {128, 256, 512, 1024}) cands.push_back(ResidCfg{kResidAuto, wg});
  cands.push_back(ResidCfg{kResidTwoPass, kResidDefaultWgs});
  size_t scr = 0;
  for (const ResidCfg& c : cands) scr = std::max(scr, residual_scratch_cfg(m, n, c));
  double *t, *r;
  int st;
  if ((st = h->need(kBufT, sizeof(double) * scr, (void**)&t)) ||
      (st = h->need(kBufR, sizeof(double) * n, (void**)&r)))
    return st;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  ResidCfg win;
  float win_ms = INFINITY;
  for (const ResidCfg& c : cands) {
    if (c.path == kResidAuto && n > 1024 && c.wgs != kResidDefaultWgs) continue;  // one pass needs n <= 1024
    launch_residual_cfg(s, p, q, n, A, lda, b, x, t, r, nullptr, c);
    (void)hipEventRecord(e0, s);
    for (int k = 0; k < reps; ++k) launch_residual_cfg(s, p, q, n, A, lda, b, x, t, r, nullptr, c);
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
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipGetLastError());
  tab_set(ILS_TUNE_RESIDUAL, ILS_PREC_FP64, 0, bucket_of(n), bucket_of(m), 16, win.wgs, win.path);
  if (best) {
    best->kernel = ILS_TUNE_RESIDUAL;
    best->precision = ILS_PREC_FP64;
    best->n = n;
    best->K = m;
    best->tile = 16;
    best->workgroups = win.wgs;
    best->ms = win_ms;
    best->kind = win.path;
    best->reserved = 0;
  }
  return ILS_OK;
}

extern "C" int ils_tune_clear(void) {
  gram_clear_cfg();
  std::lock_guard<std::mutex> lk(g_tab_mu);
  g_tab.clear();
  return ILS_OK;
}

// One entry per line so that ils_tune_load can read the file back with a
// line scanner; the whole file is ordinary JSON.
extern "C" int ils_tune_save(const char* path) {
  if (!path) return ILS_ERR_ARG;
  FILE* f = fopen(path, "w");
  if (!f) return ILS_ERR_ARG;
  const std::vector<GramCfgEntry> es = gram_cfg_entries();
  std::vector<std::pair<TabKey, std::array<int, 3>>> tab;
  {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    tab.assign(g_tab.begin(), g_tab.end());
  }
  const size_t total = es.size() + tab.size();
  size_t done = 0;
  fprintf(f, "{\"version\": 1, \"entries\": [\n");
  for (size_t i = 0; i < es.size(); ++i) {
    const GramCfgEntry& e = es[i];
    ++done;
    fprintf(f,
            "  {\"kernel\": \"gram\", \"precision\": %d, \"n_bucket\": %d, \"k_bucket\": %d, \"tile\": %d, "
            "\"workgroups\": %d, \"kind\": %d}%s\n",
            e.precision, e.n_bucket, e.k_bucket, e.cfg.tile, e.cfg.workgroups, e.cfg.kind,
            done < total ? "," : "");
  }
  for (const auto& kv : tab) {
    const int kernel = std::get<0>(kv.first);
    ++done;
    fprintf(f,
            "  {\"kernel\": \"%s\", \"precision\": %d, \"form\": %d, \"n_bucket\": %d, \"k_bucket\": %d, "
            "\"tile\": %d, \"workgroups\": %d, \"kind\": %d}%s\n",
            kernel == ILS_TUNE_BATCHED ? "batched" : "residual", std::get<1>(kv.first), std::get<2>(kv.first),
            std::get<3>(kv.first), std::get<4>(kv.first), kv.second[0], kv.second[1], kv.second[2],
            done < total ? "," : "");
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
  std::vector<std::pair<TabKey, std::array<int, 3>>> tab;
  bool ok = fgets(line, sizeof(line), f) && strstr(line, "\"version\": 1");
  while (ok && fgets(line, sizeof(line), f)) {
    const bool bat = strstr(line, "\"kernel\": \"batched\"") != nullptr;
    if (bat || strstr(line, "\"kernel\": \"residual\"")) {
      int pr, fm, nb, kb, tile, wg, kind;
      const int got = sscanf(line,
                             bat ? " {\"kernel\": \"batched\", \"precision\": %d, \"form\": %d, \"n_bucket\": %d, "
                                   "\"k_bucket\": %d, \"tile\": %d, \"workgroups\": %d, \"kind\": %d}"
                                 : " {\"kernel\": \"residual\", \"precision\": %d, \"form\": %d, \"n_bucket\": %d, "
                                   "\"k_bucket\": %d, \"tile\": %d, \"workgroups\": %d, \"kind\": %d}",
                             &pr, &fm, &nb, &kb, &tile, &wg, &kind);
      const bool good = got == 7 && nb >= 0 && nb <= 40 && kb >= 0 && kb <= 62 &&
                        (bat ? batched_entry_ok(pr, fm, tile, wg, kind)
                             : (pr == ILS_PREC_FP64 && fm == 0 && residual_entry_ok(tile, wg, kind)));
      if (!good) {
        ok = false;
        break;
      }
      tab.push_back({TabKey{bat ? ILS_TUNE_BATCHED : ILS_TUNE_RESIDUAL, pr, fm, nb, kb}, {tile, wg, kind}});
      continue;
    }
    if (!strstr(line, "\"kernel\": \"gram\"")) continue;
    GramCfgEntry e;
    e.cfg.kind = kGramSplitK;
    // "kind" is optional (absent: split-K)
    const int got = sscanf(line,
                           " {\"kernel\": \"gram\", \"precision\": %d, \"n_bucket\": %d, \"k_bucket\": %d, "
                           "\"tile\": %d, \"workgroups\": %d, \"kind\": %d}",
                           &e.precision, &e.n_bucket, &e.k_bucket, &e.cfg.tile, &e.cfg.workgroups, &e.cfg.kind);
    const bool kind_ok = e.cfg.kind == kGramSplitK
                             ? ((e.cfg.tile == 64 || e.cfg.tile == 128) && e.cfg.workgroups >= 8 &&
                                e.cfg.workgroups <= (1 << 20))
                             : (e.cfg.kind == kGramPersistent && e.cfg.tile == 64 &&
                                e.cfg.workgroups == kGramPersistentWpc);
    if (got < 5 || !kind_ok || (e.precision != ILS_PREC_FP64 && e.precision != ILS_PREC_MIXED) ||
        e.n_bucket < 0 || e.n_bucket > 40 || e.k_bucket < 0 || e.k_bucket > 62) {
      ok = false;
      break;
    }
    es.push_back(e);
  }
  fclose(f);
  if (!ok) return ILS_ERR_ARG;
  for (const GramCfgEntry& e : es) gram_set_cfg_bucket(e.precision, e.n_bucket, e.k_bucket, e.cfg);
  for (const auto& kv : tab)
    tab_set(std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
            std::get<4>(kv.first), kv.second[0], kv.second[1], kv.second[2]);
  return ILS_OK;
}
