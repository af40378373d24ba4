// SpMV lanes-per-row autotuner.
//
// The CSR kernels give L lanes to each row (vector CSR inside 256-row tiles),
// or (L = 1) stage a whole tile's nonzeros through LDS (CSR-stream).  The
// best choice depends on the row-length distribution and the value type: too
// few lanes serialise long rows, too many leave lanes idle on short ones.  At
// create (opt.autotune = 1) every L in {1, 2, 4, ..., 64} is timed on this
// matrix with HIP events (FP64 and, in mixed precision, the FP32 shadow that
// the inner solve uses) and the fastest kept.  Results can be cached in a
// small JSON file named by the environment variable MCG_TUNE_CACHE, keyed by
// n, nnz, the row-length quantiles and the precision, so repeated creates of
// the same matrix shape skip the timing.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "mcg_internal.h"

namespace {

std::string signature(const mcg_solver *h) {
  std::vector<int32_t> len(h->n);
  for (int i = 0; i < h->n; ++i) len[i] = h->h_rp[i + 1] - h->h_rp[i];
  std::sort(len.begin(), len.end());
  auto q = [&](double f) { return len.empty() ? 0 : len[(size_t)(f * (len.size() - 1))]; };
  char buf[160];
  std::snprintf(buf, sizeof buf, "n%d_nnz%lld_q%d-%d-%d-%d-%d_p%d", h->n, (long long)h->nnz, q(0.0),
                q(0.25), q(0.5), q(0.75), q(1.0), h->opt.precision);
  return buf;
}

int cache_lookup(const char *path, const std::string &key) {
  FILE *f = std::fopen(path, "r");
  if (!f) return 0;
  char line[512];
  int found = 0;
  while (std::fgets(line, sizeof line, f)) {
    // one entry per line: "<key>": <lanes>,
    const char *k = std::strstr(line, key.c_str());
    if (k && k[-1] == '"' && k[key.size()] == '"') {
      const char *colon = std::strchr(k + key.size(), ':');
      if (colon) found = std::atoi(colon + 1);
    }
  }
  std::fclose(f);
  return (found >= 1 && found <= 64 && (found & (found - 1)) == 0) ? found : 0;
}

void cache_store(const char *path, const std::string &key, int lanes) {
  std::vector<std::string> lines;
  if (FILE *f = std::fopen(path, "r")) {
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
      std::string s(line);
      if (s.find('"') != std::string::npos && s.find("\"" + key + "\"") == std::string::npos)
        lines.push_back(s.substr(0, s.find_last_not_of(",\n") + 1));
    }
    std::fclose(f);
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "  \"%s\": %d", key.c_str(), lanes);
  lines.push_back(buf);
  FILE *f = std::fopen(path, "w");
  if (!f) return;
  std::fputs("{\n", f);
  for (size_t i = 0; i < lines.size(); ++i) {
    std::string s = lines[i];
    size_t a = s.find_first_not_of(" {");
    if (a == std::string::npos) continue;
    std::fprintf(f, "  %s%s\n", s.substr(a).c_str(), i + 1 < lines.size() ? "," : "");
  }
  std::fputs("}\n", f);
  std::fclose(f);
}

template <typename T>
float time_lanes(mcg_solver *h, int L, const T *x, T *y, hipStream_t s, hipEvent_t e0,
                 hipEvent_t e1) {
  h->lanes = L;
  mcg_launch_spmv_csr<T>(h, x, y, s);  // warm-up
  (void)hipEventRecord(e0, s);
  const int reps = 5;
  for (int r = 0; r < reps; ++r) mcg_launch_spmv_csr<T>(h, x, y, s);
  (void)hipEventRecord(e1, s);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  return ms / reps;
}

// the iteration's M_mr apply with a scratch DevState (done = 0); dinv = ones
template <typename T>
float time_mmr(mcg_solver *h, const T *x, T *y, const T *dinv, hipStream_t s, hipEvent_t e0,
               hipEvent_t e1) {
  mcg_launch_mmr_diag<T>(h, x, y, dinv, h->Saux, s);
  (void)hipEventRecord(e0, s);
  const int reps = 5;
  for (int r = 0; r < reps; ++r) mcg_launch_mmr_diag<T>(h, x, y, dinv, h->Saux, s);
  (void)hipEventRecord(e1, s);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  return ms / reps;
}

}  // namespace

int mcg_autotune_lanes(mcg_solver *h, hipStream_t s) {
  const char *path = std::getenv("MCG_TUNE_CACHE");
  const std::string key = signature(h);
  if (path && *path) {
    const int L = cache_lookup(path, key);
    if (L) {
      h->lanes = L;
      return MCG_OK;
    }
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return MCG_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return MCG_EHIP; }
  // inputs: the workspace vectors (contents irrelevant for timing, but finite)
  const bool mixed = h->opt.precision == MCG_PREC_MIXED;
  k_fill<double><<<256, 256, 0, s>>>(h->n, 1.0, h->r1);
  k_fill<double><<<256, 256, 0, s>>>(h->n, 1.0, h->y);
  if (mixed) {
    k_fill<float><<<256, 256, 0, s>>>(h->n, 1.0f, (float *)h->r);
    k_fill<float><<<256, 256, 0, s>>>(h->n, 1.0f, (float *)h->z);
  }
  int best = h->lanes;
  float best_t = 1e30f;
  for (int L = 1; L <= 64; L *= 2) {  // 1 = CSR-stream tiles
    float t = time_lanes<double>(h, L, h->r1, h->r2, s, e0, e1);
    if (mixed) t += 2.f * time_lanes<float>(h, L, (const float *)h->r, (float *)h->q, s, e0, e1);
    if (t < best_t) {
      best_t = t;
      best = L;
    }
  }
  h->lanes = best;
  // fused vs split M_mr apply of the Jacobi iteration, in the inner precision
  // (with a sliced copy the iteration uses the SpMV + folded-update pair and
  // the fused/split choice does not arise)
  if (h->k > 0 && h->opt.mmr_form == 0 && !h->bsr_bs && !h->sa.bits) {
    float tf = 0.f, tsp = 0.f;
    for (int split = 0; split < 2; ++split) {
      h->mmr_split = split;
      const float t = mixed ? time_mmr<float>(h, (const float *)h->r, (float *)h->q,
                                              (const float *)h->z, s, e0, e1)
                            : time_mmr<double>(h, h->r1, h->r2, h->y, s, e0, e1);
      (split ? tsp : tf) = t;
    }
    h->mmr_split = tsp < tf ? 1 : 0;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (hipGetLastError() != hipSuccess) return MCG_EHIP;
  if (path && *path) cache_store(path, key, best);
  return MCG_OK;
}

extern "C" int minres_cg_spmv_lanes(mcg_handle_t h) { return h ? h->lanes : 0; }

extern "C" int minres_cg_mmr_split(mcg_handle_t h) { return h ? h->mmr_split : -1; }

extern "C" int minres_cg_block_csr(mcg_handle_t h) { return h ? h->bsr_bs : -1; }

extern "C" int minres_cg_sliced_ell(mcg_handle_t h) { return h ? h->sa.bits : -1; }

extern "C" int minres_cg_sliced_blocks(mcg_handle_t h) { return h ? h->bsa.bs : -1; }

extern "C" int minres_cg_xcd_sections(mcg_handle_t h) {
  if (!h || !h->bsa.bs) return -1;
  return h->bsa.xmap_sections < 0 ? 0 : h->bsa.xmap_sections;
}
