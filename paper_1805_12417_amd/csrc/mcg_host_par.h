// Host-side parallel loops for the setup code (factor copies, transposes,
// block and sliced layouts): contiguous chunks of an index range on up to 16
// threads.  Every caller writes disjoint outputs per index, so results do not
// depend on the thread count.
#pragma once
#include <algorithm>
#include <cstdint>
#include <thread>
#include <vector>

inline int mcg_host_threads() {
  const unsigned h = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(h ? h : 1u, 16u));
}

// f(lo, hi) on [0, n) cut into nt contiguous chunks (nt <= 0: mcg_host_threads;
// ranges below `grain` indices per thread use fewer threads).
template <typename F>
void mcg_parallel_chunks(int64_t n, F f, int nt = 0, int64_t grain = 1 << 14) {
  if (nt <= 0) nt = mcg_host_threads();
  nt = (int)std::max<int64_t>(1, std::min<int64_t>(nt, (n + grain - 1) / grain));
  if (nt == 1) {
    f((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  for (int t = 1; t < nt; ++t)
    th.emplace_back([&f, n, nt, t] { f(n * t / nt, n * (t + 1) / nt); });
  f((int64_t)0, n / nt);
  for (auto &x : th) x.join();
}

// As mcg_parallel_chunks, with the chunk's index: f(t, lo, hi), t < nt.  A
// chunk index runs on one thread at a time, so per-index scratch reused
// across calls needs no locking.
template <typename F>
void mcg_parallel_chunks_t(int64_t n, int nt, F f, int64_t grain = 1 << 14) {
  const int used = (int)std::max<int64_t>(1, std::min<int64_t>(nt, (n + grain - 1) / grain));
  if (used == 1) {
    f(0, (int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(used - 1);
  for (int t = 1; t < used; ++t)
    th.emplace_back([&f, n, used, t] { f(t, n * t / used, n * (t + 1) / used); });
  f(0, (int64_t)0, n / used);
  for (auto &x : th) x.join();
}

// CSR transpose (n x n), rows of the result in increasing column order of the
// input rows (the order a sequential scatter over the input rows gives):
// per-thread column counts over row chunks balanced by entries, per (column,
// chunk) cursors, then each chunk scatters its rows in order.
inline void mcg_csr_transpose_par(int n, const std::vector<int32_t> &rp,
                                  const std::vector<int32_t> &ci, const std::vector<double> &v,
                                  std::vector<int32_t> &trp, std::vector<int32_t> &tci,
                                  std::vector<double> &tv) {
  const int64_t nnz = rp[n];
  const int nt = nnz < (1 << 20) ? 1 : mcg_host_threads();
  // row chunk boundaries with about nnz / nt entries each
  std::vector<int> r0(nt + 1, n);
  r0[0] = 0;
  for (int t = 1; t < nt; ++t)
    r0[t] = (int)(std::lower_bound(rp.begin(), rp.end(), (int32_t)(nnz * t / nt)) - rp.begin());
  for (int t = 1; t <= nt; ++t) r0[t] = std::max(r0[t], r0[t - 1]);
  std::vector<std::vector<int32_t>> cnt(nt);
  mcg_parallel_chunks(nt, [&](int64_t lo, int64_t hi) {
    for (int64_t t = lo; t < hi; ++t) {
      cnt[t].assign(n, 0);
      for (int64_t p = rp[r0[t]]; p < rp[r0[t + 1]]; ++p) cnt[t][ci[p]]++;
    }
  }, nt, 1);
  trp.assign(n + 1, 0);
  mcg_parallel_chunks(n, [&](int64_t lo, int64_t hi) {
    for (int64_t c = lo; c < hi; ++c) {
      int32_t s = 0;
      for (int t = 0; t < nt; ++t) s += cnt[t][c];
      trp[c + 1] = s;
    }
  });
  for (int i = 0; i < n; ++i) trp[i + 1] += trp[i];
  mcg_parallel_chunks(n, [&](int64_t lo, int64_t hi) {  // cursors: chunk t after chunks < t
    for (int64_t c = lo; c < hi; ++c) {
      int32_t at = trp[c];
      for (int t = 0; t < nt; ++t) {
        const int32_t k = cnt[t][c];
        cnt[t][c] = at;
        at += k;
      }
    }
  });
  tci.resize(nnz);
  tv.resize(nnz);
  mcg_parallel_chunks(nt, [&](int64_t lo, int64_t hi) {
    for (int64_t t = lo; t < hi; ++t)
      for (int i = r0[t]; i < r0[t + 1]; ++i)
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
          const int32_t q = cnt[t][ci[p]]++;
          tci[q] = i;
          tv[q] = v[p];
        }
  }, nt, 1);
}
