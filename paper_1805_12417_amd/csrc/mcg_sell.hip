// Sliced ELL copies of sparse matrices (A, and the learned factor C and its
// transpose): host-side construction at setup, and the SpMV launcher.  The
// layout and the kernels are described at k_sell_spmv (mcg_kernels.h).
#include <hip/hip_runtime.h>

#include <atomic>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "mcg_host_par.h"
#include "mcg_internal.h"

void mcg_sell_free(mcg_sell *S) {
  void *b[] = {S->off, S->col, S->v, S->v32, S->v16};
  for (void *x : b)
    if (x) (void)hipFree(x);
  *S = mcg_sell{};
}

int mcg_sell_build(mcg_sell *S, int n, const std::vector<int32_t> &rp,
                   const std::vector<int32_t> &ci, const double *v, bool narrow_ok,
                   double max_pad, bool fp32, hipStream_t s, bool fp16) {
  *S = mcg_sell{};
  const int64_t nnz = rp[n];
  if (n == 0 || nnz == 0) return MCG_OK;
  const int ns = (n + 63) / 64;
  std::vector<int64_t> off(ns + 1, 0);
  for (int sl = 0; sl < ns; ++sl) {
    int w = 0;
    for (int r = sl * 64; r < std::min(n, sl * 64 + 64); ++r) w = std::max(w, rp[r + 1] - rp[r]);
    w = std::max(w, 1);  // every slice has a slot, so the kernels' clamped loads stay inside it
    off[sl + 1] = off[sl] + 64 * (int64_t)w;
  }
  const int64_t P = off[ns];
  if (max_pad >= 0.0 && (double)P > (1.0 + max_pad) * (double)nnz) return MCG_OK;
  int maxw = 0;
  for (int sl = 0; sl < ns; ++sl) maxw = std::max(maxw, (int)((off[sl + 1] - off[sl]) / 64));
  bool narrow = narrow_ok;
  for (int r = 0; r < n && narrow; ++r)
    for (int e = rp[r]; e < rp[r + 1]; ++e)
      if (ci[e] - r > 32767 || ci[e] - r < -32768) {
        narrow = false;
        break;
      }
  std::vector<double> sv((size_t)P);
  std::vector<int32_t> c32;
  std::vector<int16_t> c16;
  if (narrow)
    c16.resize((size_t)P);
  else
    c32.resize((size_t)P);
  mcg_parallel_chunks(ns, [&](int64_t s0, int64_t s1) {  // slices are independent
    for (int64_t sl = s0; sl < s1; ++sl) {
      const int w = (int)((off[sl + 1] - off[sl]) / 64);
      for (int l = 0; l < 64; ++l) {
        const int r = (int)sl * 64 + l;
        const int len = r < n ? rp[r + 1] - rp[r] : 0;
        const int pad_col = r < n ? r : n - 1;  // padding stays inside the matrix
        for (int j = 0; j < w; ++j) {
          const size_t e = (size_t)(off[sl] + 64 * (int64_t)j + l);
          const int c = j < len ? ci[rp[r] + j] : pad_col;
          sv[e] = j < len ? v[rp[r] + j] : 0.0;
          if (narrow)
            c16[e] = (int16_t)(c - r);
          else
            c32[e] = c;
        }
      }
    }
  }, 0, 256);
  mcg_sell T;
  T.n = n;
  T.nslices = ns;
  T.maxw = maxw;
  T.bits = narrow ? 16 : 32;
  const size_t cb = narrow ? sizeof(int16_t) : sizeof(int32_t);
  auto fail = [&](hipError_t e) {
    mcg_last_hip_error = e;
    mcg_sell_free(&T);
    return e == hipErrorOutOfMemory ? MCG_ENOMEM : MCG_EHIP;
  };
  hipError_t e;
  if ((e = hipMalloc((void **)&T.off, sizeof(int64_t) * (ns + 1))) != hipSuccess ||
      (e = hipMalloc(&T.col, cb * P)) != hipSuccess ||
      (e = hipMalloc((void **)&T.v, sizeof(double) * P)) != hipSuccess ||
      (fp32 && (e = hipMalloc((void **)&T.v32, sizeof(float) * P)) != hipSuccess))
    return fail(e);
  if ((e = hipMemcpy(T.off, off.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(T.col, narrow ? (const void *)c16.data() : (const void *)c32.data(), cb * P,
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(T.v, sv.data(), sizeof(double) * P, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e);
  if (fp32) {
    k_convert<float, double><<<2048, 256, 0, s>>>(P, T.v, T.v32);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
  }
  if (fp32 && fp16) {
    // no value overflows, and every diagonal value stays a normal FP16 number
    // (off-diagonal values may round to subnormals or zero: a lower
    // triangular factor then still has its positive diagonal)
    bool in_range = true;
    for (int r = 0; r < n && in_range; ++r)
      for (int q = rp[r]; q < rp[r + 1]; ++q) {
        const double a = std::fabs(v[q]);
        if (!(a <= 65504.0) || (ci[q] == r && a < 6.103515625e-05)) {
          in_range = false;
          break;
        }
      }
    if (in_range) {
      if ((e = hipMalloc((void **)&T.v16, sizeof(_Float16) * P)) != hipSuccess) return fail(e);
      k_convert<_Float16, double><<<2048, 256, 0, s>>>(P, T.v, T.v16);
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
    }
  }
  *S = T;
  return MCG_OK;
}

template <typename T>
void mcg_sell_spmv(const mcg_sell &A, const T *x, T *y, const DevState *St, hipStream_t s) {
  // two slices per wavefront, grid-stride over at most 2048 blocks (measured
  // faster than one block per slice pair on the 128^3 stencil)
  const int g = std::max(1, std::min((A.nslices + 2 * MCG_NWAVE - 1) / (2 * MCG_NWAVE), 2048));
  if constexpr (sizeof(T) == 4) {
    if (A.v16) {  // FP16 values, FP32 arithmetic
      const _Float16 *h = A.v16;
      if (A.bits == 16) {
        const int16_t *c = (const int16_t *)A.col;
        if (A.maxw <= 4)
          k_sell_spmv<T, int16_t, 4, _Float16><<<g, MCG_BLOCK, 0, s>>>(A.n, A.nslices, A.off, c, h,
                                                                       x, y, St);
        else
          k_sell_spmv<T, int16_t, 8, _Float16><<<g, MCG_BLOCK, 0, s>>>(A.n, A.nslices, A.off, c, h,
                                                                       x, y, St);
      } else {
        const int32_t *c = (const int32_t *)A.col;
        if (A.maxw <= 4)
          k_sell_spmv<T, int32_t, 4, _Float16><<<g, MCG_BLOCK, 0, s>>>(A.n, A.nslices, A.off, c, h,
                                                                       x, y, St);
        else
          k_sell_spmv<T, int32_t, 8, _Float16><<<g, MCG_BLOCK, 0, s>>>(A.n, A.nslices, A.off, c, h,
                                                                       x, y, St);
      }
      return;
    }
  }
  const T *v = mcg_sell_vals<T>(A);
  if (A.bits == 16) {
    const int16_t *c = (const int16_t *)A.col;
    if (A.maxw <= 4)
      k_sell_spmv<T, int16_t, 4><<<g, MCG_BLOCK, 0, s>>>(A.n, A.nslices, A.off, c, v, x, y, St);
    else
      k_sell_spmv<T, int16_t, 8><<<g, MCG_BLOCK, 0, s>>>(A.n, A.nslices, A.off, c, v, x, y, St);
  } else {
    const int32_t *c = (const int32_t *)A.col;
    if (A.maxw <= 4)
      k_sell_spmv<T, int32_t, 4><<<g, MCG_BLOCK, 0, s>>>(A.n, A.nslices, A.off, c, v, x, y, St);
    else
      k_sell_spmv<T, int32_t, 8><<<g, MCG_BLOCK, 0, s>>>(A.n, A.nslices, A.off, c, v, x, y, St);
  }
}
template void mcg_sell_spmv<double>(const mcg_sell &, const double *, double *, const DevState *,
                                    hipStream_t);
template void mcg_sell_spmv<float>(const mcg_sell &, const float *, float *, const DevState *,
                                   hipStream_t);

// ---------------------------------------------------------------------------
// sliced block ELL
// ---------------------------------------------------------------------------
void mcg_bsell_free(mcg_bsell *S) {
  void *b[] = {S->off, S->col, S->v, S->v32, S->v16, S->xmap};
  for (void *x : b)
    if (x) (void)hipFree(x);
  *S = mcg_bsell{};
}

// Slice order for the XCDs.  A launch's workgroup b runs on XCD b % 8, each
// XCD with its own L2; in the launch's own order (workgroup b takes slices
// 4b..4b+3) every XCD's slices are spread over the whole matrix, and so are
// the entries of x they gather.  Candidates: that order, and for P = 1, 2, 4,
// 8, 16 equal sections of the slices, XCD e taking the e-th eighth of every
// section (P = 1 suits a banded order; P = 8 a matrix in 8 colour sections,
// where a node's neighbours lie at the same place of the other sections).
// Each is scored by the x lines of 128 bytes (FP32) its XCDs touch, summed
// over the XCDs; the lowest wins, the launch's own order on a tie within 2 %.
// mode 0 asks for a section order only when x (FP32) is larger than one
// XCD's 4 MB L2: a smaller x stays in every L2 in any order, and there the
// section orders measured slower (FE-like 40^3 nodes x 3: +16 % per solve);
// mode 1: never; mode 2: at any size.  Returns the map (9 section bounds,
// then the slices) or empty for none.
static std::vector<int32_t> xcd_slice_map(int ns, int nbr, int bs, const std::vector<int64_t> &off,
                                          const std::vector<int32_t> &c, int mode, int *chosen) {
  *chosen = -1;
  constexpr int64_t kXcdL2Bytes = 4 << 20;
  if (ns < 64 || mode == 1 || (mode == 0 && (int64_t)nbr * bs * 4 <= kXcdL2Bytes)) return {};
  const int64_t nlines = ((int64_t)nbr * bs * 4 + 127) / 128;
  auto slices_of = [&](int P, int e, std::vector<int32_t> &out) {
    out.clear();
    if (P == 0) {
      for (int sl = 0; sl < ns; ++sl)
        if ((sl / MCG_NWAVE) % 8 == e) out.push_back(sl);
      return;
    }
    for (int q = 0; q < P; ++q) {
      const int64_t lo = (int64_t)ns * q / P, hi = (int64_t)ns * (q + 1) / P;
      for (int64_t sl = lo + (hi - lo) * e / 8; sl < lo + (hi - lo) * (e + 1) / 8; ++sl)
        out.push_back((int32_t)sl);
    }
  };
  const int cand[] = {0, 1, 2, 4, 8, 16};
  const int nc = (int)(sizeof(cand) / sizeof(cand[0]));
  std::vector<int64_t> score((size_t)nc * 8, 0);
  mcg_parallel_chunks((int64_t)nc * 8, [&](int64_t lo, int64_t hi) {
    std::vector<uint8_t> seen((size_t)nlines);
    std::vector<int32_t> sl;
    for (int64_t t = lo; t < hi; ++t) {
      slices_of(cand[t / 8], (int)(t % 8), sl);
      std::fill(seen.begin(), seen.end(), 0);
      int64_t cnt = 0;
      for (int32_t x : sl)
        for (int64_t e = off[x]; e < off[x + 1]; ++e) {
          const int64_t line = (int64_t)c[e] * bs * 4 / 128;
          cnt += !seen[line];
          seen[line] = 1;
        }
      score[t] = cnt;
    }
  }, 0, 1);
  int best = 0;
  int64_t tot[sizeof(cand) / sizeof(cand[0])];
  for (int i = 0; i < nc; ++i) {
    tot[i] = 0;
    for (int e = 0; e < 8; ++e) tot[i] += score[(size_t)i * 8 + e];
    if (tot[i] < tot[best]) best = i;
  }
  if (best == 0 || (double)tot[best] > 0.98 * (double)tot[0]) return {};
  *chosen = cand[best];
  std::vector<int32_t> map(9, 0), sl;
  for (int e = 0; e < 8; ++e) {
    slices_of(cand[best], e, sl);
    map.insert(map.end(), sl.begin(), sl.end());
    map[e + 1] = map[e] + (int32_t)sl.size();
  }
  return map;
}

int mcg_bsell_build(mcg_bsell *S, int bs, int nbr, const std::vector<int32_t> &brp,
                    const std::vector<int32_t> &bci, const std::vector<double> &bv,
                    double max_pad, bool fp32, hipStream_t s, bool fp16, int xcd_order) {
  *S = mcg_bsell{};
  const int64_t nb = brp[nbr];
  if (nbr == 0 || nb == 0 || bs < 2 || bs > 4) return MCG_OK;
  const int BB = bs * bs;
  const int ns = (nbr + 63) / 64;
  std::vector<int64_t> off(ns + 1, 0);
  for (int sl = 0; sl < ns; ++sl) {
    int w = 1;  // every slice has a slot, so the clamped loads stay inside it
    for (int I = sl * 64; I < std::min(nbr, sl * 64 + 64); ++I) w = std::max(w, brp[I + 1] - brp[I]);
    off[sl + 1] = off[sl] + 64 * (int64_t)w;
  }
  const int64_t P = off[ns];  // padded blocks
  if ((double)P > (1.0 + max_pad) * (double)nb) return MCG_OK;
  std::vector<int32_t> c((size_t)P);
  std::vector<double> v((size_t)P * BB, 0.0);
  mcg_parallel_chunks(ns, [&](int64_t s0, int64_t s1) {  // slices are independent
    for (int64_t sl = s0; sl < s1; ++sl) {
      const int w = (int)((off[sl + 1] - off[sl]) / 64);
      for (int l = 0; l < 64; ++l) {
        const int I = (int)sl * 64 + l;
        const int len = I < nbr ? brp[I + 1] - brp[I] : 0;
        for (int j = 0; j < w; ++j) {
          const size_t e = (size_t)(off[sl] + 64 * (int64_t)j + l);
          c[e] = j < len ? bci[brp[I] + j] : std::min(I, nbr - 1);
          if (j < len) {
            const size_t src = (size_t)(brp[I] + j) * BB;
            const size_t dst = (size_t)(off[sl] + 64 * (int64_t)j) * BB + l;
            for (int q = 0; q < BB; ++q) v[dst + (size_t)q * 64] = bv[src + q];
          }
        }
      }
    }
  }, 0, 256);
  mcg_bsell T;
  T.bs = bs;
  T.nbr = nbr;
  T.nslices = ns;
  auto fail = [&](hipError_t e) {
    mcg_last_hip_error = e;
    mcg_bsell_free(&T);
    return e == hipErrorOutOfMemory ? MCG_ENOMEM : MCG_EHIP;
  };
  hipError_t e;
  if ((e = hipMalloc((void **)&T.off, sizeof(int64_t) * (ns + 1))) != hipSuccess ||
      (e = hipMalloc((void **)&T.col, sizeof(int32_t) * P)) != hipSuccess ||
      (e = hipMalloc((void **)&T.v, sizeof(double) * P * BB)) != hipSuccess ||
      (fp32 && (e = hipMalloc((void **)&T.v32, sizeof(float) * P * BB)) != hipSuccess))
    return fail(e);
  if ((e = hipMemcpy(T.off, off.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(T.col, c.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(T.v, v.data(), sizeof(double) * P * BB, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e);
  if (fp32) {
    k_convert<float, double><<<2048, 256, 0, s>>>(P * BB, T.v, T.v32);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
  }
  {
    const std::vector<int32_t> map = xcd_slice_map(ns, nbr, bs, off, c, xcd_order,
                                                   &T.xmap_sections);
    if (!map.empty()) {
      if ((e = hipMalloc((void **)&T.xmap, sizeof(int32_t) * map.size())) != hipSuccess ||
          (e = hipMemcpy(T.xmap, map.data(), sizeof(int32_t) * map.size(),
                         hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    }
  }
  if (fp32 && fp16) {  // the rule of mcg_sell_build, at block granularity
    std::atomic<int> out_of_range{0};
    mcg_parallel_chunks(nbr, [&](int64_t lo, int64_t hi) {
      for (int64_t I = lo; I < hi; ++I)
        for (int q = brp[I]; q < brp[I + 1]; ++q)
          for (int ab = 0; ab < BB; ++ab) {
            const double a = std::fabs(bv[(size_t)q * BB + ab]);
            const bool diag = bci[q] == I && ab / bs == ab % bs;
            if (!(a <= 65504.0) || (diag && a < 6.103515625e-05)) {
              out_of_range.store(1, std::memory_order_relaxed);
              return;
            }
          }
    });
    const bool in_range = out_of_range.load() == 0;
    if (in_range) {
      if ((e = hipMalloc((void **)&T.v16, sizeof(_Float16) * P * BB)) != hipSuccess) return fail(e);
      k_convert<_Float16, double><<<2048, 256, 0, s>>>(P * BB, T.v, T.v16);
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
    }
  }
  *S = T;
  return MCG_OK;
}

template <typename T>
int mcg_bsell_spmv(const mcg_bsell &A, const T *x, T *y, DevState *St, hipStream_t s, bool dot,
                   const T *r, double *part, double *compact, const double *part_in, int nb_in,
                   int k, int max_grid) {
  const int g = std::max(1, std::min((A.nslices + MCG_NWAVE - 1) / MCG_NWAVE, max_grid));
  const int32_t *xm = g >= 8 ? A.xmap : nullptr;  // every XCD needs a workgroup
  if constexpr (sizeof(T) == 4) {
    if (A.v16) {  // FP16 values, FP32 arithmetic
      const _Float16 *h = A.v16;
#define MCG_BSELL16_CASE(BSV)                                                                  \
  case BSV:                                                                                    \
    if (dot)                                                                                   \
      k_bsell_spmv<BSV, T, true, _Float16><<<g, MCG_BLOCK, 0, s>>>(                            \
          A.nbr, A.nslices, A.off, A.col, h, x, y, St, r, part, compact, part_in, nb_in, k,    \
          xm);                                                                                 \
    else                                                                                       \
      k_bsell_spmv<BSV, T, false, _Float16><<<g, MCG_BLOCK, 0, s>>>(                           \
          A.nbr, A.nslices, A.off, A.col, h, x, y, St, r, part, compact, part_in, nb_in, k,    \
          xm);                                                                                 \
    break;
      switch (A.bs) {
        MCG_BSELL16_CASE(2)
        MCG_BSELL16_CASE(3)
        default:
        MCG_BSELL16_CASE(4)
      }
#undef MCG_BSELL16_CASE
      return g;
    }
  }
  const T *v = mcg_bsell_vals<T>(A);
#define MCG_BSELL_CASE(BSV)                                                                   \
  case BSV:                                                                                   \
    if (dot)                                                                                  \
      k_bsell_spmv<BSV, T, true><<<g, MCG_BLOCK, 0, s>>>(A.nbr, A.nslices, A.off, A.col, v, x, \
                                                         y, St, r, part, compact, part_in,     \
                                                         nb_in, k, xm);                        \
    else                                                                                      \
      k_bsell_spmv<BSV, T, false><<<g, MCG_BLOCK, 0, s>>>(A.nbr, A.nslices, A.off, A.col, v,  \
                                                          x, y, St, r, part, compact, part_in, \
                                                          nb_in, k, xm);                       \
    break;
  switch (A.bs) {
    MCG_BSELL_CASE(2)
    MCG_BSELL_CASE(3)
    default:
    MCG_BSELL_CASE(4)
  }
#undef MCG_BSELL_CASE
  return g;
}
template int mcg_bsell_spmv<double>(const mcg_bsell &, const double *, double *, DevState *,
                                    hipStream_t, bool, const double *, double *, double *,
                                    const double *, int, int, int);
template int mcg_bsell_spmv<float>(const mcg_bsell &, const float *, float *, DevState *,
                                   hipStream_t, bool, const float *, double *, double *,
                                   const double *, int, int, int);
