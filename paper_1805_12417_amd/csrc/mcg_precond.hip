// Second-level preconditioners beyond the diagonal ones.
//
// ILDL0: incomplete L D L^T with zero fill on the strictly lower pattern of
// A and signed pivots -- the symmetric form of the ILU(0) of A that the paper
// uses as the inner preconditioner (Section 4).  The factor is computed once
// at create on the host (IKJ order: row i is reduced by the already final
// rows k < i of its lower pattern); t = (L D L^T)^{-1} g is applied on the GPU
// by level-scheduled sweeps over node blocks of `block_size` unknowns: a
// block's level is one more than the highest level of the blocks its rows
// depend on, so each level is one kernel launch over independent blocks (8
// levels for the 8-colour ordered 27-point matrices).  Each level's blocks
// of L (forward) and of U = L^T (backward) are held in a sliced block copy
// (k_ildl_bsweep): dense bs x bs blocks, one int32 block column each,
// slot-major so that every load is one coalesced access, with the coupling
// inside a node block solved in registers.
//
// CCT: t = C (C^T g) with C lower triangular (the learned factor), as two
// CSR products (C^T is stored explicitly).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <type_traits>
#include <vector>

#include "mcg_host_par.h"
#include "mcg_ildlp_host.h"
#include "mcg_internal.h"

#define HIP_TRY_P(expr)                                              \
  do {                                                               \
    hipError_t e_ = (expr);                                          \
    if (e_ != hipSuccess) {                                          \
      mcg_last_hip_error = e_;                                       \
      return e_ == hipErrorOutOfMemory ? MCG_ENOMEM : MCG_EHIP;      \
    }                                                                \
  } while (0)

namespace {

constexpr int kMaxBlock = 4;  // unknowns per node block

// One triangle of the factor for the sweeps, sliced by level (layout at
// k_ildl_bsweep): block columns, values (FP64 and, in mixed precision, FP32)
// and the slot-group offsets of every slice.
struct ildl_side {
  int64_t *off = nullptr;
  int32_t *col = nullptr, *len = nullptr;
  double *v = nullptr;
  float *v32 = nullptr;
};

struct ildl_data {
  int n = 0, bs = 1, nlevels = 0, lpn = 1;
  ildl_side fwd, bwd;                    // blocks of L (forward) and of U = L^T (backward)
  int32_t *node = nullptr;               // node of (slice, lane), -1 for unused lanes
  double *dg = nullptr;                  // strictly lower L_II entries, then D_I^{-1}
  float *dg32 = nullptr;
  std::vector<int32_t> level_slice;      // host: slices of level l at [ptr[l], ptr[l+1])
  int32_t *level_slice_d = nullptr;      // device copy (read by the one-workgroup sweeps)
  // runs of levels in sweep order: {l0, l1, one_wg}; one_wg = 1: a run of
  // narrow levels swept by one workgroup, 0: one level, one launch
  std::vector<int32_t> runs;
  int64_t modified_pivots = 0;
};

// Levels of at most this many slices (64 / LPN nodes each) count as narrow:
// one pass of the one-workgroup sweep's wavefronts covers them.
constexpr int kNarrowSlices = 16;

// most Jacobi sweeps per triangle of the pivoted factor's apply
constexpr int kMaxJacobiSweeps = 64;

// kernel launches of one sweep pair
int ildl_launches(const ildl_data *D) { return 2 * (int)(D->runs.size() / 3); }

struct cct_data {
  int n = 0;
  int32_t *c_rp = nullptr, *c_ci = nullptr, *ct_rp = nullptr, *ct_ci = nullptr;
  double *c_v = nullptr, *ct_v = nullptr;
  float *c_v32 = nullptr, *ct_v32 = nullptr;
  double *tmp64 = nullptr;
  float *tmp32 = nullptr;
  int lanes = 8;
  // block CSR copies (zero-filled blocks), when the solver uses blocks
  int bsr = 0, nbr = 0;
  int32_t *cb_rp = nullptr, *cb_ci = nullptr, *ctb_rp = nullptr, *ctb_ci = nullptr;
  double *cb_v = nullptr, *ctb_v = nullptr;
  float *cb_v32 = nullptr, *ctb_v32 = nullptr;
  // sliced ELL copies, when the solver uses one for A
  mcg_sell c_sell, ct_sell;
  // sliced block copies, when the solver uses one for A
  mcg_bsell c_bsell, ct_bsell;
};

// Block CSR (blocks of bs, block columns sorted) of a CSR matrix; entries of
// a touched block that the CSR does not hold are stored as zeros.  Returns
// false (no copy) when that fill would exceed half the nonzeros.  Block rows
// are independent: counted, then filled, in parallel chunks.
bool csr_to_bsr(int n, int bs, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                const std::vector<double> &v, std::vector<int32_t> &brp,
                std::vector<int32_t> &bci, std::vector<double> &bv, double max_fill = 1.5) {
  const int N = n / bs;
  brp.assign(N + 1, 0);
  mcg_parallel_chunks(N, [&](int64_t lo, int64_t hi) {
    std::vector<int32_t> mark(N, -1);
    for (int64_t I = lo; I < hi; ++I) {
      int32_t c = 0;
      for (int a = 0; a < bs; ++a)
        for (int p = rp[I * bs + a]; p < rp[I * bs + a + 1]; ++p) {
          const int J = ci[p] / bs;
          if (mark[J] != I) {
            mark[J] = (int32_t)I;
            ++c;
          }
        }
      brp[I + 1] = c;
    }
  }, 0, 4096);
  for (int I = 0; I < N; ++I) brp[I + 1] += brp[I];
  const size_t nvals = (size_t)brp[N] * bs * bs;
  if (max_fill > 0.0 && (double)nvals > max_fill * (double)v.size()) return false;
  bci.resize(brp[N]);
  bv.assign(nvals, 0.0);
  mcg_parallel_chunks(N, [&](int64_t lo, int64_t hi) {
    std::vector<int32_t> pos(N, -1), cols;
    for (int64_t I = lo; I < hi; ++I) {
      cols.clear();
      for (int a = 0; a < bs; ++a)
        for (int p = rp[I * bs + a]; p < rp[I * bs + a + 1]; ++p) {
          const int J = ci[p] / bs;
          if (pos[J] != -2 - (int32_t)I) {  // first time in this block row
            pos[J] = -2 - (int32_t)I;
            cols.push_back(J);
          }
        }
      std::sort(cols.begin(), cols.end());
      for (size_t q = 0; q < cols.size(); ++q) {
        bci[brp[I] + q] = cols[q];
        pos[cols[q]] = brp[I] + (int32_t)q;
      }
      for (int a = 0; a < bs; ++a)
        for (int p = rp[I * bs + a]; p < rp[I * bs + a + 1]; ++p) {
          const int J = ci[p] / bs, b = ci[p] % bs;
          bv[((size_t)pos[J] * bs + a) * bs + b] = v[p];
        }
    }
  }, 0, 4096);
  return true;
}

template <typename T>
int upload(T **dst, const T *src, size_t count) {
  *dst = nullptr;
  HIP_TRY_P(hipMalloc((void **)dst, std::max<size_t>(1, count) * sizeof(T)));
  if (count) HIP_TRY_P(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return MCG_OK;
}

template <typename TO, typename TI>
std::vector<TO> convert(const std::vector<TI> &v) {
  std::vector<TO> out(v.size());
  mcg_parallel_chunks((int64_t)v.size(), [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) out[i] = (TO)v[i];
  });
  return out;
}

void csr_transpose(int n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                   const std::vector<double> &v, std::vector<int32_t> &trp,
                   std::vector<int32_t> &tci, std::vector<double> &tv) {
  mcg_csr_transpose_par(n, rp, ci, v, trp, tci, tv);
}

// ---------------------------------------------------------------------------
// Sliced block sweeps.  The nodes of one level are cut into slices of 64/LPN
// nodes; LPN consecutive lanes serve one node, lane n LPN + r taking the
// node's off-diagonal blocks r, r + LPN, ...  A slice's blocks are stored in
// groups of 64 (one per lane), slot-major as in k_bsell_spmv: the block
// column of (group j, lane l) at col[off[s] + 64 j + l], its entry (a, b) at
// val[(off[s] + 64 j) BB + (a BS + b) 64 + l].  Per node, at position
// m = l / LPN of slice s (NPS = 64 / LPN nodes per slice): node[s NPS + m]
// its index (-1 past the level's end), len[s NPS + m] its number of
// off-diagonal blocks (padding is never read into the sums: it is selected
// away, so stale values of t cannot leak in), and dg[(s ND + q) NPS + m] the
// strictly lower entries of L_II (row-major), then the BS entries of
// D_I^{-1}.
//   forward  (levels in order):   t_I = u_I = (I + L_II)^{-1} (g_I - sum_J L_IJ u_J)
//   backward (levels reversed):   t_I = (I + L_II^T)^{-1} (D_I^{-1} u_I - sum_J U_IJ t_J)
// with U_IJ = L_JI^T (J > I).  Nodes of one level never read each other's t.
// ---------------------------------------------------------------------------
template <int BS, int LPN, bool BWD, typename T>
__device__ __forceinline__ void sweep_slice(int s, int lane, const int32_t *__restrict__ node,
                                            const int32_t *__restrict__ len,
                                            const int64_t *__restrict__ off,
                                            const int32_t *__restrict__ col,
                                            const T *__restrict__ val, const T *__restrict__ dg,
                                            const T *__restrict__ g, T *__restrict__ t) {
  constexpr int BB = BS * BS, NL = BS * (BS - 1) / 2, ND = NL + BS, U = 4;
  constexpr int NPS = 64 / LPN;
  const int m = lane / LPN;
  const int I = node[(size_t)s * NPS + m];
  const int nl = len[(size_t)s * NPS + m];
  const int r = lane & (LPN - 1);
  const int64_t o = off[s];
  const int w = (int)((off[s + 1] - o) >> 6);
  const int32_t *cp = col + o + lane;
  const T *vp = val + o * BB + lane;
  T acc[BS];
#pragma unroll
  for (int a = 0; a < BS; ++a) acc[a] = 0;
  for (int j0 = 0; j0 < w; j0 += U) {
    int c[U];
    T bv[U][BB], xv[U][BS];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = min(j0 + u, w - 1);
      c[u] = cp[(size_t)j * 64];
#pragma unroll
      for (int q = 0; q < BB; ++q) bv[u][q] = vp[((size_t)j * BB + q) * 64];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int b = 0; b < BS; ++b) xv[u][b] = t[(size_t)c[u] * BS + b];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = (j0 + u) * LPN + r < nl;
#pragma unroll
      for (int a = 0; a < BS; ++a) {
        T sum = 0;
#pragma unroll
        for (int b = 0; b < BS; ++b) sum += bv[u][a * BS + b] * xv[u][b];
        acc[a] += ok ? sum : (T)0;
      }
    }
  }
#pragma unroll
  for (int m = LPN / 2; m > 0; m >>= 1)
#pragma unroll
    for (int a = 0; a < BS; ++a) acc[a] += __shfl_xor(acc[a], m, 64);
  if (r != 0 || I < 0) return;
  T d[ND];
#pragma unroll
  for (int q = 0; q < ND; ++q) d[q] = dg[((size_t)s * ND + q) * NPS + m];
  T y[BS];
  if constexpr (!BWD) {
#pragma unroll
    for (int a = 0; a < BS; ++a) {
      y[a] = g[(size_t)I * BS + a] - acc[a];
#pragma unroll
      for (int b = 0; b < a; ++b) y[a] -= d[a * (a - 1) / 2 + b] * y[b];
    }
  } else {
#pragma unroll
    for (int a = 0; a < BS; ++a) y[a] = t[(size_t)I * BS + a] * d[NL + a] - acc[a];
#pragma unroll
    for (int a = BS - 2; a >= 0; --a)
#pragma unroll
      for (int b = a + 1; b < BS; ++b) y[a] -= d[b * (b - 1) / 2 + a] * y[b];
  }
#pragma unroll
  for (int a = 0; a < BS; ++a) t[(size_t)I * BS + a] = y[a];
}


template <int BS, int LPN, bool BWD, typename T>
__global__ __launch_bounds__(256) void k_ildl_bsweep(
    int slice0, int nslices, const int32_t *__restrict__ node, const int32_t *__restrict__ len,
    const int64_t *__restrict__ off, const int32_t *__restrict__ col, const T *__restrict__ val,
    const T *__restrict__ dg, const T *__restrict__ g, T *__restrict__ t,
    const DevState *__restrict__ S, int check_done) {
  if (check_done && S->done) return;
  const int sl = blockIdx.x * MCG_NWAVE + (threadIdx.x >> 6);
  if (sl >= nslices) return;  // the whole wavefront leaves
  sweep_slice<BS, LPN, BWD, T>(slice0 + sl, threadIdx.x & 63, node, len, off, col, val, dg, g, t);
}

// A run of consecutive narrow levels [l0, l1) in one workgroup of kWgThreads
// threads: its wavefronts share each level's slices, and a workgroup barrier
// separates the levels (the backward sweep walks the run in reverse).  Deep,
// narrow level schedules (pivoted incomplete factors of grid-ordered
// matrices: thousands of levels of a few nodes) then cost a barrier per
// level instead of a kernel launch per level.  level_slice: device copy of
// the slice offsets of every level.
constexpr int kWgThreads = 1024;
template <int BS, int LPN, bool BWD, typename T>
__global__ __launch_bounds__(kWgThreads) void k_ildl_bsweep_wg(
    int l0, int l1, const int32_t *__restrict__ level_slice, const int32_t *__restrict__ node,
    const int32_t *__restrict__ len, const int64_t *__restrict__ off,
    const int32_t *__restrict__ col, const T *__restrict__ val, const T *__restrict__ dg,
    const T *__restrict__ g, T *__restrict__ t, const DevState *__restrict__ S, int check_done) {
  if (check_done && S->done) return;
  constexpr int NW = kWgThreads / 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int q = 0; q < l1 - l0; ++q) {
    const int l = BWD ? l1 - 1 - q : l0 + q;
    const int s0 = level_slice[l], s1 = level_slice[l + 1];
    for (int sl = s0 + wave; sl < s1; sl += NW)
      sweep_slice<BS, LPN, BWD, T>(sl, lane, node, len, off, col, val, dg, g, t);
    __syncthreads();
  }
}

// y = A x with a done check (C and C^T products of the learned preconditioner)
template <int L, typename T>
__global__ __launch_bounds__(256) void k_csr_apply(int n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const T *__restrict__ va,
                                                   const T *__restrict__ x, T *__restrict__ y,
                                                   const DevState *__restrict__ S,
                                                   int check_done) {
  if (check_done && S->done) return;
  __shared__ T tile[MCG_BLOCK];
  for (int row0 = blockIdx.x * MCG_BLOCK; row0 < n; row0 += gridDim.x * MCG_BLOCK) {
    csr_tile<L, T, T>(n, row0, rp, ci, va, x, tile);
    __syncthreads();
    const int row = row0 + threadIdx.x;
    if (row < n) y[row] = tile[threadIdx.x];
    __syncthreads();
  }
}

}  // namespace

// Level-scheduled sweep data (layout at k_ildl_bsweep) for a unit lower
// triangular factor L, given as its strictly lower part in CSR (lrp, lci,
// lv; consumed), in node blocks of bs unknowns; the backward sweep scales
// row i by dscale[i] (D^{-1} of an L D L^T with diagonal D, or 1 when a
// block diagonal D is applied on its own between the sweeps).
static int sweep_setup(ildl_data *D, int n, int bs, std::vector<int32_t> &lrp,
                       std::vector<int32_t> &lci, std::vector<double> &lv,
                       const std::vector<double> &dscale, bool mixed, hipStream_t s) {
  D->n = n;
  D->bs = bs;
  // level schedule over node blocks
  const int nn = n / bs;
  std::vector<int32_t> lev(nn, 0);
  int maxlev = 0;
  for (int I = 0; I < nn; ++I) {
    int l = 0;
    for (int r = I * bs; r < (I + 1) * bs; ++r)
      for (int32_t q = lrp[r]; q < lrp[r + 1]; ++q) {
        const int J = lci[q] / bs;
        if (J != I) l = std::max(l, lev[J] + 1);
      }
    lev[I] = l;
    maxlev = std::max(maxlev, l);
  }
  D->nlevels = maxlev + 1;
  std::vector<int32_t> level_ptr(D->nlevels + 1, 0);
  for (int I = 0; I < nn; ++I) level_ptr[lev[I] + 1]++;
  for (int l = 0; l < D->nlevels; ++l) level_ptr[l + 1] += level_ptr[l];
  std::vector<int32_t> order(nn);  // nodes by level, increasing within a level
  {
    std::vector<int32_t> fill(level_ptr.begin(), level_ptr.end() - 1);
    for (int I = 0; I < nn; ++I) order[fill[lev[I]]++] = I;
  }
  // U = L^T (rows hold entries of the columns of L)
  std::vector<int32_t> urp, uci;
  std::vector<double> uv;
  csr_transpose(n, lrp, lci, lv, urp, uci, uv);
  // node blocks of L and U (zeros stored for pattern gaps inside a block)
  std::vector<int32_t> lbrp, lbci, ubrp, ubci;
  std::vector<double> lbv, ubv;
  csr_to_bsr(n, bs, lrp, lci, lv, lbrp, lbci, lbv, 0.0);
  csr_to_bsr(n, bs, urp, uci, uv, ubrp, ubci, ubv, 0.0);
  lv.clear(); lv.shrink_to_fit();
  uv.clear(); uv.shrink_to_fit();
  // lanes per node: enough wavefronts per level to keep every SIMD busy
  const double per_level = (double)nn / D->nlevels;
  D->lpn = bs == 1 ? 1 : (per_level >= 4096 ? 4 : 2);
  const int lpn = D->lpn, npl = 64 / lpn;  // nodes per slice
  const int BB = bs * bs, NL = bs * (bs - 1) / 2, ND = NL + bs;
  D->level_slice.assign(D->nlevels + 1, 0);
  for (int l = 0; l < D->nlevels; ++l)
    D->level_slice[l + 1] = D->level_slice[l] + (level_ptr[l + 1] - level_ptr[l] + npl - 1) / npl;
  const int ns = D->level_slice[D->nlevels];
  // runs of narrow levels (two or more) for the one-workgroup sweep
  D->runs.clear();
  for (int l = 0; l < D->nlevels;) {
    int e = l;
    while (e < D->nlevels && D->level_slice[e + 1] - D->level_slice[e] <= kNarrowSlices) ++e;
    if (e - l >= 2) {
      D->runs.insert(D->runs.end(), {l, e, 1});
      l = e;
    } else {
      D->runs.insert(D->runs.end(), {l, l + 1, 0});
      l += 1;
    }
  }
  std::vector<int32_t> snode((size_t)ns * npl, -1);
  std::vector<double> sdg((size_t)ns * ND * npl, 0.0);
  for (int l = 0; l < D->nlevels; ++l)
    for (int k = level_ptr[l]; k < level_ptr[l + 1]; ++k) {
      const int pos = k - level_ptr[l];
      const int sl = D->level_slice[l] + pos / npl;
      const int I = order[k];
      const int mm = pos % npl;
      snode[(size_t)sl * npl + mm] = I;
      // the diagonal block of L is the last block of L's block row I (columns < I's
      // rows come first); it holds the strictly lower entries of L_II
      const int64_t db = lbrp[I + 1] - 1;
      const bool has_diag = lbrp[I + 1] > lbrp[I] && lbci[db] == I;
      for (int a2 = 1; a2 < bs; ++a2)
        for (int b2 = 0; b2 < a2; ++b2)
          sdg[((size_t)sl * ND + a2 * (a2 - 1) / 2 + b2) * npl + mm] =
              has_diag ? lbv[(size_t)db * BB + a2 * bs + b2] : 0.0;
      for (int a2 = 0; a2 < bs; ++a2)
        sdg[((size_t)sl * ND + NL + a2) * npl + mm] = dscale[(size_t)I * bs + a2];
    }
  // one triangle: blocks of row I other than the diagonal one, by level slices
  auto build_side = [&](ildl_side &sd, const std::vector<int32_t> &brp,
                        const std::vector<int32_t> &bci, const std::vector<double> &bv) -> int {
    std::vector<int64_t> off(ns + 1, 0);
    std::vector<int32_t> slen((size_t)ns * npl, 0);
    auto blocks_of = [&](int I, int j) {  // j-th off-diagonal block of row I
      const int64_t b0 = brp[I];
      const bool diag_first = brp[I + 1] > b0 && bci[b0] == I;
      const int64_t e = b0 + j + (diag_first ? 1 : 0);
      return e;
    };
    auto count_of = [&](int I) {
      int c = brp[I + 1] - brp[I];
      for (int64_t e = brp[I]; e < brp[I + 1]; ++e)
        if (bci[e] == I) --c;
      return c;
    };
    for (int sl = 0; sl < ns; ++sl) {
      int wgrp = 1;  // at least one group: the clamped loads stay inside the slice
      for (int mm = 0; mm < npl; ++mm) {
        const int I = snode[(size_t)sl * npl + mm];
        if (I < 0) continue;
        const int c = count_of(I);
        slen[(size_t)sl * npl + mm] = c;
        wgrp = std::max(wgrp, (c + lpn - 1) / lpn);
      }
      off[sl + 1] = off[sl] + 64 * (int64_t)wgrp;
    }
    const int64_t P = off[ns];
    std::vector<int32_t> c((size_t)P, 0);
    std::vector<double> v((size_t)P * BB, 0.0);
    for (int sl = 0; sl < ns; ++sl) {
      const int wgrp = (int)((off[sl + 1] - off[sl]) / 64);
      for (int ln = 0; ln < 64; ++ln) {
        const int I = snode[(size_t)sl * npl + ln / lpn];
        const int rr = ln % lpn;
        const int cnt = I >= 0 ? slen[(size_t)sl * npl + ln / lpn] : 0;
        for (int j = 0; j < wgrp; ++j) {
          const size_t e = (size_t)(off[sl] + 64 * (int64_t)j + ln);
          const int blk = j * lpn + rr;
          if (blk < cnt) {
            const int64_t src = blocks_of(I, blk);
            c[e] = bci[src];
            for (int q = 0; q < BB; ++q)
              v[(size_t)(off[sl] + 64 * (int64_t)j) * BB + (size_t)q * 64 + ln] =
                  bv[(size_t)src * BB + q];
          } else {
            c[e] = I >= 0 ? I : 0;  // any valid address: the kernel never uses it
          }
        }
      }
    }
    int rc2;
    if ((rc2 = upload(&sd.off, off.data(), off.size())) ||
        (rc2 = upload(&sd.col, c.data(), c.size())) ||
        (rc2 = upload(&sd.len, slen.data(), slen.size())) ||
        (rc2 = upload(&sd.v, v.data(), v.size())))
      return rc2;
    if (mixed) {
      HIP_TRY_P(hipMalloc((void **)&sd.v32, sizeof(float) * std::max<size_t>(1, v.size())));
      k_convert<float, double><<<2048, 256, 0, s>>>((int64_t)v.size(), sd.v, sd.v32);
      HIP_TRY_P(hipStreamSynchronize(s));
    }
    return MCG_OK;
  };
  // the forward reads blocks of L (columns J < I); the backward blocks of U (J > I)
  int rc;
  if ((rc = build_side(D->fwd, lbrp, lbci, lbv)) || (rc = build_side(D->bwd, ubrp, ubci, ubv)) ||
      (rc = upload(&D->node, snode.data(), snode.size())) ||
      (rc = upload(&D->dg, sdg.data(), sdg.size())) ||
      (rc = upload(&D->level_slice_d, D->level_slice.data(), D->level_slice.size())))
    return rc;
  if (mixed) {
    auto dg32 = convert<float>(sdg);
    if ((rc = upload(&D->dg32, dg32.data(), dg32.size()))) return rc;
  }
  return MCG_OK;
}


// ---------------------------------------------------------------------------
// ILDL0 create: factor on the host (IKJ), level schedule, upload
// ---------------------------------------------------------------------------
int mcg_ildl0_create(mcg_pc *p, double pivtol, hipStream_t s) {
  mcg_solver *h = p->h;
  const int n = h->n;
  int bs = std::max(1, h->opt.block_size);
  if (bs > kMaxBlock || n % bs != 0) return MCG_EINVAL;
  if (!(pivtol >= 0.0)) return MCG_EINVAL;
  const std::vector<int32_t> &rp = h->h_rp, &ci = h->h_ci;
  std::vector<double> va(h->nnz);
  HIP_TRY_P(hipStreamSynchronize(s));
  if (h->nnz) HIP_TRY_P(hipMemcpy(va.data(), h->va, sizeof(double) * h->nnz, hipMemcpyDeviceToHost));

  // strictly lower pattern of A and its row maxima / diagonal
  std::vector<int32_t> lrp(n + 1, 0), lci;
  std::vector<double> lv, d(n), rowmax(n, 0.0), diag(n, 0.0);
  std::vector<char> has_diag(n, 0);
  for (int i = 0; i < n; ++i) {
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
      rowmax[i] = std::max(rowmax[i], std::fabs(va[q]));
      if (ci[q] < i) {
        lci.push_back(ci[q]);
        lv.push_back(va[q]);
      } else if (ci[q] == i) {
        diag[i] = va[q];
        has_diag[i] = 1;
      }
    }
    lrp[i + 1] = (int32_t)lci.size();
  }
  for (int i = 0; i < n; ++i)
    if (!has_diag[i]) return MCG_EINVAL;
  // column lists of L: for column k, the positions q of entries (j, k), j > k
  std::vector<int32_t> crp(n + 1, 0), cpos(lci.size()), crow(lci.size());
  for (int32_t c : lci) crp[c + 1]++;
  for (int i = 0; i < n; ++i) crp[i + 1] += crp[i];
  {
    std::vector<int32_t> fill(crp.begin(), crp.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int32_t q = lrp[i]; q < lrp[i + 1]; ++q) {
        const int32_t f = fill[lci[q]]++;
        cpos[f] = q;
        crow[f] = i;
      }
  }
  // IKJ, row by row: w holds row i (lower part + diagonal) in dense form.
  // Row i reads only rows and pivots of its own pattern, all earlier in the
  // dependency order, so the rows of one level of that order are factored
  // in parallel (same operations, same order per row: the same factor).
  std::vector<int32_t> lev(n, 0);
  int nlev = 0;
  for (int i = 0; i < n; ++i) {
    int l = 0;
    for (int32_t q = lrp[i]; q < lrp[i + 1]; ++q) l = std::max(l, lev[lci[q]] + 1);
    lev[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  std::vector<int32_t> lptr(nlev + 1, 0), order(n);
  for (int i = 0; i < n; ++i) lptr[lev[i] + 1]++;
  for (int l = 0; l < nlev; ++l) lptr[l + 1] += lptr[l];
  {
    std::vector<int32_t> at(lptr.begin(), lptr.end() - 1);
    for (int i = 0; i < n; ++i) order[at[lev[i]]++] = i;
  }
  std::atomic<int64_t> modified{0};
  std::atomic<int> bad_pivot{0};
  const int nt = mcg_host_threads();
  std::vector<std::vector<double>> wbuf(nt);   // per chunk index, reused by every level
  std::vector<std::vector<int32_t>> mbuf(nt);
  for (int l = 0; l < nlev; ++l) {
    mcg_parallel_chunks_t(lptr[l + 1] - lptr[l], nt, [&](int t, int64_t lo, int64_t hi) {
      std::vector<double> &w = wbuf[t];
      std::vector<int32_t> &mark = mbuf[t];
      if (w.empty()) {
        w.assign(n, 0.0);
        mark.assign(n, -1);
      }
      int64_t mod = 0;
      for (int64_t r = lo; r < hi; ++r) {
        const int i = order[lptr[l] + r];
        for (int32_t q = lrp[i]; q < lrp[i + 1]; ++q) {
          w[lci[q]] = lv[q];
          mark[lci[q]] = i;
        }
        double wi = diag[i];
        for (int32_t q = lrp[i]; q < lrp[i + 1]; ++q) {
          const int k = lci[q];
          const double lik = w[k] / d[k];
          lv[q] = lik;
          // row k of U = D L^T: u_kj = d_k l_jk for the entries (j, k), j > k
          // rows j of column k increase; those below i hold final l_jk
          const double lik_dk = lik * d[k];
          for (int32_t c = crp[k]; c < crp[k + 1]; ++c) {
            const int j = crow[c];
            if (j >= i) break;
            if (mark[j] == i) w[j] -= lik_dk * lv[cpos[c]];
          }
          wi -= lik * lik * d[k];
        }
        const double floor_ = pivtol * rowmax[i];
        if (std::fabs(wi) < floor_) {
          wi = wi < 0.0 ? -floor_ : floor_;
          ++mod;
        }
        // an exactly zero (pivtol = 0) or non-finite pivot has no inverse
        if (!(wi != 0.0) || !std::isfinite(wi)) bad_pivot.store(1, std::memory_order_relaxed);
        d[i] = wi;
      }
      modified += mod;
    }, 256);
    if (bad_pivot.load()) return MCG_EINVAL;
  }

  // node blocks must be dense (their rows couple all earlier rows of the
  // block); otherwise schedule single rows
  for (int i = 0; i < n && bs > 1; ++i) {
    const int r0 = i - i % bs;
    int inside = 0;
    for (int32_t q = lrp[i]; q < lrp[i + 1]; ++q) inside += (lci[q] >= r0);
    if (inside != i - r0) bs = 1;
  }
  ildl_data *D = new ildl_data();
  p->ildl = D;
  D->modified_pivots = modified.load();
  std::vector<double> dinv(n);
  for (int i = 0; i < n; ++i) dinv[i] = 1.0 / d[i];
  const int rc = sweep_setup(D, n, bs, lrp, lci, lv, dinv, h->opt.precision == MCG_PREC_MIXED, s);
  p->apply_launches = ildl_launches(D);
  return rc;
}

// ---------------------------------------------------------------------------
// CCT create: copy C, build C^T
// ---------------------------------------------------------------------------
int mcg_cct_create(mcg_pc *p, const mcg_csr_t *Cm, hipStream_t s) {
  mcg_solver *h = p->h;
  if (!Cm || Cm->n != h->n || Cm->nnz < 0 || !Cm->row_ptr || (Cm->nnz && (!Cm->col || !Cm->val)))
    return MCG_EINVAL;
  const int n = h->n;
  const int64_t nnz = Cm->nnz;
  HIP_TRY_P(hipStreamSynchronize(s));
  std::vector<int32_t> rp(n + 1), ci(nnz);
  std::vector<double> v(nnz);
  HIP_TRY_P(hipMemcpy(rp.data(), Cm->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
  if (nnz) {
    HIP_TRY_P(hipMemcpy(ci.data(), Cm->col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    HIP_TRY_P(hipMemcpy(v.data(), Cm->val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
  }
  if (rp[0] != 0 || rp[n] != nnz) return MCG_EINVAL;
  for (int i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) return MCG_EINVAL;
  std::atomic<int> bad{0};
  mcg_parallel_chunks(n, [&](int64_t lo, int64_t hi) {
    bool b = false;
    for (int64_t i = lo; i < hi && !b; ++i)
      for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
        if (ci[q] < 0 || ci[q] > i ||  // lower triangular
            (q > rp[i] && ci[q] <= ci[q - 1]) || !std::isfinite(v[q])) {
          b = true;
          break;
        }
    if (b) bad.store(1, std::memory_order_relaxed);
  });
  if (bad.load()) return MCG_EINVAL;
  std::vector<int32_t> trp, tci;
  std::vector<double> tv;
  csr_transpose(n, rp, ci, v, trp, tci, tv);
  cct_data *D = new cct_data();
  p->cct = D;
  D->n = n;
  // lanes per row of the C and C^T products: 4, 16 or 32 from the mean row length
  const double mean = n ? (double)nnz / n : 1.0;
  D->lanes = mean <= 6.0 ? 4 : mean <= 20.0 ? 16 : 32;
  int rc;
  if ((rc = upload(&D->c_rp, rp.data(), rp.size())) || (rc = upload(&D->c_ci, ci.data(), ci.size())) ||
      (rc = upload(&D->c_v, v.data(), v.size())) || (rc = upload(&D->ct_rp, trp.data(), trp.size())) ||
      (rc = upload(&D->ct_ci, tci.data(), tci.size())) || (rc = upload(&D->ct_v, tv.data(), tv.size())))
    return rc;
  HIP_TRY_P(hipMalloc((void **)&D->tmp64, sizeof(double) * std::max(1, n)));
  const bool mixed = h->opt.precision == MCG_PREC_MIXED;
  if (mixed) {
    auto v32 = convert<float>(v), tv32 = convert<float>(tv);
    if ((rc = upload(&D->c_v32, v32.data(), v32.size())) || (rc = upload(&D->ct_v32, tv32.data(), tv32.size())))
      return rc;
    HIP_TRY_P(hipMalloc((void **)&D->tmp32, sizeof(float) * std::max(1, n)));
  }
  // block copies when the solver runs its SpMVs on blocks of A
  if (h->bsr_bs > 0) {
    const int bs = h->bsr_bs;
    std::vector<int32_t> brp, bci, tbrp, tbci;
    std::vector<double> bv, tbv;
    if (csr_to_bsr(n, bs, rp, ci, v, brp, bci, bv) &&
        csr_to_bsr(n, bs, trp, tci, tv, tbrp, tbci, tbv)) {
      if ((rc = upload(&D->cb_rp, brp.data(), brp.size())) ||
          (rc = upload(&D->cb_ci, bci.data(), bci.size())) ||
          (rc = upload(&D->cb_v, bv.data(), bv.size())) ||
          (rc = upload(&D->ctb_rp, tbrp.data(), tbrp.size())) ||
          (rc = upload(&D->ctb_ci, tbci.data(), tbci.size())) ||
          (rc = upload(&D->ctb_v, tbv.data(), tbv.size())))
        return rc;
      if (mixed) {
        auto bv32 = convert<float>(bv), tbv32 = convert<float>(tbv);
        if ((rc = upload(&D->cb_v32, bv32.data(), bv32.size())) ||
            (rc = upload(&D->ctb_v32, tbv32.data(), tbv32.size())))
          return rc;
      }
      D->bsr = bs;
      D->nbr = n / bs;
      if (h->bsa.bs) {
        if ((rc = mcg_bsell_build(&D->c_bsell, bs, n / bs, brp, bci, bv, 0.5, mixed, s, mixed,
                                  h->opt.xcd_order)) ||
            (rc = mcg_bsell_build(&D->ct_bsell, bs, n / bs, tbrp, tbci, tbv, 0.5, mixed, s,
                                  mixed, h->opt.xcd_order)))
          return rc;
        if (!D->c_bsell.bs || !D->ct_bsell.bs) {  // both or neither
          mcg_bsell_free(&D->c_bsell);
          mcg_bsell_free(&D->ct_bsell);
        } else if (!D->c_bsell.v16 != !D->ct_bsell.v16) {  // FP16 for both or neither
          for (mcg_bsell *c : {&D->c_bsell, &D->ct_bsell})
            if (c->v16) {
              (void)hipFree(c->v16);
              c->v16 = nullptr;
            }
        }
      }
    }
  }
  // sliced copies when the solver runs its SpMVs on a sliced copy of A
  if (h->sa.bits) {
    // in mixed precision the inner products read C and C^T as FP16 (both or
    // neither): C is the output of a BF16 network, FP16 keeps more digits
    if ((rc = mcg_sell_build(&D->c_sell, n, rp, ci, v.data(), true, 0.5, mixed, s, mixed)) ||
        (rc = mcg_sell_build(&D->ct_sell, n, trp, tci, tv.data(), true, 0.5, mixed, s, mixed)))
      return rc;
    if (!D->c_sell.bits || !D->ct_sell.bits) {  // both or neither
      mcg_sell_free(&D->c_sell);
      mcg_sell_free(&D->ct_sell);
    } else if (!D->c_sell.v16 != !D->ct_sell.v16) {
      for (mcg_sell *c : {&D->c_sell, &D->ct_sell})
        if (c->v16) {
          (void)hipFree(c->v16);
          c->v16 = nullptr;
        }
    }
  }
  return MCG_OK;
}

void mcg_ildlp_release(mcg_pc *p);

void mcg_pc_release_extra(mcg_pc *p) {
  mcg_ildlp_release(p);
  if (p->ildl) {
    ildl_data *D = (ildl_data *)p->ildl;
    void *b[] = {D->fwd.off, D->fwd.col, D->fwd.len, D->fwd.v, D->fwd.v32,
                 D->bwd.off, D->bwd.col, D->bwd.len, D->bwd.v, D->bwd.v32,
                 D->node, D->dg, D->dg32, D->level_slice_d};
    for (void *x : b)
      if (x) (void)hipFree(x);
    delete D;
    p->ildl = nullptr;
  }
  if (p->cct) {
    cct_data *D = (cct_data *)p->cct;
    void *b[] = {D->c_rp, D->c_ci, D->ct_rp, D->ct_ci, D->c_v, D->ct_v, D->c_v32, D->ct_v32,
                 D->tmp64, D->tmp32, D->cb_rp, D->cb_ci, D->ctb_rp, D->ctb_ci, D->cb_v,
                 D->ctb_v, D->cb_v32, D->ctb_v32};
    for (void *x : b)
      if (x) (void)hipFree(x);
    mcg_sell_free(&D->c_sell);
    mcg_sell_free(&D->ct_sell);
    mcg_bsell_free(&D->c_bsell);
    mcg_bsell_free(&D->ct_bsell);
    delete D;
    p->cct = nullptr;
  }
}

// ---------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------
template <typename T>
static const T *pick(const double *a64, const float *a32);
template <>
const double *pick<double>(const double *a64, const float *) { return a64; }
template <>
const float *pick<float>(const double *, const float *a32) { return a32; }

template <int BS, int LPN, typename T>
static void ildl_sweeps(const ildl_data *D, const T *g, T *t, const DevState *S, int check_done,
                        hipStream_t s, int which = 3) {
  const T *fv = pick<T>(D->fwd.v, D->fwd.v32), *bv = pick<T>(D->bwd.v, D->bwd.v32);
  const T *dg = pick<T>(D->dg, D->dg32);
  const int nr = (int)D->runs.size() / 3;
  auto sweep = [&](int r, auto bwd_tag) {
    constexpr bool BWD = decltype(bwd_tag)::value;
    const int l0 = D->runs[3 * r], l1 = D->runs[3 * r + 1];
    const ildl_side &sd = BWD ? D->bwd : D->fwd;
    const T *v = BWD ? bv : fv;
    if (D->runs[3 * r + 2]) {
      k_ildl_bsweep_wg<BS, LPN, BWD, T><<<1, kWgThreads, 0, s>>>(
          l0, l1, D->level_slice_d, D->node, sd.len, sd.off, sd.col, v, dg, g, t, S, check_done);
    } else {
      const int s0 = D->level_slice[l0], cnt = D->level_slice[l0 + 1] - s0;
      k_ildl_bsweep<BS, LPN, BWD, T><<<(cnt + MCG_NWAVE - 1) / MCG_NWAVE, MCG_BLOCK, 0, s>>>(
          s0, cnt, D->node, sd.len, sd.off, sd.col, v, dg, g, t, S, check_done);
    }
  };
  if (which & 1)
    for (int r = 0; r < nr; ++r) sweep(r, std::false_type{});
  if (which & 2)
    for (int r = nr - 1; r >= 0; --r) sweep(r, std::true_type{});
}

template <typename T>
void mcg_ildl0_apply(const mcg_pc *p, const T *g, T *t, DevState *S, int check_done,
                     hipStream_t s) {
  const ildl_data *D = (const ildl_data *)p->ildl;
  switch (D->bs * 8 + D->lpn) {
    case 1 * 8 + 1: ildl_sweeps<1, 1, T>(D, g, t, S, check_done, s); break;
    case 2 * 8 + 2: ildl_sweeps<2, 2, T>(D, g, t, S, check_done, s); break;
    case 2 * 8 + 4: ildl_sweeps<2, 4, T>(D, g, t, S, check_done, s); break;
    case 3 * 8 + 2: ildl_sweeps<3, 2, T>(D, g, t, S, check_done, s); break;
    case 3 * 8 + 4: ildl_sweeps<3, 4, T>(D, g, t, S, check_done, s); break;
    case 4 * 8 + 2: ildl_sweeps<4, 2, T>(D, g, t, S, check_done, s); break;
    default: ildl_sweeps<4, 4, T>(D, g, t, S, check_done, s); break;
  }
}

template <typename T>
void mcg_cct_apply(const mcg_pc *p, const T *g, T *t, DevState *S, int check_done,
                   hipStream_t s) {
  const cct_data *D = (const cct_data *)p->cct;
  const int grid = std::max(1, std::min((D->n + 255) / 256, 2048));
  T *tmp = (T *)pick<T>(D->tmp64, D->tmp32);
  const T *cv = pick<T>(D->c_v, D->c_v32), *ctv = pick<T>(D->ct_v, D->ct_v32);
  switch (D->lanes) {
#define MCG_CCT_CASE(LL)                                                                     \
  case LL:                                                                                   \
    k_csr_apply<LL, T><<<grid, 256, 0, s>>>(D->n, D->ct_rp, D->ct_ci, ctv, g, tmp, S, check_done); \
    k_csr_apply<LL, T><<<grid, 256, 0, s>>>(D->n, D->c_rp, D->c_ci, cv, tmp, t, S, check_done);    \
    break;
    MCG_CCT_CASE(2)
    MCG_CCT_CASE(4)
    MCG_CCT_CASE(8)
    MCG_CCT_CASE(16)
    MCG_CCT_CASE(32)
    default:
    MCG_CCT_CASE(64)
#undef MCG_CCT_CASE
  }
}

template <typename T>
void mcg_csr_apply(int lanes, int n, const int32_t *rp, const int32_t *ci, const T *va, const T *x,
                   T *y, DevState *S, int check_done, hipStream_t s) {
  const int grid = std::max(1, std::min((n + 255) / 256, 2048));
  switch (lanes) {
#define MCG_CSR_CASE(LL)                                                               \
  case LL:                                                                             \
    k_csr_apply<LL, T><<<grid, 256, 0, s>>>(n, rp, ci, va, x, y, S, check_done);        \
    break;
    MCG_CSR_CASE(2)
    MCG_CSR_CASE(4)
    MCG_CSR_CASE(8)
    MCG_CSR_CASE(16)
    MCG_CSR_CASE(32)
    default:
    MCG_CSR_CASE(64)
#undef MCG_CSR_CASE
  }
}
template void mcg_csr_apply<double>(int, int, const int32_t *, const int32_t *, const double *,
                                    const double *, double *, DevState *, int, hipStream_t);
template void mcg_csr_apply<float>(int, int, const int32_t *, const int32_t *, const float *,
                                   const float *, float *, DevState *, int, hipStream_t);

bool mcg_cct_view_get(const mcg_pc *p, bool fp32, mcg_cct_view *v) {
  if (!p || !p->cct || !v) return false;
  const cct_data *D = (const cct_data *)p->cct;
  if (fp32 && !D->c_v32) return false;
  v->lanes = D->lanes;
  v->c_rp = D->c_rp;
  v->c_ci = D->c_ci;
  v->ct_rp = D->ct_rp;
  v->ct_ci = D->ct_ci;
  v->c_v = fp32 ? (const void *)D->c_v32 : (const void *)D->c_v;
  v->ct_v = fp32 ? (const void *)D->ct_v32 : (const void *)D->ct_v;
  v->tmp = fp32 ? (void *)D->tmp32 : (void *)D->tmp64;
  v->bsr = D->bsr;
  v->nbr = D->nbr;
  v->cb_rp = D->cb_rp;
  v->cb_ci = D->cb_ci;
  v->ctb_rp = D->ctb_rp;
  v->ctb_ci = D->ctb_ci;
  v->cb_v = fp32 ? (const void *)D->cb_v32 : (const void *)D->cb_v;
  v->ctb_v = fp32 ? (const void *)D->ctb_v32 : (const void *)D->ctb_v;
  v->c_sell = D->c_sell.bits ? &D->c_sell : nullptr;
  v->ct_sell = D->ct_sell.bits ? &D->ct_sell : nullptr;
  v->c_bsell = D->c_bsell.bs ? &D->c_bsell : nullptr;
  v->ct_bsell = D->ct_bsell.bs ? &D->ct_bsell : nullptr;
  return true;
}

int mcg_ildl0_levels(const mcg_pc *p) {  // (for probes and tests)
  return p && p->ildl ? ((const ildl_data *)p->ildl)->nlevels : 0;
}

int64_t mcg_ildl0_modified_pivots(const mcg_pc *p) {
  return p && p->ildl ? ((const ildl_data *)p->ildl)->modified_pivots : 0;
}

// ---------------------------------------------------------------------------
// ILDLP: the pivoted incomplete factor P A P^T ~ L D L^T (Section 4's
// ILDL^T(fill, drop); built on the host by PivotedBuilder).  On the GPU:
// gather P g, forward sweep with L, the 1x1 / 2x2 blocks of D^{-1}, backward
// sweep with L^T (the level-sliced sweeps above, one unknown per node),
// scatter P^T.
// ---------------------------------------------------------------------------
namespace {

struct ildlp_data {
  int n = 0;
  PivotedLDL host;                        // the factor (host copy, for export)
  ildl_data sweeps_data;                  // L and L^T, one unknown per node, no D scaling
  int32_t *perm = nullptr, *bsize = nullptr;
  double *dinv = nullptr;                 // 2 per row: (D^{-1})_kk, (D^{-1})_{k,k+1}
  float *dinv32 = nullptr;
  double *tmp64 = nullptr, *tmp64b = nullptr;
  float *tmp32 = nullptr, *tmp32b = nullptr;
  int64_t nnz_l = 0, two_by_two = 0;
  // sweeps > 0: Jacobi sweeps instead of the triangular solves, over CSR
  // copies of L_s (strictly lower, logical order) and of its transpose
  int sweeps = 0;
  int lanes_l = 4, lanes_u = 4;
  int32_t *l_rp = nullptr, *l_ci = nullptr, *u_rp = nullptr, *u_ci = nullptr;
  int32_t *l_cip = nullptr;  // perm[l_ci], the first forward sweep's gather from g
  double *l_v = nullptr, *u_v = nullptr;
  float *l_v32 = nullptr, *u_v32 = nullptr;
  // w = D^{-1} u row by row: w_i = wd_i u_i + wo_i u_{wp_i} (wp_i = the other
  // row of i's 2x2 block, or i with wo_i = 0)
  double *wd = nullptr, *wo = nullptr;
  float *wd32 = nullptr, *wo32 = nullptr;
  int32_t *wp = nullptr;
};

// One Jacobi sweep v = y - L x, L lanes per row (rows in tiles of MCG_BLOCK),
// with the permutation and D^{-1} folded into the first and last sweeps:
//   FIRST: y_i = g_{perm_i} and x_j = g_{perm_j} (ci holds perm[col] for
//          this sweep); y is also written to ybuf for the later sweeps
//   TOW:   the output is w = D^{-1} v: w_i = wd_i v_i + wo_i v_{wp_i}, the
//          partner row's v taken from the tile or, across a tile edge,
//          recomputed by the thread itself
//   SCAT:  the output goes to out_{perm_i} instead of out_i
template <int L, typename T, bool FIRST, bool TOW, bool SCAT>
__global__ __launch_bounds__(256) void k_jsweep_x(
    int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const T *__restrict__ va, const int32_t *__restrict__ perm, const T *__restrict__ y,
    const T *__restrict__ x, T *__restrict__ ybuf, const T *__restrict__ wd,
    const T *__restrict__ wo, const int32_t *__restrict__ wp, T *__restrict__ out,
    const DevState *__restrict__ S, int check_done) {
  if (check_done && S->done) return;
  __shared__ T tile[MCG_BLOCK];
  for (int row0 = blockIdx.x * MCG_BLOCK; row0 < n; row0 += gridDim.x * MCG_BLOCK) {
    csr_tile<L, T, T>(n, row0, rp, ci, va, x, tile);
    __syncthreads();
    const int row = row0 + threadIdx.x;
    T v = 0;
    if (row < n) {
      const T base = FIRST ? y[perm[row]] : y[row];
      if constexpr (FIRST) ybuf[row] = base;
      v = base - tile[threadIdx.x];
    }
    if constexpr (TOW) {
      __syncthreads();
      tile[threadIdx.x] = v;
      __syncthreads();
      if (row < n) {
        const int q = wp[row];
        T vq = v;
        if (q != row) {
          const int r = q - row0;
          if (r >= 0 && r < MCG_BLOCK) {
            vq = tile[r];
          } else {
            T acc = 0;
            for (int32_t e = rp[q]; e < rp[q + 1]; ++e) acc += va[e] * x[ci[e]];
            vq = (FIRST ? y[perm[q]] : y[q]) - acc;
          }
        }
        out[row] = wd[row] * v + wo[row] * vq;
      }
    } else if (row < n) {
      if constexpr (SCAT)
        out[perm[row]] = v;
      else
        out[row] = v;
    }
    __syncthreads();
  }
}

template <bool FIRST, bool TOW, bool SCAT, typename T>
void launch_jsweep_x(int lanes, int n, const int32_t *rp, const int32_t *ci, const T *va,
                     const int32_t *perm, const T *y, const T *x, T *ybuf, const T *wd,
                     const T *wo, const int32_t *wp, T *out, const DevState *S, int check_done,
                     hipStream_t s) {
  const int grid = std::max(1, std::min((n + MCG_BLOCK - 1) / MCG_BLOCK, 2048));
#define MCG_JX(LN)                                                                       \
  k_jsweep_x<LN, T, FIRST, TOW, SCAT><<<grid, MCG_BLOCK, 0, s>>>(n, rp, ci, va, perm, y, x, \
                                                               ybuf, wd, wo, wp, out, S, check_done)
  switch (lanes) {
    case 2: MCG_JX(2); break;
    case 4: MCG_JX(4); break;
    case 8: MCG_JX(8); break;
    default: MCG_JX(16); break;
  }
#undef MCG_JX
}

// out = y - L x (one Jacobi sweep of L u = y; L given by its strictly lower
// CSR part), L lanes per row
template <int L, typename T>
__global__ __launch_bounds__(256) void k_jsweep(int n, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci,
                                                const T *__restrict__ va, const T *__restrict__ y,
                                                const T *__restrict__ x, T *__restrict__ out,
                                                const DevState *__restrict__ S, int check_done) {
  if (check_done && S->done) return;
  __shared__ T tile[MCG_BLOCK];
  for (int row0 = blockIdx.x * MCG_BLOCK; row0 < n; row0 += gridDim.x * MCG_BLOCK) {
    csr_tile<L, T, T>(n, row0, rp, ci, va, x, tile);
    __syncthreads();
    const int row = row0 + threadIdx.x;
    if (row < n) out[row] = y[row] - tile[threadIdx.x];
    __syncthreads();
  }
}

template <typename T>
void launch_jsweep(int lanes, int n, const int32_t *rp, const int32_t *ci, const T *va, const T *y,
                   const T *x, T *out, const DevState *S, int check_done, hipStream_t s) {
  const int grid = std::max(1, std::min((n + MCG_BLOCK - 1) / MCG_BLOCK, 2048));
  switch (lanes) {
    case 2: k_jsweep<2, T><<<grid, MCG_BLOCK, 0, s>>>(n, rp, ci, va, y, x, out, S, check_done); break;
    case 4: k_jsweep<4, T><<<grid, MCG_BLOCK, 0, s>>>(n, rp, ci, va, y, x, out, S, check_done); break;
    case 8: k_jsweep<8, T><<<grid, MCG_BLOCK, 0, s>>>(n, rp, ci, va, y, x, out, S, check_done); break;
    default: k_jsweep<16, T><<<grid, MCG_BLOCK, 0, s>>>(n, rp, ci, va, y, x, out, S, check_done); break;
  }
}

int lanes_for_mean(double mean) { return mean <= 2.0 ? 2 : mean <= 4.0 ? 4 : mean <= 8.0 ? 8 : 16; }

template <typename T>
__global__ void k_perm_gather(int n, const int32_t *__restrict__ perm, const T *__restrict__ g,
                              T *__restrict__ y, const DevState *__restrict__ S, int check_done) {
  if (check_done && S->done) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    y[i] = g[perm[i]];
}

template <typename T>
__global__ void k_perm_scatter(int n, const int32_t *__restrict__ perm, const T *__restrict__ v,
                               T *__restrict__ t, const DevState *__restrict__ S,
                               int check_done) {
  if (check_done && S->done) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    t[perm[i]] = v[i];
}

// y = D^{-1} u, 1x1 and 2x2 blocks; dinv holds per row (D^{-1})_kk and, at
// the first row of a 2x2 block, (D^{-1})_{k,k+1}
template <typename T>
__global__ void k_dblock_solve(int n, const int32_t *__restrict__ bsize,
                               const T *__restrict__ dinv, const T *__restrict__ u,
                               T *__restrict__ y, const DevState *__restrict__ S,
                               int check_done) {
  if (check_done && S->done) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int b = bsize[i];
    if (b == 1) {
      y[i] = dinv[2 * (size_t)i] * u[i];
    } else if (b == 2) {
      const T x0 = u[i], x1 = u[i + 1];
      const T d00 = dinv[2 * (size_t)i], d01 = dinv[2 * (size_t)i + 1];
      const T d11 = dinv[2 * (size_t)(i + 1)];
      y[i] = d00 * x0 + d01 * x1;
      y[i + 1] = d01 * x0 + d11 * x1;
    }
  }
}

}  // namespace

int mcg_ildlp_create(mcg_pc *p, double fill, double drop, int sweeps, hipStream_t s) {
  mcg_solver *h = p->h;
  const int n = h->n;
  if (!(fill >= 0.0) || !(drop >= 0.0) || !std::isfinite(fill) || !std::isfinite(drop) ||
      sweeps < 0 || sweeps > kMaxJacobiSweeps)
    return MCG_EINVAL;
  std::vector<double> va(h->nnz);
  HIP_TRY_P(hipStreamSynchronize(s));
  if (h->nnz) HIP_TRY_P(hipMemcpy(va.data(), h->va, sizeof(double) * h->nnz, hipMemcpyDeviceToHost));
  PivotedLDL F;
  {
    PivotedBuilder B(n, h->h_rp, h->h_ci, va, fill, drop);
    B.run(F);
  }
  // D^{-1} per block; a singular or non-finite block is an error
  std::vector<double> dinv(2 * (size_t)n, 0.0);
  int64_t two = 0;
  for (int k = 0; k < n; ++k) {
    if (F.bsize[k] == 1) {
      dinv[2 * (size_t)k] = 1.0 / F.dd[k];
    } else if (F.bsize[k] == 2) {
      const double a = F.dd[k], b = F.doff[k], e = F.dd[k + 1], det = a * e - b * b;
      if (!(det != 0.0) || !std::isfinite(det)) return MCG_EINVAL;
      dinv[2 * (size_t)k] = e / det;
      dinv[2 * (size_t)k + 1] = -b / det;
      dinv[2 * (size_t)(k + 1)] = a / det;
      ++two;
    }
  }
  for (double x : dinv)
    if (!std::isfinite(x)) return MCG_EINVAL;
  for (double x : F.lv)
    if (!std::isfinite(x)) return MCG_EINVAL;
  ildlp_data *D = new ildlp_data();
  p->ildlp = D;
  D->n = n;
  D->nnz_l = (int64_t)F.lv.size();
  D->two_by_two = two;
  const bool mixed = h->opt.precision == MCG_PREC_MIXED;
  int rc;
  if ((rc = upload(&D->perm, F.perm.data(), F.perm.size())) ||
      (rc = upload(&D->bsize, F.bsize.data(), F.bsize.size())) ||
      (rc = upload(&D->dinv, dinv.data(), dinv.size())))
    return rc;
  HIP_TRY_P(hipMalloc((void **)&D->tmp64, sizeof(double) * std::max(1, n)));
  if (mixed) {
    auto d32 = convert<float>(dinv);
    if ((rc = upload(&D->dinv32, d32.data(), d32.size()))) return rc;
    HIP_TRY_P(hipMalloc((void **)&D->tmp32, sizeof(float) * std::max(1, n)));
  }
  D->host = F;
  if (sweeps > 0) {
    // CSR copies of L_s and L_s^T for the Jacobi sweeps
    D->sweeps = sweeps;
    std::vector<int32_t> urp, uci;
    std::vector<double> uv;
    csr_transpose(n, F.lrp, F.lci, F.lv, urp, uci, uv);
    const double mean = n ? (double)F.lv.size() / n : 0.0;
    D->lanes_l = lanes_for_mean(mean);
    D->lanes_u = lanes_for_mean(mean);
    std::vector<int32_t> lcip(F.lci.size());
    for (size_t e = 0; e < lcip.size(); ++e) lcip[e] = F.perm[F.lci[e]];
    if ((rc = upload(&D->l_rp, F.lrp.data(), F.lrp.size())) ||
        (rc = upload(&D->l_ci, F.lci.data(), F.lci.size())) ||
        (rc = upload(&D->l_cip, lcip.data(), lcip.size())) ||
        (rc = upload(&D->l_v, F.lv.data(), F.lv.size())) ||
        (rc = upload(&D->u_rp, urp.data(), urp.size())) ||
        (rc = upload(&D->u_ci, uci.data(), uci.size())) ||
        (rc = upload(&D->u_v, uv.data(), uv.size())))
      return rc;
    HIP_TRY_P(hipMalloc((void **)&D->tmp64b, sizeof(double) * std::max(1, n)));
    {
      std::vector<double> wd(n), wo(n, 0.0);
      std::vector<int32_t> wp(n);
      for (int i = 0; i < n; ++i) {
        wd[i] = dinv[2 * (size_t)i];
        wp[i] = i;
        if (F.bsize[i] == 2) {
          wp[i] = i + 1;
          wo[i] = dinv[2 * (size_t)i + 1];
        } else if (F.bsize[i] == 0) {
          wp[i] = i - 1;
          wo[i] = dinv[2 * (size_t)(i - 1) + 1];
        }
      }
      if ((rc = upload(&D->wd, wd.data(), wd.size())) ||
          (rc = upload(&D->wo, wo.data(), wo.size())) ||
          (rc = upload(&D->wp, wp.data(), wp.size())))
        return rc;
      if (mixed) {
        auto wd32 = convert<float>(wd), wo32 = convert<float>(wo);
        if ((rc = upload(&D->wd32, wd32.data(), wd32.size())) ||
            (rc = upload(&D->wo32, wo32.data(), wo32.size())))
          return rc;
      }
    }
    if (mixed) {
      auto l32 = convert<float>(F.lv);
      auto u32 = convert<float>(uv);
      if ((rc = upload(&D->l_v32, l32.data(), l32.size())) ||
          (rc = upload(&D->u_v32, u32.data(), u32.size())))
        return rc;
      HIP_TRY_P(hipMalloc((void **)&D->tmp32b, sizeof(float) * std::max(1, n)));
    }
    p->apply_launches = 2 * sweeps;
    return MCG_OK;
  }
  const std::vector<double> ones(n, 1.0);
  rc = sweep_setup(&D->sweeps_data, n, 1, F.lrp, F.lci, F.lv, ones, mixed, s);
  p->apply_launches = ildl_launches(&D->sweeps_data) + 3;
  return rc;
}

void mcg_ildlp_release(mcg_pc *p) {
  if (!p->ildlp) return;
  ildlp_data *D = (ildlp_data *)p->ildlp;
  ildl_data &W = D->sweeps_data;
  void *b[] = {W.fwd.off, W.fwd.col, W.fwd.len, W.fwd.v, W.fwd.v32, W.bwd.off, W.bwd.col,
               W.bwd.len, W.bwd.v, W.bwd.v32, W.node, W.dg, W.dg32, W.level_slice_d, D->perm,
               D->bsize, D->dinv, D->dinv32, D->tmp64, D->tmp32, D->tmp64b, D->tmp32b,
               D->l_rp, D->l_ci, D->l_cip, D->l_v, D->l_v32, D->u_rp, D->u_ci, D->u_v, D->u_v32,
               D->wd, D->wo, D->wd32, D->wo32, D->wp};
  for (void *x : b)
    if (x) (void)hipFree(x);
  delete D;
  p->ildlp = nullptr;
}

extern "C" int mcg_ildlp_factor_get(mcg_precond_t p, int32_t *perm, int32_t *bsize, double *dd,
                                    double *doff, int32_t *l_ptr, int32_t *l_col, double *l_val,
                                    int64_t *nnz_l) {
  if (!p || !p->ildlp || !nnz_l) return MCG_EINVAL;
  const PivotedLDL &F = ((const ildlp_data *)p->ildlp)->host;
  const size_t n = F.perm.size(), nz = F.lv.size();
  if (perm) std::copy(F.perm.begin(), F.perm.end(), perm);
  if (bsize) std::copy(F.bsize.begin(), F.bsize.end(), bsize);
  if (dd) std::copy(F.dd.begin(), F.dd.end(), dd);
  if (doff) std::copy(F.doff.begin(), F.doff.end(), doff);
  if (l_ptr) std::copy(F.lrp.begin(), F.lrp.begin() + n + 1, l_ptr);
  if (l_col) std::copy(F.lci.begin(), F.lci.end(), l_col);
  if (l_val) std::copy(F.lv.begin(), F.lv.end(), l_val);
  *nnz_l = (int64_t)nz;
  return MCG_OK;
}

template <typename T>
void mcg_ildlp_apply(const mcg_pc *p, const T *g, T *t, DevState *S, int check_done,
                     hipStream_t s) {
  const ildlp_data *D = (const ildlp_data *)p->ildlp;
  const int n = D->n;
  const int grid = std::max(1, std::min((n + 255) / 256, 1024));
  T *y = const_cast<T *>(pick<T>(D->tmp64, D->tmp32));
  const T *dinv = pick<T>(D->dinv, D->dinv32);
  if (D->sweeps > 0) {
    // 2s launches.  Forward u_j = y - L_s u_{j-1} (u_0 = y): the first sweep
    // forms y = P g in ybuf, the last one writes w = D^{-1} u_s to b.
    // Backward v_j = w - L_s^T v_{j-1} (v_0 = w), the last one written to t
    // through P^T.  u_1..u_{s-1} alternate between t and b with u_{s-1} in
    // t, so that the last forward sweep can write w to b; v_1..v_{s-1}
    // alternate between ybuf and t with v_{s-1} in ybuf.
    T *b = const_cast<T *>(pick<T>(D->tmp64b, D->tmp32b));
    const T *lv = pick<T>(D->l_v, D->l_v32), *uv = pick<T>(D->u_v, D->u_v32);
    const T *wd = pick<T>(D->wd, D->wd32), *wo = pick<T>(D->wo, D->wo32);
    const int sw = D->sweeps;
    auto fwd_out = [&](int j) { return ((sw - j) % 2 == 0) ? b : t; };
    auto bwd_out = [&](int j) { return ((sw - 1 - j) % 2 == 0) ? y : t; };
    if ((const void *)g == (const void *)t && sw > 1 && fwd_out(1) == t) {
      // in place: the first sweep would overwrite g while other rows still
      // read it; b is free until the second sweep
      (void)hipMemcpyAsync(b, g, sizeof(T) * (size_t)n, hipMemcpyDeviceToDevice, s);
      g = b;
    }
    const int32_t *pm = D->perm, *wp = D->wp;
    const int ll = D->lanes_l, lu = D->lanes_u;
    if (sw == 1) {
      launch_jsweep_x<true, true, false, T>(ll, n, D->l_rp, D->l_cip, lv, pm, g, g, y, wd, wo, wp,
                                            b, S, check_done, s);
    } else {
      launch_jsweep_x<true, false, false, T>(ll, n, D->l_rp, D->l_cip, lv, pm, g, g, y, wd, wo,
                                             wp, fwd_out(1), S, check_done, s);
      for (int j = 2; j < sw; ++j)
        launch_jsweep<T>(ll, n, D->l_rp, D->l_ci, lv, y, fwd_out(j - 1), fwd_out(j), S,
                         check_done, s);
      launch_jsweep_x<false, true, false, T>(ll, n, D->l_rp, D->l_ci, lv, pm, y, fwd_out(sw - 1),
                                             nullptr, wd, wo, wp, b, S, check_done, s);
    }
    // b holds w
    const T *x = b;
    for (int j = 1; j < sw; ++j) {
      launch_jsweep<T>(lu, n, D->u_rp, D->u_ci, uv, b, x, bwd_out(j), S, check_done, s);
      x = bwd_out(j);
    }
    launch_jsweep_x<false, false, true, T>(lu, n, D->u_rp, D->u_ci, uv, pm, b, x, nullptr, wd, wo,
                                           wp, t, S, check_done, s);
    return;
  }
  k_perm_gather<T><<<grid, 256, 0, s>>>(n, D->perm, g, y, S, check_done);      // y = P g
  ildl_sweeps<1, 1, T>(&D->sweeps_data, y, t, S, check_done, s, 1);           // t = L^{-1} y
  k_dblock_solve<T><<<grid, 256, 0, s>>>(n, D->bsize, dinv, t, y, S, check_done);  // y = D^{-1} t
  ildl_sweeps<1, 1, T>(&D->sweeps_data, t, y, S, check_done, s, 2);           // y = L^{-T} y
  k_perm_scatter<T><<<grid, 256, 0, s>>>(n, D->perm, y, t, S, check_done);    // t = P^T y
}

template void mcg_ildl0_apply<double>(const mcg_pc *, const double *, double *, DevState *, int,
                                      hipStream_t);
template void mcg_ildl0_apply<float>(const mcg_pc *, const float *, float *, DevState *, int,
                                     hipStream_t);
template void mcg_ildlp_apply<double>(const mcg_pc *, const double *, double *, DevState *, int,
                                      hipStream_t);
template void mcg_ildlp_apply<float>(const mcg_pc *, const float *, float *, DevState *, int,
                                     hipStream_t);
template void mcg_cct_apply<double>(const mcg_pc *, const double *, double *, DevState *, int,
                                    hipStream_t);
template void mcg_cct_apply<float>(const mcg_pc *, const float *, float *, DevState *, int,
                                   hipStream_t);
