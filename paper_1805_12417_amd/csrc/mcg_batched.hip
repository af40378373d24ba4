// Batched MINRES-CG: many independent systems (e.g. the shifted systems of a
// shift-and-invert eigensolver, Section 3.1), each with up to 8 right-hand
// sides, solved by persistent kernel launches: one per k bucket (systems
// grouped by their number of deflation vectors, so that register arrays are
// sized by the bucket), one after the other.
//
// * Each system gets a team of its group's workgroups, sized by its work
//   (nnz + (k + 1) n), or by work x inner iterations after a re-plan from an
//   earlier solve (minres_cg_batch_rebalance).  A team runs the whole method
//   for its system: outer MINRES per right-hand side (FP64), inner CG per
//   right-hand side (FP32 or FP64), Jacobi M_cg.
// * Vectors of a system are row-interleaved n x NR (entry (i, c) at i*NR + c),
//   so the SpMM reads each CSR value / column index once for all columns and
//   the NR values of a gathered row are contiguous.  A thread owns one (row,
//   column) pair; a wavefront covers 64/NR rows.  In the buckets of k >= 32
//   the NR lanes of a row share the row's Vhat entries (each reads k/NR of
//   them and the lanes exchange partial sums).
// * Team synchronisation: sense-free generation barrier on two counters per
//   team (atomic arrive, spin on the generation with s_sleep).  Reductions are
//   team all-reduces: each block writes its partial sums, the barrier, then
//   every block sums all partials of its team in block order, so every block
//   holds bitwise identical totals and derives the CG / MINRES scalars itself
//   (kept in LDS; no scalar goes through global memory).  Partials alternate
//   between two buffers, which is enough because a block cannot reach the
//   reduction after next before every block has passed the next barrier.
// * Control flow inside a team depends only on those totals, so all blocks of
//   a team take the same number of barriers.  Every spin has a wall-clock
//   limit: a block that waits too long raises a global abort flag, every
//   other waiter sees it and leaves, and the solve reports an error -- no
//   wave can wait forever.  The grid is capped at the number of blocks the
//   GPU holds at once (occupancy query), so all blocks of a team are resident.
// * Converged columns are masked (their entries are no longer written).
#include <algorithm>
#include <thread>
#include <cmath>
#include <cstring>
#include <queue>
#include <vector>

#include "mcg_internal.h"

#define HIP_TRY_B(expr)                                          \
  do {                                                           \
    hipError_t e_ = (expr);                                      \
    if (e_ != hipSuccess) {                                      \
      mcg_last_hip_error = e_;                                   \
      return e_ == hipErrorOutOfMemory ? MCG_ENOMEM : MCG_EHIP;  \
    }                                                            \
  } while (0)

namespace {

constexpr int BB = 256;               // threads per block
constexpr int BW = BB / 64;           // waves per block
constexpr int kBatchKMax = 64;
constexpr int kRefresh = 32;          // direct recomputation period of Vhat^T p, Vhat^T t
constexpr int kRows = 4;              // rows per thread in flight in the streaming phases
constexpr int kProfPerSys = 9;        // t_begin, t_end, team iterations, 6 phase times

struct BSys {
  int32_t n, k, team0, nteam;
  const int32_t *rp, *ci;
  const double *va;   // FP64 values (outer)
  const void *vaT;    // inner-precision values
  const void *VT;     // Vhat (inner precision), n x k column-major
  const void *dinvT;  // 1 / diag(A), inner precision
  double c[kBatchKMax];  // 2 |lambda_j|
  const double *b;       // n x NR interleaved (filled by the solve)
  double *x;             // n x NR interleaved
  double *r1, *r2, *y, *v, *w, *w1, *w2, *rt, *xbest;
  void *z, *r, *p, *q;   // inner precision
  double *part;          // 2 buffers x nteam x pw
  unsigned *bar;         // [0] arrivals, [1] generation
};

struct BOut {
  int32_t status, outer_its;
  int64_t inner_its;
  double relres, bnorm;
};

struct BParams {
  double rtol_out, rtol_in;
  int32_t maxit_out, stag_window, keep_best, pw;
  int64_t maxit_in;
  unsigned *abort_flag;
  int64_t timeout_ticks;  // wall_clock64 ticks a barrier may wait
  int64_t *prof;          // per system: wall clock at the team's start and end, team iterations
};

// ---------------------------------------------------------------------------
// team barrier with abort
// ---------------------------------------------------------------------------
__device__ bool team_barrier(unsigned *bar, int nteam, unsigned *abort_flag, int64_t timeout) {
  __shared__ int aborted;
  __syncthreads();
  if (threadIdx.x == 0) {
    aborted = 0;
    // The wait polls with relaxed agent-scope loads (coherent, no cache
    // maintenance) and acquires once when it ends: an acquire load inside
    // the loop would invalidate this XCD's L2 on every poll, under the feet
    // of every other team that shares it.
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // release: this block's stores (ordered by __syncthreads) and the read of
    // gen before arriving
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned arrived = atomicAdd(&bar[0], 1u);
    if (arrived == (unsigned)nteam - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      atomicAdd(&bar[1], 1u);
    } else {
      const int64_t t0 = wall_clock64();
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          aborted = 1;
          break;
        }
        if (wall_clock64() - t0 > timeout) {
          atomicOr(abort_flag, 1u);
          aborted = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the team's stores are visible
    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) aborted = 1;
  }
  __syncthreads();
  return aborted == 0;
}

// ---------------------------------------------------------------------------
// per-block state (LDS): every block of a team holds the same values
// ---------------------------------------------------------------------------
template <int NR, int KB>
struct Lds {
  // reduction scratch and totals
  static constexpr int kMaxNV = (3 + KB > 2 * KB) ? 3 + KB : 2 * KB;  // widest reduction
  double red[kMaxNV * NR * BW];
  double tot[(1 + 2 * KB) * NR + 3 * NR + 8];
  double sc[BB];  // per thread-group sums of the team partials
  // inner CG, per column
  double rho[NR], alpha[NR], beta[NR], yy[NR], rtol2;
  int act_in[NR], in_status[NR];
  int64_t its[NR];
  double s[KB][NR], vt[KB][NR], wv[KB][NR], csv[KB][NR];
  float csvf[KB][NR];  // csv rounded to FP32, read by the FP32 inner iteration
  // boundary
  double scale[NR], inv_scale[NR];
  // outer MINRES, per column
  double beta_cur[NR], oldb[NR], dbar[NR], epsln[NR], oldeps[NR], phibar[NR], cs[NR], sn[NR];
  double delta[NR], gamma[NR], phi[NR], alfa[NR], bnorm[NR], best[NR], rnorm[NR];
  int since_best[NR], status[NR], act_out[NR], outer_its[NR], improved[NR];
  int64_t inner_total[NR];
  int64_t team_its;  // inner iterations the team ran (any column active)
  // block 0 of the team: wall-clock ticks spent in the inner iteration's
  // phases (A, B, C), each split into local work and the team reduction
  int64_t ph[6], ph_t;
  int any;
  int buf;
  int ok;
};

template <int NR, int KB, int NV>
__device__ bool team_allreduce_finish(Lds<NR, KB> &L, const BSys &S, const BParams &P, int lb);

// Coefficient c_j s_j of column c in the inner precision (FP32: the copy
// rounded once when the coefficients change).
template <typename T, int NR, int KB>
__device__ __forceinline__ T csv_coef(const Lds<NR, KB> &L, int j, int c) {
  if constexpr (sizeof(T) == 4) return L.csvf[j][c];
  else return (T)L.csv[j][c];
}

// Team all-reduce of per-thread values.  A thread contributes v[0..nv-1] for
// its column c = lane % NR; the result tot[e*NR + c] is the team sum of entry
// e of column c.  Returns false if the team aborted.
// The values come from get(e) (e a compile-time-unrolled index), so callers
// can reduce straight from their own accumulators without a copy.
template <int NR, int KB, int NV, typename Get>
__device__ bool team_allreduce_get(Get get, Lds<NR, KB> &L, const BSys &S, const BParams &P,
                                   int lb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int e = 0; e < NV; ++e) {
    double x = get(e);
#pragma unroll
    for (int off = 32; off >= NR; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane < NR) L.red[(e * NR + lane) * BW + wave] = x;
  }
  return team_allreduce_finish<NR, KB, NV>(L, S, P, lb);
}

// The team sums of W partial values (see team_allreduce_finish): G = BB / W
// thread groups, each over every G-th block in eight interleaved running
// sums, then the G group sums in group order (sc: BB doubles of LDS).  Not
// inlined, so that its registers do not add to the iteration's.
template <int W>
__device__ __noinline__ void sum_partials(const double *part, int pw, int nteam, double *sc,
                                          double *tot) {
  constexpr int G = BB / W > 1 ? BB / W : 1;
  for (int jt = threadIdx.x; jt < W * G; jt += BB) {
    const int j = jt % W, g = jt / W;
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = 0.0;
    int b = g;
    for (; b + 7 * G < nteam; b += 8 * G)
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += part[(size_t)(b + u * G) * pw + j];
#pragma unroll
    for (int u = 0; u < 7; ++u)  // fewer than 8 of the group's blocks are left
      if (b + u * G < nteam) a[u] += part[(size_t)(b + u * G) * pw + j];
    const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    if constexpr (G > 1)
      sc[g * W + j] = s;
    else
      tot[j] = s;
  }
  if constexpr (G > 1) {
    __syncthreads();
    for (int j = threadIdx.x; j < W; j += BB) {
      double s = 0.0;
      for (int g = 0; g < G; ++g) s += sc[g * W + j];
      tot[j] = s;
    }
  }
}

// Second half of a team all-reduce: L.red holds every wave's sums (entry e
// of column c at (e NR + c) BW + wave); the block sums go to the team's
// partials, and after the barrier every block adds all partials of its team
// (sum_partials: spread over the block's threads, in a fixed order, so every
// block of the team gets bitwise the same totals).
template <int NR, int KB, int NV>
__device__ bool team_allreduce_finish(Lds<NR, KB> &L, const BSys &S, const BParams &P, int lb) {
  static_assert(NV <= Lds<NR, KB>::kMaxNV, "reduction wider than the LDS scratch");
  constexpr int W = NV * NR;
  __syncthreads();
  double *part = S.part + (size_t)L.buf * S.nteam * P.pw;
  for (int j = threadIdx.x; j < W; j += BB) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < BW; ++q) s += L.red[j * BW + q];
    part[(size_t)lb * P.pw + j] = s;
  }
  // team_barrier orders these stores: workgroup barrier, then one
  // device-scope release by thread 0 before it arrives
  if (!team_barrier(S.bar, S.nteam, P.abort_flag, P.timeout_ticks)) return false;
  sum_partials<W>(part, P.pw, S.nteam, L.sc, L.tot);
  __syncthreads();
  if (threadIdx.x == 0) L.buf ^= 1;
  __syncthreads();
  return true;
}

template <int NR, int KB, int NV>
__device__ bool team_allreduce(const double (&v)[NV], int nv, Lds<NR, KB> &L, const BSys &S,
                               const BParams &P, int lb) {
  (void)nv;
  return team_allreduce_get<NR, KB, NV>([&](int e) { return v[e]; }, L, S, P, lb);
}

// Vhat row i (clamped column index, see vhat_row)
template <int KB, typename T>
__device__ __forceinline__ void vrow(const T *__restrict__ V, int n, int k, int i, T (&v)[KB]) {
  vhat_row<KB, T>(V, n, k, i, v);  // blocked device layout (mcg_kernels.h)
}

// Row i of A times column c of a row-interleaved vector u: the row's entries
// in chunks of 8 whose index, value and gathered loads are all issued before
// the first use (clamped to the row's last entry, so every load is in
// bounds), so a thread waits about three memory latencies per chunk instead
// of two per entry.  With NR >= 2 lanes per row, the lanes of a row split a
// chunk's indices and values (8 / NR loads each instead of 8) and hand them
// round through lane exchanges; the lanes of a row share beg and end, so
// they run the loop together.  The sum runs over the entries in order, as a
// plain loop.
template <int NR, typename T>
__device__ __forceinline__ T csr_row_dot(const int32_t *__restrict__ ci, const T *__restrict__ va,
                                         const T *__restrict__ u, int beg, int end, int c) {
  T acc = 0;
  for (int p0 = beg; p0 < end; p0 += 8) {
    int cols[8];
    T vals[8], xs[8];
    if constexpr (NR >= 2) {
      constexpr int PER = 8 / NR;
      const int base = (int)(threadIdx.x & 63) & ~(NR - 1);
      int mc[PER];
      T mv[PER];
#pragma unroll
      for (int v = 0; v < PER; ++v) {
        const int pp = p0 + c + v * NR < end ? p0 + c + v * NR : end - 1;
        mc[v] = ci[pp];
        mv[v] = va[pp];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        cols[j] = __shfl(mc[j / NR], base + j % NR, 64);
        vals[j] = __shfl(mv[j / NR], base + j % NR, 64);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int pp = p0 + j < end ? p0 + j : end - 1;
        cols[j] = ci[pp];
        vals[j] = va[pp];
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) xs[j] = u[(size_t)cols[j] * NR + c];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (p0 + j < end) acc += vals[j] * xs[j];
  }
  return acc;
}

// The NR lanes of a row (lanes aligned on NR) each hold v[0..NR-1], one value
// per right-hand side; returns to lane c the sum over the row's lanes of
// v[c] (recursive halving: NR - 1 exchanges).
template <int NR, typename T>
__device__ __forceinline__ T row_reduce_scatter(T (&v)[NR], int c) {
#pragma unroll
  for (int o = NR / 2; o >= 1; o >>= 1) {
    const bool hi = (c & o) != 0;
#pragma unroll
    for (int a = 0; a < o; ++a) {
      const T send = hi ? v[a] : v[a + o];
      const T keep = hi ? v[a + o] : v[a];
      v[a] = keep + __shfl_xor(send, o, 64);
    }
  }
  return v[0];
}

// out[c2] = x of lane c2 of this lane's row (all NR right-hand sides).
template <int NR, typename T>
__device__ __forceinline__ void row_all_gather(T x, T (&out)[NR]) {
  const int base = (int)(threadIdx.x & 63) & ~(NR - 1);
#pragma unroll
  for (int c2 = 0; c2 < NR; ++c2) out[c2] = __shfl(x, base + c2, 64);
}

// ---------------------------------------------------------------------------
// the persistent kernel
// ---------------------------------------------------------------------------
template <typename T, int NR, int KB>
__global__ __launch_bounds__(BB) __attribute__((amdgpu_waves_per_eu(2))) void k_batched_minres_cg(const BSys *__restrict__ systems,
                                                         const int32_t *__restrict__ block_sys,
                                                         BParams P, BOut *__restrict__ out) {
  __shared__ Lds<NR, KB> L;
  const int sid = block_sys[blockIdx.x];
  const BSys &S = systems[sid];
  const int lb = blockIdx.x - S.team0;
  const int n = S.n, k = S.k;
  const int c = threadIdx.x % NR;         // column of this thread
  const int rsub = threadIdx.x / NR;      // row slot within a block pass
  constexpr int RPB = BB / NR;            // rows per block pass
  const int rstride = S.nteam * RPB;
  const int rstart = lb * RPB + rsub;
  const int32_t *__restrict__ rp = S.rp;
  const int32_t *__restrict__ ci = S.ci;
  const T *__restrict__ vaT = (const T *)S.vaT;
  const T *__restrict__ VT = (const T *)S.VT;
  const T *__restrict__ dinv = (const T *)S.dinvT;
  T *__restrict__ z = (T *)S.z;
  T *__restrict__ r = (T *)S.r;
  T *__restrict__ p = (T *)S.p;
  T *__restrict__ q = (T *)S.q;
  double *r1 = S.r1, *r2 = S.r2, *y = S.y, *v = S.v, *w = S.w, *w1 = S.w1, *w2 = S.w2;
  double *x = S.x;
  const double *b = S.b;
  const bool mixed = sizeof(T) == 4;
  const double eps = mixed ? 1.1920928955078125e-07 : 2.220446049250313e-16;
  if (threadIdx.x == 0) {
    L.buf = 0;
    L.team_its = 0;
    for (int q = 0; q < 6; ++q) L.ph[q] = 0;
    if (lb == 0) P.prof[kProfPerSys * (size_t)sid] = wall_clock64();
  }
  __syncthreads();
  bool ok = true;

  // ---- O0: rt = b - A x0, ||rt||^2, ||b||^2; r1 = rt; xbest = x ----------
  {
    double a0 = 0.0, a1 = 0.0;
    for (int i = rstart; i < n; i += rstride) {
      const double acc = csr_row_dot<NR, double>(ci, S.va, x, rp[i], rp[i + 1], c);
      const size_t e = (size_t)i * NR + c;
      const double bi = b[e];
      const double ri = bi - acc;
      r1[e] = ri;
      S.xbest[e] = x[e];
      // the direction vectors start at zero (their first two updates scale
      // them by zero, which must not meet stale NaN bit patterns)
      w[e] = 0.0;
      w1[e] = 0.0;
      w2[e] = 0.0;
      a0 += ri * ri;
      a1 += bi * bi;
    }
    double vv[2] = {a0, a1};
    ok = team_allreduce<NR, KB, 2>(vv, 2, L, S, P, lb);
    if (threadIdx.x < NR) {
      const int cc = threadIdx.x;
      const double rn = sqrt(L.tot[cc]), bn = sqrt(L.tot[NR + cc]);
      L.bnorm[cc] = bn;
      L.rnorm[cc] = rn;
      L.best[cc] = rn;
      L.since_best[cc] = 0;
      L.outer_its[cc] = 0;
      L.inner_total[cc] = 0;
      L.status[cc] = 1;  // MAXIT until decided otherwise
      L.act_out[cc] = 1;
      if (!(bn == bn) || !(rn == rn) || isinf(bn) || isinf(rn)) {
        L.status[cc] = -1;
        L.act_out[cc] = 0;
      } else if (bn == 0.0) {
        L.status[cc] = 0;
        L.act_out[cc] = 0;
      } else if (rn <= P.rtol_out * bn) {
        L.status[cc] = 0;
        L.act_out[cc] = 0;
      }
      L.scale[cc] = mixed ? rn : 1.0;
      L.inv_scale[cc] = mixed ? (rn > 0.0 ? 1.0 / rn : 0.0) : 1.0;
    }
    __syncthreads();
  }
  // b = 0 columns: x = 0
  for (int i = rstart; i < n; i += rstride)
    if (L.status[c] == 0 && L.bnorm[c] == 0.0) x[(size_t)i * NR + c] = 0.0;
  // no inner iteration allowed: nothing is solved, x stays x0 (MAXIT)
  if (P.maxit_in <= 0) {
    if (threadIdx.x < NR && L.act_out[threadIdx.x]) L.act_out[threadIdx.x] = 0;
    __syncthreads();
  }

  // inner solve on the FP64 vector yin (scaled by inv_scale), result in z
  auto inner_solve = [&](const double *yin) -> bool {
    // I0: r = yin * inv_scale, z = 0, t = D^-1 r, p = t; rr, rt, tt, Vhat^T t
    {
      double a[3] = {0.0, 0.0, 0.0};
      T accv[KB];
#pragma unroll
      for (int j = 0; j < KB; ++j) accv[j] = 0;
      const bool act = L.act_out[c] != 0;
      for (int i = rstart; i < n; i += rstride) {
        const size_t e = (size_t)i * NR + c;
        const T ri = act ? (T)(yin[e] * L.inv_scale[c]) : (T)0;
        const T ti = dinv[i] * ri;
        r[e] = ri;
        z[e] = 0;
        p[e] = ti;
        a[0] += (double)(ri * ri);
        a[1] += (double)(ri * ti);
        a[2] += (double)(ti * ti);
        if (k > 0) {
          const T *vb = VT + (size_t)(i / MCG_VBLK) * ((size_t)MCG_VBLK * k) + (i % MCG_VBLK);
#pragma unroll
          for (int j = 0; j < KB; ++j) accv[j] += vb[(size_t)(j < k ? j : k - 1) * MCG_VBLK] * ti;
        }
      }
      if (!team_allreduce_get<NR, KB, 3 + KB>(
              [&](int e) { return e < 3 ? a[e < 3 ? e : 0] : (double)accv[e >= 3 ? e - 3 : 0]; },
              L, S, P, lb))
        return false;
      if (threadIdx.x < NR) {
        const int cc = threadIdx.x;
        const double rr = L.tot[cc], rt = L.tot[NR + cc], tt = L.tot[2 * NR + cc];
        L.yy[cc] = rr;
        L.rho[cc] = rt;
        L.its[cc] = 0;
        L.in_status[cc] = 0;
        L.act_in[cc] = L.act_out[cc] && rr > 0.0;
        if (L.act_in[cc] && !(fabs(rt) > eps * sqrt(rr) * sqrt(tt))) {
          L.act_in[cc] = 0;
          L.in_status[cc] = 3;
        }
        for (int j = 0; j < KB; ++j) {
          const double sj = j < k ? L.tot[(3 + j) * NR + cc] : 0.0;
          L.s[j][cc] = sj;
          L.vt[j][cc] = sj;
          L.csv[j][cc] = j < k ? S.c[j] * sj : 0.0;
          L.csvf[j][cc] = (float)L.csv[j][cc];
        }
      }
      if (threadIdx.x == 0) {
        int any = 0;
        for (int cc = 0; cc < NR; ++cc) any |= L.act_in[cc];
        L.any = any;
        L.rtol2 = P.rtol_in * P.rtol_in;
      }
      __syncthreads();
    }
    const int64_t cap = n < P.maxit_in ? n : P.maxit_in;
    // phase clock of block 0 (thread 0 only; no synchronisation)
    auto mark = [&](int q) {
      if (lb == 0 && threadIdx.x == 0) {
        const int64_t now = wall_clock64();
        if (q >= 0) L.ph[q] += now - L.ph_t;
        L.ph_t = now;
      }
    };
    for (int64_t it = 0; it < cap && L.any; ++it) {
      if (threadIdx.x == 0) L.team_its += 1;
      mark(-1);
      // A: q = A p + Vhat (c o s); pi = p^T q; w = Vhat^T D^-1 q.
      // Column indices are clamped to k-1 (unconditional loads); the
      // coefficients of j >= k are zero and w_j for j >= k is ignored.  The
      // coefficients c o s are read from LDS.
      if constexpr (NR > 1 && KB >= 32) {
        // Wide buckets: the NR lanes of a row share its Vhat row.  Lane c
        // reads columns j = c + NR jj (KJ of them, once), forms its part of
        // Vhat (c o s) for all NR right-hand sides and the lanes exchange
        // those parts (reduce-scatter); then each lane takes D^-1 q of all NR
        // right-hand sides (all-gather) to accumulate w_j for its own j.
        // KB / NR loads of the row per lane instead of 2 KB.
        constexpr int KJ = KB / NR;
        static_assert(KB % NR == 0, "k bucket not a multiple of the rhs count");
        T pq = 0, wacc[KJ][NR];
#pragma unroll
        for (int jj = 0; jj < KJ; ++jj)
#pragma unroll
          for (int c2 = 0; c2 < NR; ++c2) wacc[jj][c2] = 0;
        // the next row's bounds are loaded while this row is processed
        // (index clamped to this row on the last pass)
        int beg = rstart < n ? rp[rstart] : 0, end = rstart < n ? rp[rstart + 1] : 0;
        for (int i = rstart; i < n; i += rstride) {
          const int inext = i + rstride < n ? i + rstride : i;
          const int nbeg = rp[inext], nend = rp[inext + 1];
          T acc = csr_row_dot<NR, T>(ci, vaT, p, beg, end, c);
          beg = nbeg;
          end = nend;
          const size_t e = (size_t)i * NR + c;
          if (k > 0) {
            const T *vb = VT + (size_t)(i / MCG_VBLK) * ((size_t)MCG_VBLK * k) + (i % MCG_VBLK);
            T vr[KJ];
#pragma unroll
            for (int jj = 0; jj < KJ; ++jj) {
              const int j = c + NR * jj;
              vr[jj] = vb[(size_t)(j < k ? j : k - 1) * MCG_VBLK];
            }
            T ps[NR];
#pragma unroll
            for (int c2 = 0; c2 < NR; ++c2) {
              T sum = 0;
#pragma unroll
              for (int jj = 0; jj < KJ; ++jj) sum += vr[jj] * csv_coef<T>(L, c + NR * jj, c2);
              ps[c2] = sum;
            }
            acc += row_reduce_scatter<NR, T>(ps, c);
            q[e] = acc;
            pq += p[e] * acc;
            T dqs[NR];
            row_all_gather<NR, T>(dinv[i] * acc, dqs);
#pragma unroll
            for (int jj = 0; jj < KJ; ++jj)
#pragma unroll
              for (int c2 = 0; c2 < NR; ++c2) wacc[jj][c2] += vr[jj] * dqs[c2];
          } else {
            q[e] = acc;
            pq += p[e] * acc;
          }
        }
        // wave sums: entry 0 is p^T q of the lane's column; lane c's
        // wacc[jj][c2] is entry 1 + c + NR jj of column c2
        {
          const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
          double x = (double)pq;
#pragma unroll
          for (int off = 32; off >= NR; off >>= 1) x += __shfl_xor(x, off, 64);
          if (lane < NR) L.red[lane * BW + wave] = x;
#pragma unroll
          for (int jj = 0; jj < KJ; ++jj)
#pragma unroll
            for (int c2 = 0; c2 < NR; ++c2) {
              double y = (double)wacc[jj][c2];
#pragma unroll
              for (int off = 32; off >= NR; off >>= 1) y += __shfl_xor(y, off, 64);
              if (lane < NR) L.red[((1 + lane + NR * jj) * NR + c2) * BW + wave] = y;
            }
        }
        mark(0);
        if (!team_allreduce_finish<NR, KB, 1 + KB>(L, S, P, lb)) return false;
        mark(1);
      } else {
        // Narrow buckets and single right-hand sides: each lane reads the
        // whole Vhat row, twice (the second read hits the cache), so that
        // only w stays in registers across rows.
        T pq = 0, wacc[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) wacc[j] = 0;
        for (int i = rstart; i < n; i += rstride) {
          T acc = csr_row_dot<NR, T>(ci, vaT, p, rp[i], rp[i + 1], c);
          const T *vb = VT + (size_t)(i / MCG_VBLK) * ((size_t)MCG_VBLK * k) + (i % MCG_VBLK);
          if (k > 0) {
#pragma unroll
            for (int j = 0; j < KB; ++j)
              acc += vb[(size_t)(j < k ? j : k - 1) * MCG_VBLK] * csv_coef<T>(L, j, c);
          }
          const size_t e = (size_t)i * NR + c;
          q[e] = acc;
          pq += p[e] * acc;
          if (k > 0) {
            const T dq = dinv[i] * acc;
            asm volatile("" ::: "memory");  // re-read the row rather than keep it live
#pragma unroll
            for (int j = 0; j < KB; ++j) wacc[j] += vb[(size_t)(j < k ? j : k - 1) * MCG_VBLK] * dq;
          }
        }
        mark(0);
        if (!team_allreduce_get<NR, KB, 1 + KB>(
                [&](int e) { return e == 0 ? (double)pq : (double)wacc[e > 0 ? e - 1 : 0]; }, L,
                S, P, lb))
          return false;
        mark(1);
      }
      {
        if (threadIdx.x < NR) {
          const int cc = threadIdx.x;
          if (L.act_in[cc]) {
            const double pi = L.tot[cc];
            if (!(pi > 0.0)) {
              L.act_in[cc] = 0;
              L.in_status[cc] = 4;  // NOT_SPD
              L.alpha[cc] = 0.0;
            } else {
              L.alpha[cc] = L.rho[cc] / pi;
            }
            for (int j = 0; j < KB; ++j) L.wv[j][cc] = L.tot[(1 + j) * NR + cc];
          } else {
            L.alpha[cc] = 0.0;
          }
        }
        __syncthreads();
      }
      // B: z += alpha p; r -= alpha q; t = D^-1 r; rr, rt, tt; beta, stop tests
      {
        double a[3] = {0.0, 0.0, 0.0};
        const bool act = L.act_in[c] != 0;
        const T alpha = (T)L.alpha[c];
        // kRows rows per thread in flight (loads clamped to row n-1, stores
        // guarded); the sums run over the rows in order, as a plain loop
        for (int i0 = rstart; i0 < n; i0 += kRows * rstride) {
          T rv[kRows], zv[kRows], pv[kRows], qv[kRows], dv[kRows];
#pragma unroll
          for (int u = 0; u < kRows; ++u) {
            const int i = min(i0 + u * rstride, n - 1);
            const size_t e = (size_t)i * NR + c;
            rv[u] = r[e];
            dv[u] = dinv[i];
            zv[u] = act ? z[e] : (T)0;
            pv[u] = act ? p[e] : (T)0;
            qv[u] = act ? q[e] : (T)0;
          }
#pragma unroll
          for (int u = 0; u < kRows; ++u) {
            const int i = i0 + u * rstride;
            if (i < n) {
              const size_t e = (size_t)i * NR + c;
              T ri = rv[u];
              if (act) {
                z[e] = zv[u] + alpha * pv[u];
                ri -= alpha * qv[u];
                r[e] = ri;
              }
              const T ti = dv[u] * ri;
              a[0] += (double)(ri * ri);
              a[1] += (double)(ri * ti);
              a[2] += (double)(ti * ti);
            }
          }
        }
        mark(2);
        if (!team_allreduce<NR, KB, 3>(a, 3, L, S, P, lb)) return false;
        mark(3);
        if (threadIdx.x < NR) {
          const int cc = threadIdx.x;
          if (L.act_in[cc]) {
            const double rr = L.tot[cc], rt = L.tot[NR + cc], tt = L.tot[2 * NR + cc];
            L.its[cc] += 1;
            if (rr <= L.rtol2 * L.yy[cc]) {
              L.act_in[cc] = 0;
              L.in_status[cc] = 0;
            } else if (L.its[cc] >= cap) {
              L.act_in[cc] = 0;
              L.in_status[cc] = 1;
            } else if (!(fabs(rt) > eps * sqrt(rr) * sqrt(tt))) {
              L.act_in[cc] = 0;
              L.in_status[cc] = 3;
            } else {
              const double beta = rt / L.rho[cc];
              L.beta[cc] = beta;
              L.rho[cc] = rt;
              for (int j = 0; j < KB; ++j) {
                const double vtj = L.vt[j][cc] - L.alpha[cc] * L.wv[j][cc];
                const double sj = vtj + beta * L.s[j][cc];
                L.vt[j][cc] = vtj;
                L.s[j][cc] = sj;
                L.csv[j][cc] = j < k ? S.c[j] * sj : 0.0;
                L.csvf[j][cc] = (float)L.csv[j][cc];
              }
            }
          }
        }
        if (threadIdx.x == 0) {
          int any = 0;
          for (int cc = 0; cc < NR; ++cc) any |= L.act_in[cc];
          L.any = any;
        }
        __syncthreads();
      }
      if (!L.any) break;
      // C: p = t + beta p (active columns); periodic direct refresh of s, vt
      {
        const bool act = L.act_in[c] != 0;
        const T beta = (T)L.beta[c];
        const bool refresh = k > 0 && (it % kRefresh) == kRefresh - 1;
        T as[KB], at[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) { as[j] = 0; at[j] = 0; }
        if (!refresh && act) {
          // kRows rows per thread in flight, as in B
          for (int i0 = rstart; i0 < n; i0 += kRows * rstride) {
            T tv[kRows], pv[kRows];
#pragma unroll
            for (int u = 0; u < kRows; ++u) {
              const int i = min(i0 + u * rstride, n - 1);
              const size_t e = (size_t)i * NR + c;
              tv[u] = dinv[i] * r[e];
              pv[u] = p[e];
            }
#pragma unroll
            for (int u = 0; u < kRows; ++u) {
              const int i = i0 + u * rstride;
              if (i < n) p[(size_t)i * NR + c] = tv[u] + beta * pv[u];
            }
          }
        }
        for (int i = refresh ? rstart : n; i < n; i += rstride) {
          const size_t e = (size_t)i * NR + c;
          const T ti = dinv[i] * r[e];
          T pi = p[e];
          if (act) {
            pi = ti + beta * pi;
            p[e] = pi;
          }
          {
            const T *vb = VT + (size_t)(i / MCG_VBLK) * ((size_t)MCG_VBLK * k) + (i % MCG_VBLK);
#pragma unroll
            for (int j = 0; j < KB; ++j) {
              const T v = vb[(size_t)(j < k ? j : k - 1) * MCG_VBLK];
              as[j] += v * pi;
              at[j] += v * ti;
            }
          }
        }
        mark(4);
        if (refresh) {
          if (!team_allreduce_get<NR, KB, 2 * KB>(
                  [&](int e) { return e < KB ? (double)as[e < KB ? e : 0]
                                             : (double)at[e >= KB ? e - KB : 0]; },
                  L, S, P, lb))
            return false;
          if (threadIdx.x < NR) {
            const int cc = threadIdx.x;
            if (L.act_in[cc]) {
              for (int j = 0; j < KB; ++j) {
                const double sj = j < k ? L.tot[j * NR + cc] : 0.0;
                L.s[j][cc] = sj;
                L.vt[j][cc] = j < k ? L.tot[(KB + j) * NR + cc] : 0.0;
                L.csv[j][cc] = j < k ? S.c[j] * sj : 0.0;
                L.csvf[j][cc] = (float)L.csv[j][cc];
              }
            }
          }
          __syncthreads();
        } else {
          if (!team_barrier(S.bar, S.nteam, P.abort_flag, P.timeout_ticks)) return false;
        }
        mark(5);
      }
    }
    if (threadIdx.x < NR) L.inner_total[threadIdx.x] += L.its[threadIdx.x];
    __syncthreads();
    return true;
  };

  // ---- first inner solve on r1, beta1 ---------------------------------------
  if (ok) ok = inner_solve(r1);
  if (ok) {
    double a = 0.0;
    for (int i = rstart; i < n; i += rstride) {
      const size_t e = (size_t)i * NR + c;
      const double yi = L.scale[c] * (double)z[e];
      y[e] = yi;
      r2[e] = r1[e];
      a += r1[e] * yi;
    }
    double vv[1] = {a};
    ok = team_allreduce<NR, KB, 1>(vv, 1, L, S, P, lb);
    if (ok && threadIdx.x < NR) {
      const int cc = threadIdx.x;
      if (L.act_out[cc]) {
        const double b2 = L.tot[cc];
        if (L.in_status[cc] >= 3) {
          L.status[cc] = L.in_status[cc];
          L.act_out[cc] = 0;
        } else if (!(b2 > 0.0)) {
          L.status[cc] = 3;
          L.act_out[cc] = 0;
        } else {
          const double be = sqrt(b2);
          L.beta_cur[cc] = be;
          L.oldb[cc] = 0.0;
          L.dbar[cc] = 0.0;
          L.epsln[cc] = 0.0;
          L.phibar[cc] = be;
          L.cs[cc] = -1.0;
          L.sn[cc] = 0.0;
        }
      }
    }
    __syncthreads();
  }

  // ---- outer MINRES iterations ---------------------------------------------
  for (int itn = 1; ok && itn <= P.maxit_out; ++itn) {
    if (threadIdx.x == 0) {
      int any = 0;
      for (int cc = 0; cc < NR; ++cc) any |= L.act_out[cc];
      L.any = any;
    }
    __syncthreads();
    if (!L.any) break;
    const bool act = L.act_out[c] != 0;
    // L1: v = y / beta; r1 <- (A y)/beta - (beta/oldb) r1; alfa = v^T r1
    {
      const double beta = L.beta_cur[c];
      const double sc = act ? 1.0 / beta : 0.0;
      const double f = (itn == 1 || !act) ? 0.0 : beta / L.oldb[c];
      double a = 0.0;
      for (int i = rstart; i < n; i += rstride) {
        const double acc = csr_row_dot<NR, double>(ci, S.va, y, rp[i], rp[i + 1], c);
        const size_t e = (size_t)i * NR + c;
        if (act) {
          const double vi = sc * y[e];
          const double yi = sc * acc - f * r1[e];
          v[e] = vi;
          r1[e] = yi;
          a += vi * yi;
        }
      }
      double vv[1] = {a};
      if (!(ok = team_allreduce<NR, KB, 1>(vv, 1, L, S, P, lb))) break;
      if (threadIdx.x < NR) L.alfa[threadIdx.x] = L.tot[threadIdx.x];
      __syncthreads();
    }
    // L2: r1 -= (alfa/beta) r2; ||r1||^2 -> boundary scale
    {
      const double f = act ? L.alfa[c] / L.beta_cur[c] : 0.0;
      double a = 0.0;
      for (int i = rstart; i < n; i += rstride) {
        const size_t e = (size_t)i * NR + c;
        if (act) {
          const double yi = r1[e] - f * r2[e];
          r1[e] = yi;
          a += yi * yi;
        }
      }
      double vv[1] = {a};
      if (!(ok = team_allreduce<NR, KB, 1>(vv, 1, L, S, P, lb))) break;
      if (threadIdx.x < NR) {
        const int cc = threadIdx.x;
        const double s = sqrt(L.tot[cc]);
        L.scale[cc] = mixed ? s : 1.0;
        L.inv_scale[cc] = mixed ? (s > 0.0 ? 1.0 / s : 0.0) : 1.0;
      }
      __syncthreads();
    }
    {
      double *t_ = r1;
      r1 = r2;
      r2 = t_;
    }
    if (!(ok = inner_solve(r2))) break;
    // L3: y = scale z; beta^2 = r2^T y; Givens
    {
      double a = 0.0;
      for (int i = rstart; i < n; i += rstride) {
        const size_t e = (size_t)i * NR + c;
        if (act) {
          const double yi = L.scale[c] * (double)z[e];
          y[e] = yi;
          a += r2[e] * yi;
        }
      }
      double vv[1] = {a};
      if (!(ok = team_allreduce<NR, KB, 1>(vv, 1, L, S, P, lb))) break;
      if (threadIdx.x < NR) {
        const int cc = threadIdx.x;
        L.improved[cc] = 0;
        if (L.act_out[cc]) {
          const double b2 = L.tot[cc];
          if (L.in_status[cc] >= 3) {
            L.status[cc] = L.in_status[cc];
            L.act_out[cc] = 0;
            L.gamma[cc] = 1.0;
            L.phi[cc] = 0.0;
            L.oldeps[cc] = 0.0;
            L.delta[cc] = 0.0;
          } else if (!(b2 >= 0.0)) {
            L.status[cc] = 3;
            L.act_out[cc] = 0;
            L.gamma[cc] = 1.0;
            L.phi[cc] = 0.0;
            L.oldeps[cc] = 0.0;
            L.delta[cc] = 0.0;
          } else {
            const double be = sqrt(b2);
            L.oldb[cc] = L.beta_cur[cc];
            L.beta_cur[cc] = be;
            const double alfa = L.alfa[cc], cs = L.cs[cc], sn = L.sn[cc], dbar = L.dbar[cc];
            L.oldeps[cc] = L.epsln[cc];
            L.delta[cc] = cs * dbar + sn * alfa;
            const double gbar = sn * dbar - cs * alfa;
            L.epsln[cc] = sn * be;
            L.dbar[cc] = -cs * be;
            double gamma = hypot(gbar, be);
            if (gamma < 2.220446049250313e-16) gamma = 2.220446049250313e-16;
            L.gamma[cc] = gamma;
            L.cs[cc] = gbar / gamma;
            L.sn[cc] = be / gamma;
            L.phi[cc] = L.cs[cc] * L.phibar[cc];
            L.phibar[cc] = L.sn[cc] * L.phibar[cc];
          }
        }
      }
      __syncthreads();
    }
    // L4: w = (v - oldeps w1 - delta w2)/gamma; x += phi w
    {
      double *t_ = w1;
      w1 = w2;
      w2 = w;
      w = t_;
      const bool act2 = L.act_out[c] != 0;
      const double oldeps = L.oldeps[c], delta = L.delta[c], ig = 1.0 / L.gamma[c], phi = L.phi[c];
      for (int i = rstart; i < n; i += rstride) {
        const size_t e = (size_t)i * NR + c;
        if (act2) {
          const double wi = (v[e] - oldeps * w1[e] - delta * w2[e]) * ig;
          w[e] = wi;
          x[e] += phi * wi;
        }
      }
      if (!(ok = team_barrier(S.bar, S.nteam, P.abort_flag, P.timeout_ticks))) break;
    }
    // L5: rt = b - A x; ||rt||^2; stop tests
    {
      double a = 0.0;
      for (int i = rstart; i < n; i += rstride) {
        const double acc = csr_row_dot<NR, double>(ci, S.va, x, rp[i], rp[i + 1], c);
        const size_t e = (size_t)i * NR + c;
        const double ri = b[e] - acc;
        a += ri * ri;
      }
      double vv[1] = {a};
      if (!(ok = team_allreduce<NR, KB, 1>(vv, 1, L, S, P, lb))) break;
      if (threadIdx.x < NR) {
        const int cc = threadIdx.x;
        if (L.act_out[cc] || L.status[cc] >= 3) {
          // columns that ended in this iteration by a breakdown still count it
        }
        if (L.act_out[cc]) {
          const double rn = sqrt(L.tot[cc]);
          L.rnorm[cc] = rn;
          L.outer_its[cc] = itn;
          if (rn < L.best[cc]) {
            L.since_best[cc] = (rn < L.best[cc] * (1.0 - 1e-3)) ? 0 : L.since_best[cc] + 1;
            L.best[cc] = rn;
            L.improved[cc] = 1;
          } else {
            L.since_best[cc] += 1;
          }
          if (rn <= P.rtol_out * L.bnorm[cc]) {
            L.status[cc] = 0;
            L.act_out[cc] = 0;
          } else if (!(rn == rn)) {
            L.status[cc] = 3;
            L.act_out[cc] = 0;
          } else if (P.stag_window > 0 && L.since_best[cc] >= P.stag_window) {
            L.status[cc] = 2;
            L.act_out[cc] = 0;
          } else if (L.beta_cur[cc] == 0.0) {
            L.status[cc] = 3;
            L.act_out[cc] = 0;
          }
        }
      }
      __syncthreads();
    }
    // L6: xbest <- x for improved columns (rows owned by this thread only)
    if (L.improved[c])
      for (int i = rstart; i < n; i += rstride) {
        const size_t e = (size_t)i * NR + c;
        S.xbest[e] = x[e];
      }
  }
  if (!ok) {
    if (lb == 0 && threadIdx.x < NR) out[(size_t)sid * NR + threadIdx.x].status = -2;
    if (lb == 0 && threadIdx.x == 0) {
      P.prof[kProfPerSys * (size_t)sid + 1] = wall_clock64();
      P.prof[kProfPerSys * (size_t)sid + 2] = L.team_its;
    }
    return;
  }
  // final: non-converged columns return their best iterate
  const bool restore = P.keep_best && L.status[c] != 0;
  if (restore)
    for (int i = rstart; i < n; i += rstride) {
      const size_t e = (size_t)i * NR + c;
      x[e] = S.xbest[e];
    }
  if (lb == 0 && threadIdx.x < NR) {
    const int cc = threadIdx.x;
    BOut o;
    o.status = L.status[cc];
    o.outer_its = L.outer_its[cc];
    o.inner_its = L.inner_total[cc];
    const double rn = (P.keep_best && L.status[cc] != 0) ? L.best[cc] : L.rnorm[cc];
    o.bnorm = L.bnorm[cc];
    o.relres = L.bnorm[cc] > 0.0 ? rn / L.bnorm[cc] : 0.0;
    out[(size_t)sid * NR + cc] = o;
  }
  if (lb == 0 && threadIdx.x == 0) {
    P.prof[kProfPerSys * (size_t)sid + 1] = wall_clock64();
    P.prof[kProfPerSys * (size_t)sid + 2] = L.team_its;
    for (int q = 0; q < 6; ++q) P.prof[kProfPerSys * (size_t)sid + 3 + q] = L.ph[q];
  }
}

// column-major (n x nrhs, caller layout) <-> row-interleaved (n x NR)
__global__ void k_interleave(int n, int nrhs, int NR, const double *__restrict__ cm,
                             double *__restrict__ ri) {
  const int64_t total = (int64_t)n * NR;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / NR), cc = (int)(e % NR);
    ri[e] = cc < nrhs ? cm[(size_t)cc * n + i] : 0.0;
  }
}

__global__ void k_deinterleave(int n, int nrhs, int NR, const double *__restrict__ ri,
                               double *__restrict__ cm) {
  const int64_t total = (int64_t)n * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int cc = (int)(e / n), i = (int)(e % n);
    cm[e] = ri[(size_t)i * NR + cc];
  }
}

__global__ void k_zero_u32(int n, unsigned *p) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

int nr_bucket(int nrhs) { return nrhs <= 1 ? 1 : nrhs <= 2 ? 2 : nrhs <= 4 ? 4 : 8; }
int kb_bucket_batch(int k) {
  return k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : k <= 40 ? 40 : k <= 48 ? 48 : 64;
}

}  // namespace

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
// Systems are grouped by their k bucket; each group is one persistent launch
// compiled for that bucket (register arrays sized by the group's k, not the
// batch's largest), and the launches follow each other on the stream.
struct BGroup {
  int KB = 8;
  int nblocks = 0;
  int cap = 0;                   // blocks of this kernel the GPU holds at once
  std::vector<int> members;      // systems of the group
  int32_t *block_sys = nullptr;  // device: system of each block of the launch (cap entries)
};

struct mcg_batch {
  int nsys = 0, nrhs = 0, NR = 1, KB = 8, precision = 0, nblocks = 0, ncu = 0;
  std::vector<double> work;      // nnz + n (1 + k) per system
  std::vector<int> rows, ks, team, team0;
  std::vector<BGroup> groups;
  mcg_options_t opt{};
  std::vector<mcg_handle_t> solvers;   // owns A, Vhat, FP32 shadows per system
  std::vector<mcg_precond_t> jacobi;   // diag^{-1} per system
  std::vector<BSys> hsys;
  BSys *dsys = nullptr;
  BOut *dout = nullptr;
  unsigned *abort_flag = nullptr;
  unsigned *bars = nullptr;
  int64_t *prof = nullptr;  // kProfPerSys per system, written by the persistent launches
  std::vector<int> prof_team;  // team sizes of the last persistent solve (empty: none yet)
  double *part = nullptr;
  std::vector<void *> owned;
  int pw = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<const void *> graph_key;
  double graph_params[2] = {0.0, 0.0};
  int64_t graph_iparams[2] = {0, 0};
};

static void batch_free(mcg_batch *B) {
  if (!B) return;
  if (B->graph_exec) (void)hipGraphExecDestroy(B->graph_exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  for (auto p : B->jacobi) minres_cg_precond_free(p);
  for (auto h : B->solvers) minres_cg_free(h);
  for (void *p : B->owned) (void)hipFree(p);
  delete B;
}

extern "C" void minres_cg_batch_free(mcg_batch_t B) { batch_free(B); }

template <typename T, int NR, int KB>
static const void *batch_kernel() {
  return (const void *)&k_batched_minres_cg<T, NR, KB>;
}

template <typename T>
static const void *pick_kernel(int NR, int KB) {
#define KSEL(NRV)                                              \
  case NRV:                                                    \
    switch (KB) {                                              \
      case 8: return batch_kernel<T, NRV, 8>();                \
      case 16: return batch_kernel<T, NRV, 16>();              \
      case 32: return batch_kernel<T, NRV, 32>();              \
      case 40: return batch_kernel<T, NRV, 40>();              \
      case 48: return batch_kernel<T, NRV, 48>();              \
      default: return batch_kernel<T, NRV, 64>();              \
    }
  switch (NR) {
    KSEL(1)
    KSEL(2)
    KSEL(4)
    default:
    KSEL(8)
  }
#undef KSEL
}

// Team sizes: within each group, blocks in proportion to weight[i] (at least
// one, at most one block per 256 / NR rows of the system), within the
// group's resident blocks; teams laid out one after another.
static void plan_teams(mcg_batch *B, const std::vector<double> &weight) {
  B->team.assign(B->nsys, 1);
  B->team0.assign(B->nsys, 0);
  for (BGroup &G : B->groups) {
    const int ng = (int)G.members.size();
    const int target = std::min(G.cap, std::max(ng, 4 * B->ncu));
    double wsum = 0.0;
    for (int i : G.members) wsum += weight[i];
    int total = 0;
    for (int i : G.members) {
      const int rows_passes = std::max(1, (B->rows[i] + BB / B->NR - 1) / (BB / B->NR));
      B->team[i] =
          std::max(1, std::min(rows_passes, (int)std::floor(target * weight[i] / wsum)));
      total += B->team[i];
    }
    while (total > G.cap) {  // shrink the largest teams
      int jbest = G.members[0];
      for (int i : G.members)
        if (B->team[i] > B->team[jbest]) jbest = i;
      if (B->team[jbest] == 1) break;
      --B->team[jbest];
      --total;
    }
    int t = 0;
    for (int i : G.members) {
      B->team0[i] = t;
      t += B->team[i];
    }
    G.nblocks = total;
  }
}

// Teams for measured block-times w[i] (span x team size of a solve): each
// launch's blocks handed out one at a time to the team whose predicted span
// w[i] / team[i] is the longest (at most one block per 64 / NR rows), the
// integer allocation that minimises the launch's longest predicted span.
static void plan_teams_makespan(mcg_batch *B, const std::vector<double> &w) {
  B->team.assign(B->nsys, 1);
  B->team0.assign(B->nsys, 0);
  for (BGroup &G : B->groups) {
    const int ng = (int)G.members.size();
    const int target = std::min(G.cap, std::max(ng, 4 * B->ncu));
    std::priority_queue<std::pair<double, int>> q;  // (predicted span, system)
    for (int i : G.members) q.push({w[i], i});
    int total = ng;
    while (total < target && !q.empty()) {
      const int i = q.top().second;
      q.pop();
      const int rows_passes = std::max(1, (B->rows[i] + BB / B->NR - 1) / (BB / B->NR));
      if (B->team[i] >= rows_passes) continue;  // no more rows to hand out
      ++B->team[i];
      ++total;
      q.push({w[i] / B->team[i], i});
    }
    int t = 0;
    for (int i : G.members) {
      B->team0[i] = t;
      t += B->team[i];
    }
    G.nblocks = total;
  }
}

// Copy the team layout to the systems' descriptors and the groups' block
// tables on the device (synchronous; no launch of the batch may be running).
static int upload_teams(mcg_batch *B) {
  int total = 0;
  for (const BGroup &G : B->groups) total += G.nblocks;
  B->nblocks = total;
  for (int i = 0; i < B->nsys; ++i) {
    BSys &S = B->hsys[i];
    S.team0 = B->team0[i];
    S.nteam = B->team[i];
    // launches of different groups run one after the other on the stream,
    // so their teams may share the partials buffer
    S.part = B->part + 2 * (size_t)B->team0[i] * B->pw;
  }
  HIP_TRY_B(hipMemcpy(B->dsys, B->hsys.data(), sizeof(BSys) * B->nsys, hipMemcpyHostToDevice));
  for (const BGroup &G : B->groups) {
    std::vector<int32_t> bsys(G.nblocks);
    for (int i : G.members)
      for (int b = 0; b < B->team[i]; ++b) bsys[B->team0[i] + b] = i;
    HIP_TRY_B(hipMemcpy(G.block_sys, bsys.data(), sizeof(int32_t) * G.nblocks,
                        hipMemcpyHostToDevice));
  }
  return MCG_OK;
}

extern "C" int minres_cg_batch_create(mcg_batch_t *out, int32_t nsys, const mcg_csr_t *As,
                                      const int32_t *ks, const double *const *Vhats,
                                      const double *const *lams, int32_t nrhs,
                                      const mcg_options_t *opt, void *stream) {
  if (!out || nsys <= 0 || !As || !ks || nrhs < 1 || nrhs > 8) return MCG_EINVAL;
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  mcg_batch *B = new mcg_batch();
  if (opt) B->opt = *opt; else minres_cg_default_options(&B->opt);
  B->nsys = nsys;
  B->nrhs = nrhs;
  B->NR = nr_bucket(nrhs);
  B->precision = B->opt.precision;
  int kmax = 1;
  for (int i = 0; i < nsys; ++i) {
    if (ks[i] < 0 || ks[i] > kBatchKMax) { batch_free(B); return MCG_EINVAL; }
    kmax = std::max(kmax, ks[i]);
  }
  B->KB = kb_bucket_batch(kmax);
  mcg_options_t so = B->opt;
  so.autotune = 0;
  so.profile = 0;
  // the per-system handles also serve the stream-parallel mode (sliced ELL
  // copies and the one-pass M_mr apply chosen as for a single system)
  // per-system solver handles: validated copies of A, Vhat, FP32 shadows, workspaces
  for (int i = 0; i < nsys; ++i) {
    mcg_handle_t h = nullptr;
    int rc = minres_cg_create(&h, &As[i], ks[i], ks[i] ? Vhats[i] : nullptr,
                              ks[i] ? lams[i] : nullptr, &so, stream);
    if (rc) { batch_free(B); return rc; }
    B->solvers.push_back(h);
    mcg_precond_t pc = nullptr;
    rc = minres_cg_precond_create(&pc, h, MCG_PC_JACOBI, nullptr, stream);
    if (rc) { batch_free(B); return rc; }
    B->jacobi.push_back(pc);
  }
  // groups by k bucket, each with the blocks the GPU holds at once for its
  // kernel; team sizes within a group in proportion to (nnz + k n)
  int dev = 0, ncu = 0;
  HIP_TRY_B(hipGetDevice(&dev));
  HIP_TRY_B(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const bool mixed = B->precision == MCG_PREC_MIXED;
  B->ncu = ncu;
  B->work.resize(nsys);
  B->rows.resize(nsys);
  B->ks.resize(nsys);
  for (int i = 0; i < nsys; ++i) {
    B->work[i] = (double)As[i].nnz + (double)As[i].n * (1.0 + ks[i]);
    B->rows[i] = As[i].n;
    B->ks[i] = ks[i];
  }
  int max_cap = 0;
  for (int kb : {8, 16, 32, 40, 48, 64}) {
    std::vector<int> sys;
    for (int i = 0; i < nsys; ++i)
      if (kb_bucket_batch(std::max(1, ks[i])) == kb) sys.push_back(i);
    if (sys.empty()) continue;
    const void *kfn = mixed ? pick_kernel<float>(B->NR, kb) : pick_kernel<double>(B->NR, kb);
    int per_cu = 0;
    HIP_TRY_B(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, BB, 0));
    if (per_cu <= 0) { batch_free(B); return MCG_EHIP; }
    BGroup G;
    G.KB = kb;
    G.cap = per_cu * ncu;
    G.members = sys;
    if ((int)sys.size() > G.cap) { batch_free(B); return MCG_EINVAL; }
    max_cap = std::max(max_cap, G.cap);
    B->groups.push_back(G);
  }
  plan_teams(B, B->work);
  // buffers
  const size_t es = mixed ? sizeof(float) : sizeof(double);
  const int NR = B->NR;
  B->pw = (1 + 2 * B->KB) * NR + 3 * NR + 8;
  auto dmalloc = [&](void **p, size_t bytes) -> int {
    HIP_TRY_B(hipMalloc(p, std::max<size_t>(bytes, 8)));
    B->owned.push_back(*p);
    return MCG_OK;
  };
  int rc;
  if ((rc = dmalloc((void **)&B->dsys, sizeof(BSys) * nsys)) ||
      (rc = dmalloc((void **)&B->dout, sizeof(BOut) * nsys * NR)) ||
      (rc = dmalloc((void **)&B->abort_flag, 64)) ||
      (rc = dmalloc((void **)&B->prof, sizeof(int64_t) * kProfPerSys * nsys)) ||
      (rc = dmalloc((void **)&B->bars, sizeof(unsigned) * 2 * nsys)) ||
      (rc = dmalloc((void **)&B->part, sizeof(double) * 2 * (size_t)max_cap * B->pw))) {
    batch_free(B);
    return rc;
  }
  for (BGroup &G : B->groups)
    if ((rc = dmalloc((void **)&G.block_sys, sizeof(int32_t) * G.cap))) {
      batch_free(B);
      return rc;
    }
  B->hsys.resize(nsys);
  for (int i = 0; i < nsys; ++i) {
    mcg_solver *h = B->solvers[i];
    BSys &S = B->hsys[i];
    std::memset(&S, 0, sizeof(S));
    S.n = h->n;
    S.k = h->k;
    S.rp = h->rp;
    S.ci = h->ci;
    S.va = h->va;
    S.vaT = mixed ? (const void *)h->va32 : (const void *)h->va;
    S.VT = mixed ? (const void *)h->V32 : (const void *)h->V;
    S.dinvT = mixed ? (const void *)B->jacobi[i]->dinv32 : (const void *)B->jacobi[i]->dinv64;
    std::vector<double> lam(h->k);
    if (h->k) HIP_TRY_B(hipMemcpy(lam.data(), lams[i], sizeof(double) * h->k, hipMemcpyDeviceToHost));
    for (int j = 0; j < h->k; ++j) S.c[j] = 2.0 * std::fabs(lam[j]);
    const size_t nv = (size_t)h->n * NR;
    double **d64[] = {(double **)&S.b, &S.x, &S.r1, &S.r2, &S.y, &S.v, &S.w, &S.w1, &S.w2, &S.rt,
                      &S.xbest};
    for (double **pp : d64)
      if ((rc = dmalloc((void **)pp, sizeof(double) * nv))) { batch_free(B); return rc; }
    void **dT[] = {&S.z, &S.r, &S.p, &S.q};
    for (void **pp : dT)
      if ((rc = dmalloc(pp, es * nv))) { batch_free(B); return rc; }
    S.bar = B->bars + 2 * i;
  }
  if ((rc = upload_teams(B))) { batch_free(B); return rc; }
  // no persistent solve yet: the timing reads as zeros
  if (hipMemsetAsync(B->prof, 0, sizeof(int64_t) * kProfPerSys * nsys, s) != hipSuccess) {
    batch_free(B);
    return MCG_EHIP;
  }
  HIP_TRY_B(hipStreamSynchronize(s));
  *out = B;
  return MCG_OK;
}

extern "C" int minres_cg_create_batch(mcg_batch_t *out, int32_t nsys, const mcg_csr_t *As,
                                      const int32_t *ks, const double *const *Vhats,
                                      const double *const *lams, int32_t nrhs,
                                      const mcg_options_t *opt, void *stream) {
  return minres_cg_batch_create(out, nsys, As, ks, Vhats, lams, nrhs, opt, stream);
}

// Enqueue one whole batched solve on s (data movement + the persistent kernel).
static int batch_enqueue(mcg_batch *B, const double *const *Bs, double *const *Xs, double rtol_out,
                         double rtol_in, int32_t maxit_out, int64_t maxit_in, hipStream_t s) {
  const int NR = B->NR;
  for (int i = 0; i < B->nsys; ++i) {
    const BSys &S = B->hsys[i];
    const int g = std::max(1, std::min(1024, (int)(((int64_t)S.n * NR + 255) / 256)));
    k_interleave<<<g, 256, 0, s>>>(S.n, B->nrhs, NR, Bs[i], (double *)S.b);
    k_interleave<<<g, 256, 0, s>>>(S.n, B->nrhs, NR, Xs[i], S.x);
  }
  k_zero_u32<<<1, 256, 0, s>>>(2 * B->nsys, B->bars);
  k_zero_u32<<<1, 64, 0, s>>>(16, B->abort_flag);
  BParams P;
  P.rtol_out = rtol_out;
  P.rtol_in = rtol_in;
  P.maxit_out = maxit_out;
  P.maxit_in = maxit_in;
  P.stag_window = B->opt.stag_window;
  P.keep_best = B->opt.keep_best;
  P.pw = B->pw;
  P.abort_flag = B->abort_flag;
  P.timeout_ticks = (int64_t)100000000 * 20;  // 20 s at the 100 MHz wall clock
  P.prof = B->prof;
  const bool mixed = B->precision == MCG_PREC_MIXED;
  for (BGroup &G : B->groups) {
    const void *kfn = mixed ? pick_kernel<float>(NR, G.KB) : pick_kernel<double>(NR, G.KB);
    void *args[] = {(void *)&B->dsys, (void *)&G.block_sys, (void *)&P, (void *)&B->dout};
    HIP_TRY_B(hipLaunchKernel(kfn, dim3(G.nblocks), dim3(BB), args, 0, s));
  }
  for (int i = 0; i < B->nsys; ++i) {
    const BSys &S = B->hsys[i];
    const int g = std::max(1, std::min(1024, (int)(((int64_t)S.n * B->nrhs + 255) / 256)));
    k_deinterleave<<<g, 256, 0, s>>>(S.n, B->nrhs, NR, S.x, Xs[i]);
  }
  return MCG_OK;
}

extern "C" int minres_cg_batch_solve(mcg_batch_t B, const double *const *Bs, double *const *Xs,
                                     double rtol_out, double rtol_in, int32_t maxit_out,
                                     int64_t maxit_inner, int32_t use_graph, mcg_batch_stats_t *st,
                                     void *stream) {
  if (!B || !Bs || !Xs || !(rtol_out >= 0.0) || !(rtol_in >= 0.0) || maxit_out < 0 ||
      maxit_inner < 0)
    return MCG_EINVAL;
  for (int i = 0; i < B->nsys; ++i)
    if (!Bs[i] || !Xs[i]) return MCG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if (use_graph) {
    // one graph per (B, X) pointer set: captured on first use, replayed after
    std::vector<const void *> key;
    for (int i = 0; i < B->nsys; ++i) {
      key.push_back(Bs[i]);
      key.push_back(Xs[i]);
    }
    const bool same = B->graph_exec && B->graph_key == key;
    if (!same) {
      if (B->graph_exec) { (void)hipGraphExecDestroy(B->graph_exec); B->graph_exec = nullptr; }
      if (B->graph) { (void)hipGraphDestroy(B->graph); B->graph = nullptr; }
      hipStream_t cs;
      HIP_TRY_B(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      HIP_TRY_B(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      rc = batch_enqueue(B, Bs, Xs, rtol_out, rtol_in, maxit_out, maxit_inner, cs);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(cs, &g);
      (void)hipStreamDestroy(cs);
      if (rc) return rc;
      HIP_TRY_B(e);
      B->graph = g;
      HIP_TRY_B(hipGraphInstantiate(&B->graph_exec, g, nullptr, nullptr, 0));
      B->graph_key = key;
      B->graph_params[0] = rtol_out;
      B->graph_params[1] = rtol_in;
      B->graph_iparams[0] = maxit_out;
      B->graph_iparams[1] = maxit_inner;
    } else if (B->graph_params[0] != rtol_out || B->graph_params[1] != rtol_in ||
               B->graph_iparams[0] != maxit_out || B->graph_iparams[1] != maxit_inner) {
      return MCG_EINVAL;  // a captured graph replays the parameters it was captured with
    }
    HIP_TRY_B(hipGraphLaunch(B->graph_exec, s));
  } else {
    if ((rc = batch_enqueue(B, Bs, Xs, rtol_out, rtol_in, maxit_out, maxit_inner, s))) return rc;
  }
  B->prof_team = B->team;  // what the profile's team clocks were measured with
  unsigned abort_h = 0;
  HIP_TRY_B(hipMemcpyAsync(&abort_h, B->abort_flag, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  std::vector<BOut> o((size_t)B->nsys * B->NR);
  HIP_TRY_B(hipMemcpyAsync(o.data(), B->dout, sizeof(BOut) * o.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY_B(hipStreamSynchronize(s));
  if (abort_h) return MCG_EHIP;
  int worst = MCG_OK;
  for (int i = 0; i < B->nsys; ++i)
    for (int c = 0; c < B->nrhs; ++c) {
      const BOut &b = o[(size_t)i * B->NR + c];
      if (st) {
        const size_t e = (size_t)i * B->nrhs + c;
        if (st->status) st->status[e] = b.status;
        if (st->outer_its) st->outer_its[e] = b.outer_its;
        if (st->inner_its) st->inner_its[e] = b.inner_its;
        if (st->relres) st->relres[e] = b.relres;
      }
      if (b.status < 0) return b.status == -1 ? MCG_EINVAL : MCG_EHIP;
      worst = std::max(worst, (int)b.status);
    }
  return worst;
}

// The stream-parallel solve with per-system second levels (pcs[i], or the
// batch's Jacobi where pcs is NULL or pcs[i] is NULL).
static int solve_streams_impl(mcg_batch_t B, const mcg_precond_t *pcs, const double *const *Bs,
                              double *const *Xs, double rtol_out, double rtol_in,
                              int32_t maxit_out, int64_t maxit_inner, int32_t nstreams,
                              mcg_batch_stats_t *st, void *stream) {
  if (!B || !Bs || !Xs || !(rtol_out >= 0.0) || !(rtol_in >= 0.0) || maxit_out < 0 ||
      maxit_inner < 0 || nstreams < 1 || nstreams > 16)
    return MCG_EINVAL;
  for (int i = 0; i < B->nsys; ++i) {
    if (!Bs[i] || !Xs[i]) return MCG_EINVAL;
    if (pcs && pcs[i] && pcs[i]->h != B->solvers[i]) return MCG_EINVAL;
  }
  int dev = 0;
  HIP_TRY_B(hipGetDevice(&dev));
  // work queued on the caller's stream (inputs being written) comes first
  hipEvent_t ready;
  HIP_TRY_B(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  HIP_TRY_B(hipEventRecord(ready, (hipStream_t)stream));
  // longest-processing-time assignment of systems to streams
  std::vector<int> order(B->nsys);
  std::vector<double> work(B->nsys);
  for (int i = 0; i < B->nsys; ++i) {
    const mcg_solver *h = B->solvers[i];
    order[i] = i;
    work[i] = ((double)h->nnz + (double)h->n * (h->k + 1)) * B->nrhs;
  }
  std::sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  const int ns = std::min<int>(nstreams, B->nsys);
  std::vector<std::vector<int>> lists(ns);
  std::vector<double> load(ns, 0.0);
  for (int i : order) {
    const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lists[w].push_back(i);
    load[w] += work[i];
  }
  const size_t nout = (size_t)B->nsys * B->nrhs;
  std::vector<int32_t> status(nout, 0), outer(nout, 0);
  std::vector<int64_t> inner(nout, 0);
  std::vector<double> relres(nout, 0.0);
  std::vector<int> rcs(ns, MCG_OK);
  auto worker = [&](int w) {
    int rc = MCG_OK;
    hipStream_t ws = nullptr;
    if (hipSetDevice(dev) != hipSuccess ||
        hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess ||
        hipStreamWaitEvent(ws, ready, 0) != hipSuccess) {
      rcs[w] = MCG_EHIP;
      if (ws) (void)hipStreamDestroy(ws);
      return;
    }
    for (int i : lists[w]) {
      mcg_solver *h = B->solvers[i];
      for (int c = 0; c < B->nrhs && rc >= 0; ++c) {
        mcg_stats_t so;
        std::memset(&so, 0, sizeof so);
        mcg_precond_t pc = (pcs && pcs[i]) ? pcs[i] : B->jacobi[i];
        const int r = minres_cg_solve(h, pc, Bs[i] + (size_t)c * h->n,
                                      Xs[i] + (size_t)c * h->n, 1, rtol_out, rtol_in, maxit_out,
                                      maxit_inner, &so, ws);
        const size_t e = (size_t)i * B->nrhs + c;
        if (r < 0) {
          rc = r;
          break;
        }
        status[e] = so.status;
        outer[e] = so.outer_its;
        inner[e] = so.inner_its_total;
        relres[e] = so.final_relres;
      }
    }
    (void)hipStreamDestroy(ws);
    rcs[w] = rc;
  };
  std::vector<std::thread> threads;
  for (int w = 1; w < ns; ++w) threads.emplace_back(worker, w);
  worker(0);
  for (auto &t : threads) t.join();
  (void)hipEventDestroy(ready);
  for (int w = 0; w < ns; ++w)
    if (rcs[w] < 0) return rcs[w];
  int worst = MCG_OK;
  for (size_t e = 0; e < nout; ++e) {
    if (st) {
      if (st->status) st->status[e] = status[e];
      if (st->outer_its) st->outer_its[e] = outer[e];
      if (st->inner_its) st->inner_its[e] = inner[e];
      if (st->relres) st->relres[e] = relres[e];
    }
    worst = std::max(worst, (int)status[e]);
  }
  return worst;
}

extern "C" int minres_cg_batch_solve_streams(mcg_batch_t B, const double *const *Bs,
                                             double *const *Xs, double rtol_out, double rtol_in,
                                             int32_t maxit_out, int64_t maxit_inner,
                                             int32_t nstreams, mcg_batch_stats_t *st,
                                             void *stream) {
  return solve_streams_impl(B, nullptr, Bs, Xs, rtol_out, rtol_in, maxit_out, maxit_inner,
                            nstreams, st, stream);
}

extern "C" int minres_cg_batch_solve_streams_pc(mcg_batch_t B, const mcg_precond_t *pcs,
                                                const double *const *Bs, double *const *Xs,
                                                double rtol_out, double rtol_in,
                                                int32_t maxit_out, int64_t maxit_inner,
                                                int32_t nstreams, mcg_batch_stats_t *st,
                                                void *stream) {
  if (!pcs) return MCG_EINVAL;
  return solve_streams_impl(B, pcs, Bs, Xs, rtol_out, rtol_in, maxit_out, maxit_inner, nstreams,
                            st, stream);
}

extern "C" int minres_cg_batch_system(mcg_batch_t B, int32_t i, mcg_handle_t *h) {
  if (!B || !h || i < 0 || i >= B->nsys) return MCG_EINVAL;
  *h = B->solvers[i];
  return MCG_OK;
}

extern "C" int minres_cg_batch_rebalance(mcg_batch_t B, const double *weights) {
  if (!B || !weights) return MCG_EINVAL;
  double wmax = 0.0;
  for (int i = 0; i < B->nsys; ++i) {
    if (!(weights[i] > 0.0) || !std::isfinite(weights[i])) return MCG_EINVAL;
    wmax = std::max(wmax, weights[i]);
  }
  // scaled by the largest weight, so that no product overflows
  std::vector<double> w(B->nsys);
  for (int i = 0; i < B->nsys; ++i) w[i] = B->work[i] * (weights[i] / wmax);
  plan_teams(B, w);
  const int rc = upload_teams(B);
  if (rc) return rc;
  // a captured graph holds the old grid sizes
  if (B->graph_exec) { (void)hipGraphExecDestroy(B->graph_exec); B->graph_exec = nullptr; }
  if (B->graph) { (void)hipGraphDestroy(B->graph); B->graph = nullptr; }
  B->graph_key.clear();
  return MCG_OK;
}

extern "C" int minres_cg_batch_rebalance_measured(mcg_batch_t B) {
  if (!B) return MCG_EINVAL;
  if (B->prof_team.size() != (size_t)B->nsys) return MCG_EINVAL;  // no persistent solve yet
  std::vector<int64_t> h(kProfPerSys * (size_t)B->nsys);
  HIP_TRY_B(hipMemcpy(h.data(), B->prof, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost));
  // block-time each system took: its team's span times its team size
  std::vector<double> w(B->nsys);
  for (int i = 0; i < B->nsys; ++i) {
    const int64_t *q = h.data() + kProfPerSys * (size_t)i;
    if (q[0] <= 0 || q[1] < q[0]) return MCG_EINVAL;  // no clocks for this team
    // a team that ended within a tick (nothing to iterate) counts one tick
    const double span = (double)std::max<int64_t>(1, q[1] - q[0]);
    w[i] = span * B->prof_team[i];
  }
  plan_teams_makespan(B, w);
  const int rc = upload_teams(B);
  if (rc) return rc;
  if (B->graph_exec) { (void)hipGraphExecDestroy(B->graph_exec); B->graph_exec = nullptr; }
  if (B->graph) { (void)hipGraphDestroy(B->graph); B->graph = nullptr; }
  B->graph_key.clear();
  return MCG_OK;
}

extern "C" int minres_cg_batch_profile(mcg_batch_t B, int64_t *t_begin, int64_t *t_end,
                                       int64_t *team_iters, int64_t *phase_ticks, int32_t *group,
                                       double *clock_hz) {
  if (!B) return MCG_EINVAL;
  std::vector<int64_t> h(kProfPerSys * (size_t)B->nsys);
  HIP_TRY_B(hipMemcpy(h.data(), B->prof, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost));
  for (int i = 0; i < B->nsys; ++i) {
    const int64_t *q = h.data() + kProfPerSys * (size_t)i;
    if (t_begin) t_begin[i] = q[0];
    if (t_end) t_end[i] = q[1];
    if (team_iters) team_iters[i] = q[2];
    if (phase_ticks)
      for (int j = 0; j < 6; ++j) phase_ticks[6 * (size_t)i + j] = q[3 + j];
  }
  if (group)
    for (size_t g = 0; g < B->groups.size(); ++g)
      for (int i : B->groups[g].members) group[i] = (int32_t)g;
  if (clock_hz) {
    int dev = 0, khz = 0;
    HIP_TRY_B(hipGetDevice(&dev));
    HIP_TRY_B(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    *clock_hz = 1e3 * khz;
  }
  return MCG_OK;
}

extern "C" int minres_cg_batch_info(mcg_batch_t B, int32_t *nblocks, int32_t *team_sizes) {
  if (!B) return MCG_EINVAL;
  if (nblocks) *nblocks = B->nblocks;
  if (team_sizes)
    for (int i = 0; i < B->nsys; ++i) team_sizes[i] = B->hsys[i].nteam;
  return MCG_OK;
}
