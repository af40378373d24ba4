// Device kernels of the MINRES-CG hot path for CDNA4 (gfx950, wave64).
//
// Layout: CSR with int32 indices; dense vectors contiguous; Vhat n x k
// column-major.  Every kernel runs 256-thread blocks (4 waves) over a
// grid-stride loop of 256-row tiles.  Reductions are deterministic: each
// block reduces its values with wave shuffles and LDS and writes one partial
// per value.  Inside the CG iteration the kernel that consumes a scalar sums
// the producer's partials itself, in block order, at its start (so no
// separate reduction launch sits between two steps); the outer MINRES
// kernels and a few setup paths instead let the last block to arrive
// (atomic ticket + device-scope fences) sum the partials and update the
// solver scalars held in device memory (DevState).  No scalar leaves the GPU
// inside an iteration.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MCG_BLOCK 256
#define MCG_NWAVE (MCG_BLOCK / 64)
#define MCG_KMAX 64

// Solver scalars resident in device memory.  The first 32 bytes are what
// the host polls between chunks of inner iterations.
struct DevState {
  int32_t done;         // inner solve finished (any reason)
  int32_t status;       // inner status (mcg_status)
  int64_t its;          // inner iterations of the current inner solve
  int64_t maxit;        // cap of the current inner solve
  int32_t outer_flag;   // outer breakdown flag (beta^2 < 0, non-finite)
  int32_t pad0;
  // inner CG scalars
  double rho, alpha, beta, rr, yy, rtol2, pi, eps;
  // precision boundary (outer FP64 -> inner): r_in = y * inv_scale
  double scale, inv_scale;
  // outer MINRES scalars (Paige-Saunders recurrences)
  double alfa, beta_cur, oldb, dbar, epsln, oldeps, phibar, cs, sn, delta, gamma, phi, beta2;
  double rt2, bb;       // ||b - A x||^2, ||b||^2
  double rho_par[2];    // rho of the Jacobi iteration by parity: iteration it reads
                        // rho_par[it & 1] and its direction kernel writes the other
  double s[MCG_KMAX];   // Vhat^T p
  double cs_[MCG_KMAX]; // 2|lam_j| * s_j
  double c[MCG_KMAX];   // 2|lam_j|
  double smw[MCG_KMAX]; // -2 / lam_j   (MINRES-CG*)
  double u[MCG_KMAX];   // Vhat^T r    (MINRES-CG* scratch)
  double vt[MCG_KMAX];  // Vhat^T t, t = D^{-1} r   (diagonal M_cg recurrences)
  double w[MCG_KMAX];   // Vhat^T D^{-1} q
};

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-level sum of W per-thread values; thread j < w_used writes the
// block's total of value j to part[blockIdx.x * w_used + j].
// compact0 != nullptr: thread 0 also stores the block's total of value 0 at
// compact0[blockIdx.x] (a contiguous array that consumer kernels can sum
// from every block cheaply).
template <int W>
__device__ void block_partials(const double (&v)[W], int w_used, double *__restrict__ part,
                               double *__restrict__ compact0 = nullptr) {
  __shared__ double red[W * MCG_NWAVE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // all W sums unconditionally (independent shuffle chains the compiler can
  // interleave); values j >= w_used are ignored
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const double s = wave_sum(v[j]);
    if (lane == 0) red[j * MCG_NWAVE + wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < w_used) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < MCG_NWAVE; ++q) s += red[threadIdx.x * MCG_NWAVE + q];
    part[(size_t)blockIdx.x * w_used + threadIdx.x] = s;
    if (compact0 && threadIdx.x == 0) compact0[blockIdx.x] = s;
  }
}

// As block_partials for KB FP32 values (per-thread FP32 accumulations),
// summed across the wavefront in FP32 and across wavefronts in FP64.
template <int KB>
__device__ void block_partials_f(const float (&vf)[KB], int w_used, double *__restrict__ part) {
  __shared__ double red[KB * MCG_NWAVE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    float x = vf[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[j * MCG_NWAVE + wave] = (double)x;
  }
  __syncthreads();
  if (threadIdx.x < w_used) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < MCG_NWAVE; ++q) s += red[threadIdx.x * MCG_NWAVE + q];
    part[(size_t)blockIdx.x * w_used + threadIdx.x] = s;
  }
}

// As block_partials for one FP64 value v0 followed by KB FP32 values vf:
// the FP32 values (per-thread FP32 accumulations already) are summed across
// the wavefront in FP32, which halves the shuffle traffic of the block's
// closing reduction; the wavefront totals are then added in FP64.
template <int KB>
__device__ void block_partials_f(double v0, const float (&vf)[KB], int w_used,
                                 double *__restrict__ part, double *__restrict__ compact0) {
  __shared__ double red[(1 + KB) * MCG_NWAVE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double s0 = wave_sum(v0);
  if (lane == 0) red[wave] = s0;
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    float x = vf[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[(1 + j) * MCG_NWAVE + wave] = (double)x;
  }
  __syncthreads();
  if (threadIdx.x < w_used) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < MCG_NWAVE; ++q) s += red[threadIdx.x * MCG_NWAVE + q];
    part[(size_t)blockIdx.x * w_used + threadIdx.x] = s;
    if (compact0 && threadIdx.x == 0) compact0[blockIdx.x] = s;
  }
}

// Sum the partials of nb blocks (fixed order) into tot[0..w_used-1] (LDS),
// using all threads of the calling block (blockDim.x <= 1024).
static __device__ inline void sum_partials(const double *__restrict__ part, int nb, int w_used, double *tot) {
  __shared__ double red2[1024];
  const int groups = blockDim.x / w_used;
  const int g = threadIdx.x / w_used, j = threadIdx.x - g * w_used;
  if (g < groups) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = g;
    for (; b + 3 * groups < nb; b += 4 * groups) {
      a0 += part[(size_t)b * w_used + j];
      a1 += part[(size_t)(b + groups) * w_used + j];
      a2 += part[(size_t)(b + 2 * groups) * w_used + j];
      a3 += part[(size_t)(b + 3 * groups) * w_used + j];
    }
    for (; b < nb; b += groups) a0 += part[(size_t)b * w_used + j];
    red2[threadIdx.x] = (a0 + a1) + (a2 + a3);
  }
  __syncthreads();
  if (threadIdx.x < w_used) {
    double s = 0.0;
    for (int q = 0; q < groups; ++q) s += red2[q * w_used + threadIdx.x];
    tot[threadIdx.x] = s;
  }
  __syncthreads();
}

// Reduce W per-thread values over the grid in one kernel: block partials,
// then the last block to arrive (atomic ticket) sums them in block order.
// Returns true in that block, with the totals in tot (LDS).  Costs one
// device-scope release per block (an L2 write-back on this GPU), so the
// CG iteration kernels use block_partials plus a separate finalize kernel
// instead; this form is kept for kernels that run a few times per solve.
template <int W>
__device__ bool grid_sum(const double (&v)[W], int w_used, double *__restrict__ part,
                         unsigned *__restrict__ ticket, double *tot) {
  __shared__ bool last;
  block_partials<W>(v, w_used, part);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned prev = atomicAdd(ticket, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  sum_partials(part, gridDim.x, w_used, tot);
  if (threadIdx.x == 0) *ticket = 0u;
  return true;
}

// ---------------------------------------------------------------------------
// CSR tile product: tile[r] = (A x)[row0 + r] for the 256 rows of a tile,
// L lanes per row (vector CSR), values/columns streamed contiguously.
// ---------------------------------------------------------------------------
// CSR-stream form (selected as L == 1): the tile's nonzeros are contiguous in
// CSR, so the whole block loads them with independent coalesced loads
// (MCG_STREAM_PER_THREAD per thread), stages the products in LDS, and then each
// thread sums its own row.  Three dependent load levels per tile (row bounds,
// values/columns, gathered x) instead of three per L-lane pass.  Tiles with
// more nonzeros than the stage holds fall back to 8 lanes per row.
#define MCG_STREAM_PER_THREAD 16
#define MCG_STREAM_CAP (MCG_BLOCK * MCG_STREAM_PER_THREAD)
template <int L, typename TA, typename TX>
__device__ __forceinline__ void csr_tile(int n, int row0, const int32_t *__restrict__ rp,
                                         const int32_t *__restrict__ ci,
                                         const TA *__restrict__ va, const TX *__restrict__ x,
                                         TX *tile);

template <typename TA, typename TX>
__device__ __forceinline__ void csr_tile_stream(int n, int row0, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci,
                                                const TA *__restrict__ va,
                                                const TX *__restrict__ x, TX *tile) {
  __shared__ TX prod[MCG_STREAM_CAP];
  const int rend = min(row0 + MCG_BLOCK, n);
  const int nz0 = rp[row0], nz1 = rp[rend];
  const int cnt = nz1 - nz0;
  if (cnt > MCG_STREAM_CAP) {  // uniform across the block
    csr_tile<8, TA, TX>(n, row0, rp, ci, va, x, tile);
    return;
  }
  const int row = row0 + threadIdx.x;
  const int rs = row < n ? rp[row] : nz1;
  const int re = row < n ? rp[row + 1] : nz1;
  TX pv[MCG_STREAM_PER_THREAD];
#pragma unroll
  for (int u = 0; u < MCG_STREAM_PER_THREAD; ++u) {
    const int e = threadIdx.x + u * MCG_BLOCK;
    const int ec = e < cnt ? e : (cnt > 0 ? cnt - 1 : 0);
    pv[u] = (cnt > 0) ? (TX)va[nz0 + ec] * x[ci[nz0 + ec]] : (TX)0;
  }
#pragma unroll
  for (int u = 0; u < MCG_STREAM_PER_THREAD; ++u) {
    const int e = threadIdx.x + u * MCG_BLOCK;
    if (e < cnt) prod[e] = pv[u];
  }
  __syncthreads();
  TX acc = 0;
  for (int e = rs - nz0; e < re - nz0; ++e) acc += prod[e];
  tile[threadIdx.x] = acc;
  __syncthreads();  // prod is reused by the next tile
}

template <int L, typename TA, typename TX>
__device__ __forceinline__ void csr_tile(int n, int row0, const int32_t *__restrict__ rp,
                                         const int32_t *__restrict__ ci,
                                         const TA *__restrict__ va, const TX *__restrict__ x,
                                         TX *tile) {
  if constexpr (L == 1) {
    csr_tile_stream<TA, TX>(n, row0, rp, ci, va, x, tile);
    return;
  }
  constexpr int NG = MCG_BLOCK / (L > 1 ? L : 2);
  const int lane = threadIdx.x & (L - 1);
  const int grp = threadIdx.x / L;
  for (int r = grp; r < MCG_BLOCK; r += NG) {
    const int row = row0 + r;
    TX acc = 0;
    if (row < n) {
      const int s = rp[row], e = rp[row + 1];
      for (int p = s + lane; p < e; p += L) acc += (TX)va[p] * x[ci[p]];
    }
    if constexpr (L > 1) {
#pragma unroll
      for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, L);
    }
    if (lane == 0) tile[r] = acc;
  }
}

// Device layout of Vhat: blocks of 64 rows, column-major inside a block:
// entry (i, j) at (i / 64) * 64k + 64 j + i % 64.  A wavefront reading
// column j of its 64 rows gets one contiguous 256-byte (FP32) segment, and
// the k columns of a row block lie together (one page instead of k pages
// n elements apart).  Allocation: ceil(n / 64) * 64 * k elements.
#define MCG_VBLK 64
__host__ __device__ inline size_t vhat_index(int i, int j, int k) {
  return (size_t)(i / MCG_VBLK) * ((size_t)MCG_VBLK * k) + (size_t)j * MCG_VBLK + (i % MCG_VBLK);
}

// Row `row` of Vhat into registers: KB unconditional loads, the column index
// clamped to k-1 so that no load is guarded (guarded loads would each wait
// for their own result).  Entries j >= k are copies of column k-1 and must be
// multiplied by zero (or ignored) by the caller.
template <int KB, typename T>
__device__ __forceinline__ void vhat_row(const T *__restrict__ V, int n, int k, int row,
                                         T (&v)[KB > 0 ? KB : 1]) {
  (void)n;
  const T *base = V + (size_t)(row / MCG_VBLK) * ((size_t)MCG_VBLK * k) + (row % MCG_VBLK);
#pragma unroll
  for (int j = 0; j < KB; ++j) v[j] = base[(size_t)(j < k ? j : k - 1) * MCG_VBLK];
}

// column-major n x k (caller layout) -> blocked device layout, converting type
template <typename TO>
__global__ void k_vhat_to_blocked(int n, int k, const double *__restrict__ cm,
                                  TO *__restrict__ blk) {
  const int64_t total = (int64_t)((n + MCG_VBLK - 1) / MCG_VBLK) * MCG_VBLK * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / ((int64_t)MCG_VBLK * k);
    const int rem = (int)(e - b * MCG_VBLK * k);
    const int j = rem / MCG_VBLK, r = rem % MCG_VBLK;
    const int64_t i = b * MCG_VBLK + r;
    blk[e] = i < n ? (TO)cm[(size_t)j * n + i] : (TO)0;
  }
}

// ---------------------------------------------------------------------------
// a1: y = A x
// ---------------------------------------------------------------------------
template <int L, typename T>
__global__ __launch_bounds__(MCG_BLOCK) void k_spmv(int n, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci,
                                                    const T *__restrict__ va,
                                                    const T *__restrict__ x, T *__restrict__ y) {
  __shared__ T tile[MCG_BLOCK];
  for (int row0 = blockIdx.x * MCG_BLOCK; row0 < n; row0 += gridDim.x * MCG_BLOCK) {
    csr_tile<L, T, T>(n, row0, rp, ci, va, x, tile);
    __syncthreads();
    const int row = row0 + threadIdx.x;
    if (row < n) y[row] = tile[threadIdx.x];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Block CSR SpMV for matrices made of dense BS x BS blocks (FE-like systems
// with BS unknowns per node): one column index per BS^2 values instead of one
// per value.  G lanes share a block row; each lane takes whole blocks (U of
// them in flight, block indices clamped so that every load is unconditional
// and issued before any is used), multiplies the block by its BS entries of
// x into BS row sums, and the G lanes then add their sums by shuffles.
// With S != nullptr the kernel returns at once after the inner stop.
// ---------------------------------------------------------------------------
// DOT: also r^T y and y^T y as block partials (the C product of the C C^T
// preconditioner, finished by FIN_RHO).
template <int BS, int G, typename T, bool DOT = false>
__global__ __launch_bounds__(MCG_BLOCK) void k_bsr_spmv(int nbr, const int32_t *__restrict__ b_rp,
                                                        const int32_t *__restrict__ b_ci,
                                                        const T *__restrict__ b_v,
                                                        const T *__restrict__ x,
                                                        T *__restrict__ y,
                                                        const DevState *__restrict__ S,
                                                        const T *__restrict__ r = nullptr,
                                                        double *__restrict__ part = nullptr,
                                                        double *__restrict__ compact = nullptr) {
  if (S && S->done) return;
  T rt = 0, tt = 0;
  constexpr int BB = BS * BS;
  constexpr int U = 2;
  const int lane = threadIdx.x & (G - 1);
  const int per_block = MCG_BLOCK / G;
  for (int I = blockIdx.x * per_block + threadIdx.x / G; I < nbr; I += gridDim.x * per_block) {
    const int b0 = b_rp[I], b1 = b_rp[I + 1];
    T acc[BS];
#pragma unroll
    for (int q = 0; q < BS; ++q) acc[q] = 0;
    for (int base = b0 + lane; base < b1; base += G * U) {
      T xv[U][BS], bv[U][BB];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int blk = min(base + u * G, b1 - 1);
        const size_t c = (size_t)b_ci[blk] * BS;
#pragma unroll
        for (int b = 0; b < BS; ++b) xv[u][b] = x[c + b];
#pragma unroll
        for (int q = 0; q < BB; ++q) bv[u][q] = b_v[(size_t)blk * BB + q];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = base + u * G < b1;
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
    for (int q = 0; q < BS; ++q) {
#pragma unroll
      for (int off = G / 2; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off, G);
    }
    if (lane < BS) {
      T out = acc[0];
#pragma unroll
      for (int q = 1; q < BS; ++q) out = (lane == q) ? acc[q] : out;
      y[(size_t)I * BS + lane] = out;
      if (DOT) {
        rt += r[(size_t)I * BS + lane] * out;
        tt += out * out;
      }
    }
  }
  if (DOT) {
    double v[2] = {(double)rt, (double)tt};
    block_partials<2>(v, 2, part, compact);
  }
}

// ---------------------------------------------------------------------------
// a2 + first scalar of a4: q = A p + Vhat (c o s), pi = p^T q, alpha = rho/pi
// (s = Vhat^T p was reduced by the kernel that produced p).
// stage_alpha = 0 only computes q (the standalone M_mr apply).
// ---------------------------------------------------------------------------
// WQ (diagonal M_cg with dinv): also w = Vhat^T (D^{-1} q), reduced with pi,
// so that the direction kernel needs no pass over Vhat (see k_cg_update_diag).
template <int L, typename T, int KB, bool WQ = false>
__global__ __launch_bounds__(MCG_BLOCK) void k_mmr(int n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const T *__restrict__ va,
                                                   const T *__restrict__ p, T *__restrict__ q,
                                                   const T *__restrict__ V, int k,
                                                   DevState *__restrict__ S, double *part,
                                                   unsigned *ticket, int stage_alpha,
                                                   const T *__restrict__ dinv = nullptr,
                                                   double *__restrict__ pi_compact = nullptr) {
  if (stage_alpha && S->done) return;
  __shared__ T tile[MCG_BLOCK];
  __shared__ T cs[KB > 0 ? KB : 1];
  if (KB > 0 && threadIdx.x < KB) cs[threadIdx.x] = threadIdx.x < k ? (T)S->cs_[threadIdx.x] : (T)0;
  __syncthreads();
  T pq = 0;
  constexpr int KW = (WQ && KB > 0) ? KB : 1;
  T wacc[KW];
#pragma unroll
  for (int j = 0; j < KW; ++j) wacc[j] = 0;
  for (int row0 = blockIdx.x * MCG_BLOCK; row0 < n; row0 += gridDim.x * MCG_BLOCK) {
    const int row = row0 + threadIdx.x;
    const int rowc = row < n ? row : n - 1;
    // issue this row's Vhat and p loads before the SpMV phase
    T vr[KB > 0 ? KB : 1];
    vhat_row<KB, T>(V, n, k, rowc, vr);
    const T prow = p[rowc];
    const T drow = WQ ? dinv[rowc] : (T)0;
    csr_tile<L, T, T>(n, row0, rp, ci, va, p, tile);
    __syncthreads();
    if (row < n) {
      T acc = tile[threadIdx.x];
#pragma unroll
      for (int j = 0; j < KB; ++j) acc += vr[j] * cs[j];
      q[row] = acc;
      pq += prow * acc;
      if (WQ) {
        const T dq = drow * acc;
#pragma unroll
        for (int j = 0; j < KW; ++j) wacc[j] += vr[j] * dq;
      }
    }
    __syncthreads();
  }
  if (!stage_alpha) return;
  constexpr int W = 1 + ((WQ && KB > 0) ? KB : 0);
  double v[W];
  v[0] = (double)pq;
  if (WQ) {
#pragma unroll
    for (int j = 1; j < W; ++j) v[j] = (double)wacc[j - 1];
  }
  block_partials<W>(v, WQ ? 1 + k : 1, part, pi_compact);  // FIN_MMR or the Jacobi update
}

// Split form of the iteration's M_mr apply, part 1: q = A p (the done flag
// lets launches after the inner stop return at once).
template <int L, typename T>
__global__ __launch_bounds__(MCG_BLOCK) void k_spmv_chk(int n, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        const T *__restrict__ va,
                                                        const T *__restrict__ x, T *__restrict__ y,
                                                        const DevState *__restrict__ S) {
  if (S->done) return;
  __shared__ T tile[MCG_BLOCK];
  for (int row0 = blockIdx.x * MCG_BLOCK; row0 < n; row0 += gridDim.x * MCG_BLOCK) {
    csr_tile<L, T, T>(n, row0, rp, ci, va, x, tile);
    __syncthreads();
    const int row = row0 + threadIdx.x;
    if (row < n) y[row] = tile[threadIdx.x];
    __syncthreads();
  }
}

// Split form, part 2 (streaming, one row per thread, two rows in flight):
// q += Vhat (c o s); partials of p^T q and w = Vhat^T D^{-1} q.
// WQ = false (general M_cg): only q and p^T q; dinv is not read.
template <typename T, int KB, bool WQ = true>
__global__ __launch_bounds__(MCG_BLOCK) void k_mmr_vpart(int n, const T *__restrict__ p,
                                                         T *__restrict__ q,
                                                         const T *__restrict__ dinv,
                                                         const T *__restrict__ V, int k,
                                                         const DevState *__restrict__ S,
                                                         double *__restrict__ part,
                                                         double *__restrict__ pi_compact = nullptr) {
  if (S->done) return;
  __shared__ T cs[KB];
  if (threadIdx.x < KB) cs[threadIdx.x] = threadIdx.x < k ? (T)S->cs_[threadIdx.x] : (T)0;
  __syncthreads();
  T pq = 0, wacc[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) wacc[j] = 0;
  constexpr int U = 2;
  const int stride = gridDim.x * MCG_BLOCK;
  for (int base = blockIdx.x * MCG_BLOCK + threadIdx.x; base < n; base += U * stride) {
    T qv[U], pv[U], dv[U], vr[U][KB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = min(base + u * stride, n - 1);
      qv[u] = q[i];
      pv[u] = p[i];
      dv[u] = WQ ? dinv[i] : (T)0;
      vhat_row<KB, T>(V, n, k, i, vr[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * stride;
      if (i < n) {
        T acc = qv[u];
#pragma unroll
        for (int j = 0; j < KB; ++j) acc += vr[u][j] * cs[j];
        q[i] = acc;
        pq += pv[u] * acc;
        if (WQ) {
          const T dq = dv[u] * acc;
#pragma unroll
          for (int j = 0; j < KB; ++j) wacc[j] += vr[u][j] * dq;
        }
      }
    }
  }
  if (WQ) {
    if constexpr (sizeof(T) == 4) {
      block_partials_f<KB>((double)pq, wacc, 1 + k, part, pi_compact);  // the Jacobi update
    } else {
      double v[1 + KB];
      v[0] = (double)pq;
#pragma unroll
      for (int j = 0; j < KB; ++j) v[1 + j] = (double)wacc[j];
      block_partials<1 + KB>(v, 1 + k, part, pi_compact);  // the Jacobi update
    }
  } else {
    double v[1] = {(double)pq};
    block_partials<1>(v, 1, part, pi_compact);  // finished by k_finalize(FIN_MMR)
  }
}

// ---------------------------------------------------------------------------
// Sliced ELL copy of A for the inner products.  Rows are cut into slices of 64
// (one wavefront; the same 64-row blocks as the Vhat layout), each slice
// padded to its longest row and stored slot-major: entry (slot j, row 64 s + l)
// at off[s] + 64 j + l.  Every load of a slot is one coalesced 64-lane
// access, no row pointers are read per row, and on grid stencils the x
// gathers of a slot are nearly contiguous too.  Columns are 16-bit offsets
// from the row (IDX = int16_t) when every |col - row| < 2^15, else absolute
// int32.  Padding entries hold value 0 and a column inside the matrix (the
// row itself, or n - 1 for the rows past n of the last slice).
// ---------------------------------------------------------------------------
template <typename IDX>
__device__ __forceinline__ int sell_col(IDX c, int row) {
  if constexpr (sizeof(IDX) == 2)
    return row + (int)c;
  else
    return (int)c;
}

// (A x)[64 s + lane] for one slice; all slots' columns and values of a group
// of 8 are loaded before their gathers (slot indices clamped, so no load is
// guarded; the clamped duplicates are multiplied by zero)
template <typename T, typename IDX>
__device__ __forceinline__ T sell_row(const int64_t *__restrict__ off, const IDX *__restrict__ col,
                                      const T *__restrict__ val, const T *__restrict__ x,
                                      int slice, int lane) {
  const int64_t o = off[slice];
  const int w = (int)((off[slice + 1] - o) >> 6);
  const int row = slice * 64 + lane;
  const IDX *cp = col + o + lane;
  const T *vp = val + o + lane;
  T acc = 0;
  for (int j0 = 0; j0 < w; j0 += 8) {
    IDX c[8];
    T a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = min(j0 + u, w - 1);
      c[u] = cp[(size_t)j * 64];
      a[u] = vp[(size_t)j * 64];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const T xv = x[sell_col<IDX>(c[u], row)];
      acc += (j0 + u < w) ? a[u] * xv : (T)0;
    }
  }
  return acc;
}

// (A x) for the rows of two slices s0, s1 (s1 may repeat s0; its result is
// then discarded by the caller): both slices' columns and values of a group
// of G slots are loaded before any gather, which keeps twice the loads of
// sell_row in flight per wavefront.  G = 4 for copies whose slices are at
// most 4 wide (the learned factor C and its transpose on 7-point stencils),
// so that no load is spent on clamped duplicates.
template <typename T, typename IDX, int G = 8, typename TV = T>
__device__ __forceinline__ void sell_rows2(const int64_t *__restrict__ off,
                                           const IDX *__restrict__ col, const TV *__restrict__ val,
                                           const T *__restrict__ x, int s0, int s1, int lane,
                                           T &acc0, T &acc1) {
  const int64_t o0 = off[s0], o1 = off[s1];
  const int w0 = (int)((off[s0 + 1] - o0) >> 6), w1 = (int)((off[s1 + 1] - o1) >> 6);
  const int row0 = s0 * 64 + lane, row1 = s1 * 64 + lane;
  const IDX *c0p = col + o0 + lane, *c1p = col + o1 + lane;
  const TV *v0p = val + o0 + lane, *v1p = val + o1 + lane;
  const int wm = max(w0, w1);
  acc0 = 0;
  acc1 = 0;
  for (int j0 = 0; j0 < wm; j0 += G) {
    IDX c0[G], c1[G];
    T a0[G], a1[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int j = min(j0 + u, w0 - 1), k = min(j0 + u, w1 - 1);
      c0[u] = c0p[(size_t)j * 64];
      a0[u] = (T)v0p[(size_t)j * 64];
      c1[u] = c1p[(size_t)k * 64];
      a1[u] = (T)v1p[(size_t)k * 64];
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const T x0 = x[sell_col<IDX>(c0[u], row0)], x1 = x[sell_col<IDX>(c1[u], row1)];
      acc0 += (j0 + u < w0) ? a0[u] * x0 : (T)0;
      acc1 += (j0 + u < w1) ? a1[u] * x1 : (T)0;
    }
  }
}

// y = A x from the sliced copy, two slices per wavefront (S != nullptr:
// return at once after the inner stop)
template <typename T, typename IDX, int G = 8, typename TV = T>
__global__ __launch_bounds__(MCG_BLOCK) void k_sell_spmv(int n, int nslices,
                                                         const int64_t *__restrict__ off,
                                                         const IDX *__restrict__ col,
                                                         const TV *__restrict__ val,
                                                         const T *__restrict__ x,
                                                         T *__restrict__ y,
                                                         const DevState *__restrict__ S) {
  if (S && S->done) return;
  const int lane = threadIdx.x & 63;
  for (int wv = blockIdx.x * MCG_NWAVE + (threadIdx.x >> 6); 2 * wv < nslices;
       wv += gridDim.x * MCG_NWAVE) {
    const int s0 = 2 * wv, s1 = min(s0 + 1, nslices - 1);
    T a0, a1;
    sell_rows2<T, IDX, G, TV>(off, col, val, x, s0, s1, lane, a0, a1);
    const int r0 = s0 * 64 + lane, r1 = (s0 + 1) * 64 + lane;
    if (r0 < n) y[r0] = a0;
    if (s0 + 1 < nslices && r1 < n) y[r1] = a1;
  }
}

// The whole M_mr apply in one pass from the sliced copy: each wavefront owns
// a slice of 64 rows, which is also one 64-row block of Vhat, so
// q = A p + Vhat (c o s) needs A's slice, the Vhat block and p, dinv, q of
// those rows once.  stage = 1: done check and block partials as k_mmr (p^T q,
// and with WQ the Vhat^T D^{-1} q of the Jacobi recurrence); stage = 0 only
// writes q (standalone apply).
template <typename T, typename IDX, int KB, bool WQ>
__global__ __launch_bounds__(MCG_BLOCK) void k_sell_mmr(
    int n, int nslices, const int64_t *__restrict__ off, const IDX *__restrict__ col,
    const T *__restrict__ val, const T *__restrict__ p, T *__restrict__ q,
    const T *__restrict__ dinv, const T *__restrict__ V, int k, const DevState *__restrict__ S,
    int stage, double *__restrict__ part, double *__restrict__ pi_compact) {
  if (stage && S->done) return;
  __shared__ T cs[KB > 0 ? KB : 1];
  if (KB > 0 && threadIdx.x < KB) cs[threadIdx.x] = threadIdx.x < k ? (T)S->cs_[threadIdx.x] : (T)0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  T pq = 0;
  constexpr int KW = (WQ && KB > 0) ? KB : 1;
  T wacc[KW];
#pragma unroll
  for (int j = 0; j < KW; ++j) wacc[j] = 0;
  for (int sl = blockIdx.x * MCG_NWAVE + (threadIdx.x >> 6); sl < nslices;
       sl += gridDim.x * MCG_NWAVE) {
    const int row = sl * 64 + lane;
    const int rowc = row < n ? row : n - 1;
    T vr[KB > 0 ? KB : 1];
    vhat_row<KB, T>(V, n, k, rowc, vr);  // issued ahead of the gathers
    const T prow = p[rowc];
    const T drow = WQ ? dinv[rowc] : (T)0;
    T acc = sell_row<T, IDX>(off, col, val, p, sl, lane);
#pragma unroll
    for (int j = 0; j < KB; ++j) acc += vr[j] * cs[j];
    if (row < n) {
      q[row] = acc;
      pq += prow * acc;
      if constexpr (WQ && KB > 0) {
        const T dq = drow * acc;
#pragma unroll
        for (int j = 0; j < KB; ++j) wacc[j] += vr[j] * dq;
      }
    }
  }
  if (!stage) return;
  constexpr int W = 1 + ((WQ && KB > 0) ? KB : 0);
  double v[W];
  v[0] = (double)pq;
#pragma unroll
  for (int j = 1; j < W; ++j) v[j] = (double)wacc[j - 1];
  block_partials<W>(v, (WQ && KB > 0) ? 1 + k : 1, part, pi_compact);
}

// s = Vhat^T u, cs = c o s  (standalone M_mr apply, first half)
template <typename T, int KB>
__global__ __launch_bounds__(MCG_BLOCK) void k_vtu(int n, const T *__restrict__ u,
                                                   const T *__restrict__ V, int k,
                                                   DevState *__restrict__ S, double *part,
                                                   unsigned *ticket) {
  T acc[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) acc[j] = 0;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    const T ui = u[i];
    T vr[KB];
    vhat_row<KB, T>(V, n, k, i, vr);
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] += vr[j] * ui;
  }
  double v[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) v[j] = (double)acc[j];
  __shared__ double tot[KB];
  if (grid_sum<KB>(v, k, part, ticket, tot)) {
    if (threadIdx.x < k) {
      S->s[threadIdx.x] = tot[threadIdx.x];
      S->cs_[threadIdx.x] = S->c[threadIdx.x] * tot[threadIdx.x];
    }
  }
}

// ---------------------------------------------------------------------------
// Jacobi iteration with the reductions finished inside the consumer kernels
// (no one-block finalize launches): every block sums the producer's block
// partials it needs, in the same fixed order, so all blocks see bitwise the
// same scalars; block 0 alone writes the state.  rho is kept in two slots by
// iteration parity so that the block writing the new rho never races a block
// still reading the current one.
// ---------------------------------------------------------------------------

// tot[c] = sum over rows b < nb of part[b * stride + c], c < NC; all threads
// of the block take part (fixed order: thread t sums rows t, t + blockDim, ...)
// (columns c >= ncols are not read and come out 0)
template <int NC>
__device__ void block_sum_cols(const double *__restrict__ part, int nb, int stride,
                               double (&tot)[NC], int ncols = NC) {
  __shared__ double red[(NC > 0 ? NC : 1) * MCG_NWAVE];
  double a[NC > 0 ? NC : 1];
#pragma unroll
  for (int c = 0; c < NC; ++c) a[c] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < ncols) a[c] += part[(size_t)b * stride + c];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double s = wave_sum(a[c]);
    if (lane == 0) red[c * MCG_NWAVE + wave] = s;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < MCG_NWAVE; ++q) s += red[c * MCG_NWAVE + q];
    tot[c] = s;
  }
  __syncthreads();
}

// y = A x from the sliced copy inside a CG iteration.  part_in != nullptr:
// also finish the Vhat^T p reduction of the preceding direction kernel (nb_in
// blocks of k partials in part_in): blocks take one column each and store
// s = Vhat^T p and cs = c o s for the kernels that follow.  pap_out !=
// nullptr: per-block x^T y into pap_out[blockIdx.x] (x = p gives p^T A p).
template <typename T, typename IDX>
__global__ __launch_bounds__(MCG_BLOCK) void k_sell_spmv_vtp(int n, int nslices,
                                                             const int64_t *__restrict__ off,
                                                             const IDX *__restrict__ col,
                                                             const T *__restrict__ val,
                                                             const T *__restrict__ x,
                                                             T *__restrict__ y,
                                                             DevState *__restrict__ S,
                                                             const double *__restrict__ part_in,
                                                             int nb_in, int k,
                                                             double *__restrict__ pap_out) {
  if (S->done) return;
  if (part_in) {
    for (int j = blockIdx.x; j < k; j += gridDim.x) {  // block-uniform bound
      double tot[1];
      block_sum_cols<1>(part_in + j, nb_in, k, tot);
      if (threadIdx.x == 0) {
        S->s[j] = tot[0];
        S->cs_[j] = S->c[j] * tot[0];
      }
    }
  }
  const int lane = threadIdx.x & 63;
  T xy = 0;
  for (int wv = blockIdx.x * MCG_NWAVE + (threadIdx.x >> 6); 2 * wv < nslices;
       wv += gridDim.x * MCG_NWAVE) {
    const int s0 = 2 * wv, s1 = min(s0 + 1, nslices - 1);
    T a0, a1;
    sell_rows2<T, IDX>(off, col, val, x, s0, s1, lane, a0, a1);
    const int r0 = s0 * 64 + lane, r1 = (s0 + 1) * 64 + lane;
    if (r0 < n) {
      y[r0] = a0;
      if (pap_out) xy += x[r0] * a0;
    }
    if (s0 + 1 < nslices && r1 < n) {
      y[r1] = a1;
      if (pap_out) xy += x[r1] * a1;
    }
  }
  if (pap_out) {
    double v[1] = {(double)xy};
    block_partials<1>(v, 1, pap_out);
  }
}

// CG update with the rank-k part of the M_mr apply folded in.  The SpMV
// kernel left Ap (in Ap) and per-block p^T A p (pap_in, nb_in); with
// s = Vhat^T p as kept in S->s, p^T M_mr p = p^T A p + sum_j c_j s_j^2, so
// alpha = rho / pi is known before the pass, and q = A p + Vhat (c o s) is
// formed row by row from the streamed Vhat rows and used at once:
// z += alpha p, r -= alpha q (q is never stored).  DIAG (Jacobi M_cg, dinv):
// block partials of (r^T t, r^T r, t^T t), t = dinv o r, into part3 (and
// r^T t into rt_compact) and of w = Vhat^T D^-1 q into part_w (rows of 1 + k,
// column 0 unused), for k_cg_dir_f.  General M_cg: per-block r^T r into
// rr_out.  pi <= 0: NOT_SPD, nothing updated.
template <typename T, int KB, bool DIAG>
__global__ __launch_bounds__(MCG_BLOCK) void k_cg_update_v(
    int n, T *__restrict__ z, T *__restrict__ r, const T *__restrict__ p,
    const T *__restrict__ Ap, const T *__restrict__ dinv, const T *__restrict__ V, int k,
    DevState *__restrict__ S, const double *__restrict__ pap_in, int nb_in,
    double *__restrict__ part3, double *__restrict__ rt_compact, double *__restrict__ part_w,
    double *__restrict__ rr_out, int par) {
  if (S->done) return;
  __shared__ T cs[KB];
  if (threadIdx.x < KB) cs[threadIdx.x] = threadIdx.x < k ? (T)S->cs_[threadIdx.x] : (T)0;
  double pap[1];
  block_sum_cols<1>(pap_in, nb_in, 1, pap);  // its barriers also publish cs
  double quad = 0.0;
  for (int j = 0; j < k; ++j) quad += S->c[j] * S->s[j] * S->s[j];
  const double pi = pap[0] + quad;
  const bool spd = pi > 0.0;  // false also for NaN
  const double alpha_d = spd ? S->rho_par[par] / pi : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S->pi = pi;
    S->alpha = alpha_d;
    if (!spd) {
      S->status = 4;  // MCG_NOT_SPD: M_mr not positive along p
      S->done = 1;
    }
  }
  if (!spd) return;
  const T alpha = (T)alpha_d;
  T rr = 0, rt = 0, tt = 0;
  T wacc[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) wacc[j] = 0;
  constexpr int U = 2;
  const int stride = gridDim.x * MCG_BLOCK;
  for (int base = blockIdx.x * MCG_BLOCK + threadIdx.x; base < n; base += U * stride) {
    T zv[U], pv[U], rv[U], av[U], dv[U], vr[U][KB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = min(base + u * stride, n - 1);
      zv[u] = z[i];
      pv[u] = p[i];
      rv[u] = r[i];
      av[u] = Ap[i];
      dv[u] = DIAG ? dinv[i] : (T)0;
      vhat_row<KB, T>(V, n, k, i, vr[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * stride;
      if (i < n) {
        T q = av[u];
#pragma unroll
        for (int j = 0; j < KB; ++j) q += vr[u][j] * cs[j];
        const T zi = zv[u] + alpha * pv[u];
        const T ri = rv[u] - alpha * q;
        z[i] = zi;
        r[i] = ri;
        rr += ri * ri;
        if constexpr (DIAG) {
          const T ti = dv[u] * ri;
          rt += ri * ti;
          tt += ti * ti;
          const T dq = dv[u] * q;
#pragma unroll
          for (int j = 0; j < KB; ++j) wacc[j] += vr[u][j] * dq;
        }
      }
    }
  }
  if constexpr (DIAG) {
    double v[3] = {(double)rt, (double)rr, (double)tt};
    block_partials<3>(v, 3, part3, rt_compact);
    if constexpr (sizeof(T) == 4) {
      block_partials_f<KB>(0.0, wacc, 1 + k, part_w, nullptr);
    } else {
      double w[1 + KB];
      w[0] = 0.0;
#pragma unroll
      for (int j = 0; j < KB; ++j) w[1 + j] = (double)wacc[j];
      block_partials<1 + KB>(w, 1 + k, part_w);
    }
  } else {
    double v[1] = {(double)rr};
    block_partials<1>(v, 1, rr_out);
  }
}

// ---------------------------------------------------------------------------
// Sliced block ELL: the dense BS x BS blocks of a block matrix, with block
// rows cut into slices of 64 (one wavefront, one block row per lane), each
// slice padded to its longest block row and stored slot-major: the block
// column of (slot j, block row 64 s + l) at col[off[s] + 64 j + l], its
// entry (a, b) at val[(off[s] + 64 j) BS^2 + (a BS + b) 64 + l].  Every load
// of a slot is one coalesced 64-lane access.  Padding blocks are zeros whose
// block column is the row's own (or nbr - 1 past the last block row).
// DOT: block partials of r^T y and y^T y (the C product of C C^T).  TV:
// the stored value type (FP16 for the learned factor in FP32 iterations).
// part_in != nullptr: first finish the Vhat^T p reduction of the preceding
// direction kernel (nb_in blocks of k partials; one column per block), as
// k_sell_spmv_vtp.  xmap != nullptr (grids of at least 8 workgroups): the
// slices of XCD e (workgroups b with b % 8 == e) are xmap[9 + i] for
// xmap[e] <= i < xmap[e + 1], shared by that XCD's workgroups.
// ---------------------------------------------------------------------------
template <int BS, typename T, bool DOT, typename TV = T>
__global__ __launch_bounds__(MCG_BLOCK) void k_bsell_spmv(
    int nbr, int nslices, const int64_t *__restrict__ off, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const T *__restrict__ x, T *__restrict__ y,
    DevState *__restrict__ S, const T *__restrict__ r, double *__restrict__ part,
    double *__restrict__ compact, const double *__restrict__ part_in, int nb_in, int k,
    const int32_t *__restrict__ xmap) {
  if (S && S->done) return;
  if (part_in) {
    for (int j = blockIdx.x; j < k; j += gridDim.x) {  // block-uniform bound
      double tot[1];
      block_sum_cols<1>(part_in + j, nb_in, k, tot);
      if (threadIdx.x == 0) {
        S->s[j] = tot[0];
        S->cs_[j] = S->c[j] * tot[0];
      }
    }
  }
  constexpr int BB = BS * BS;
  constexpr int U = 4;  // slots in flight per lane
  const int lane = threadIdx.x & 63;
  T rt = 0, tt = 0;
  int i0 = blockIdx.x * MCG_NWAVE + (threadIdx.x >> 6), i1 = nslices,
      step = gridDim.x * MCG_NWAVE;
  if (xmap) {
    const int e = blockIdx.x & 7;
    i0 = xmap[e] + (blockIdx.x >> 3) * MCG_NWAVE + (threadIdx.x >> 6);
    i1 = xmap[e + 1];
    step = ((gridDim.x - e + 7) >> 3) * MCG_NWAVE;  // this XCD's workgroups
  }
  for (int i = i0; i < i1; i += step) {
    const int sl = xmap ? xmap[9 + i] : i;
    const int64_t o = off[sl];
    const int w = (int)((off[sl + 1] - o) >> 6);
    const int32_t *cp = col + o + lane;
    const TV *vp = val + o * BB + lane;
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
        for (int q = 0; q < BB; ++q) bv[u][q] = (T)vp[((size_t)j * BB + q) * 64];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int b = 0; b < BS; ++b) xv[u][b] = x[(size_t)c[u] * BS + b];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = j0 + u < w;
#pragma unroll
        for (int a = 0; a < BS; ++a) {
          T sum = 0;
#pragma unroll
          for (int b = 0; b < BS; ++b) sum += bv[u][a * BS + b] * xv[u][b];
          acc[a] += ok ? sum : (T)0;
        }
      }
    }
    const int I = sl * 64 + lane;
    if (I < nbr) {
#pragma unroll
      for (int a = 0; a < BS; ++a) {
        y[(size_t)I * BS + a] = acc[a];
        if constexpr (DOT) {
          rt += r[(size_t)I * BS + a] * acc[a];
          tt += acc[a] * acc[a];
        }
      }
    }
  }
  if constexpr (DOT) {
    double v[2] = {(double)rt, (double)tt};
    block_partials<2>(v, 2, part, compact);  // finished by k_cg_dir_gf
  }
}

// alpha = rho / pi from the M_mr apply's per-block pi values (pi_in, nb_in
// contiguous doubles); z += alpha p; r -= alpha q; block partials of r^T t,
// r^T r, t^T t (t = dinv o r) into part_out (rows of 3) and r^T t alone into
// rt_compact.  pi <= 0: NOT_SPD, nothing updated.
template <typename T>
__global__ __launch_bounds__(MCG_BLOCK) void k_cg_update_diag_f(
    int n, T *__restrict__ z, T *__restrict__ r, const T *__restrict__ p,
    const T *__restrict__ q, const T *__restrict__ dinv, DevState *__restrict__ S,
    const double *__restrict__ pi_in, int nb_in, double *__restrict__ part_out,
    double *__restrict__ rt_compact, int par) {
  if (S->done) return;
  double pi[1];
  block_sum_cols<1>(pi_in, nb_in, 1, pi);
  const bool spd = pi[0] > 0.0;  // false also for NaN
  const double alpha_d = spd ? S->rho_par[par] / pi[0] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S->pi = pi[0];
    S->alpha = alpha_d;
    if (!spd) {
      S->status = 4;  // MCG_NOT_SPD: M_mr not positive along p
      S->done = 1;
    }
  }
  if (!spd) return;
  const T alpha = (T)alpha_d;
  T rr = 0, rt = 0, tt = 0;
  constexpr int U = 4;
  const int stride = gridDim.x * MCG_BLOCK;
  for (int base = blockIdx.x * MCG_BLOCK + threadIdx.x; base < n; base += U * stride) {
    T zv[U], pv[U], rv[U], qv[U], dv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = min(base + u * stride, n - 1);
      zv[u] = z[i]; pv[u] = p[i]; rv[u] = r[i]; qv[u] = q[i]; dv[u] = dinv[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * stride;
      if (i < n) {
        const T zi = zv[u] + alpha * pv[u];
        const T ri = rv[u] - alpha * qv[u];
        z[i] = zi;
        r[i] = ri;
        const T ti = dv[u] * ri;
        rr += ri * ri;
        rt += ri * ti;
        tt += ti * ti;
      }
    }
  }
  double v[3] = {(double)rt, (double)rr, (double)tt};
  block_partials<3>(v, 3, part_out, rt_compact);
}

// From the update's partials (nb_in rows of r^T t, r^T r, t^T t, and the
// compact r^T t in rt_in): stop tests, beta = r^T t / rho;
// p = dinv o r + beta p.  Block 0 records the state: its,
// rr, status/done, the new rho in the other parity slot, and (not REFRESH) the
// projected recurrences Vhat^T t -= alpha w, Vhat^T p = Vhat^T t + beta Vhat^T p
// with w = Vhat^T D^-1 q summed from the M_mr partials (columns 1..k of nb_w
// rows of width 1 + k).  REFRESH instead recomputes Vhat^T p and Vhat^T t
// directly: block partials of 2 KB values into part_out (FIN_REFRESH).
template <typename T, int KB, bool REFRESH>
__global__ __launch_bounds__(MCG_BLOCK) void k_cg_dir_f(
    int n, T *__restrict__ p, const T *__restrict__ r, const T *__restrict__ dinv,
    const T *__restrict__ V, int k, DevState *__restrict__ S,
    const double *__restrict__ part_in, int nb_in, const double *__restrict__ part_w, int nb_w,
    double *__restrict__ part_out, const double *__restrict__ rt_in, int par) {
  if (S->done) return;
  double rts[1];
  block_sum_cols<1>(rt_in, nb_in, 1, rts);
  const double beta_d = rts[0] / S->rho_par[par];
  if (blockIdx.x == 0) {
    double tot3[3];  // r^T t, r^T r, t^T t
    block_sum_cols<3>(part_in, nb_in, 3, tot3);
    const double tot[3] = {tot3[1], rts[0], tot3[2]};  // rr, r^T t (the value all blocks use), tt
    if (threadIdx.x == 0) {
      const int64_t its = S->its + 1;
      S->its = its;
      S->rr = tot[0];
      if (tot[0] <= S->rtol2 * S->yy) {
        S->status = 0;
        S->done = 1;
      } else if (its >= S->maxit) {
        S->status = 1;
        S->done = 1;
      } else if (!(fabs(tot[1]) > S->eps * sqrt(tot[0]) * sqrt(tot[2]))) {
        S->status = 3;  // breakdown: rho' ~ 0
        S->done = 1;
      } else {
        S->beta = beta_d;
        S->rho = tot[1];
        S->rho_par[par ^ 1] = tot[1];
      }
    }
  }
  if (!REFRESH && KB > 0) {
    // projected recurrences, one column per block (block j reduces column j
    // of w = Vhat^T D^-1 q from the M_mr partials): Vhat^T t -= alpha w,
    // Vhat^T p = Vhat^T t + beta Vhat^T p.  On a stopping iteration the
    // update is unused (the next inner solve starts them afresh).
    for (int j = blockIdx.x; j < k; j += gridDim.x) {
      double wj[1];
      block_sum_cols<1>(part_w + 1 + j, nb_w, 1 + k, wj);
      if (threadIdx.x == 0) {
        const double vt = S->vt[j] - S->alpha * wj[0];
        const double sj = vt + beta_d * S->s[j];
        S->vt[j] = vt;
        S->s[j] = sj;
        S->cs_[j] = S->c[j] * sj;
      }
    }
  }
  const T beta = (T)beta_d;
  if constexpr (!REFRESH || KB == 0) {
    constexpr int U = 4;
    const int stride = gridDim.x * MCG_BLOCK;
    for (int base = blockIdx.x * MCG_BLOCK + threadIdx.x; base < n; base += U * stride) {
      T tv[U], pv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = min(base + u * stride, n - 1);
        tv[u] = dinv[i] * r[i];
        pv[u] = p[i];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = base + u * stride;
        if (i < n) p[i] = tv[u] + beta * pv[u];
      }
    }
  } else {
    constexpr int K2 = 2 * KB;
    T acc2[K2];
#pragma unroll
    for (int j = 0; j < K2; ++j) acc2[j] = 0;
    for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
      const T ti = dinv[i] * r[i];
      const T pi = ti + beta * p[i];
      p[i] = pi;
      T vr[KB];
      vhat_row<KB, T>(V, n, k, i, vr);
#pragma unroll
      for (int j = 0; j < KB; ++j) {
        acc2[j] += vr[j] * pi;
        acc2[KB + j] += vr[j] * ti;
      }
    }
    double v2[K2];
#pragma unroll
    for (int j = 0; j < K2; ++j) v2[j] = (double)acc2[j];
    block_partials<K2>(v2, K2, part_out);  // finished by k_finalize(FIN_REFRESH)
  }
}

// Inner solve start, diagonal M_cg: r = y * inv_scale, z = 0, t = dinv o r,
// p = t; rho = r^T t, yy = r^T r, s = Vhat^T p.  TY is the type of y.
template <typename T, typename TY, int KB>
__global__ __launch_bounds__(MCG_BLOCK) void k_cg_init_diag(
    int n, const TY *__restrict__ y, T *__restrict__ z, T *__restrict__ r, T *__restrict__ p,
    const T *__restrict__ dinv, const T *__restrict__ V, int k, DevState *__restrict__ S,
    double *part, unsigned *ticket) {
  constexpr int W = KB + 3;
  const double inv_scale = S->inv_scale;
  T acc[KB > 0 ? KB : 1];
#pragma unroll
  for (int j = 0; j < (KB > 0 ? KB : 1); ++j) acc[j] = 0;
  T rr = 0, rt = 0, tt = 0;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    const T ri = (T)((double)y[i] * inv_scale);
    const T ti = dinv[i] * ri;
    r[i] = ri;
    z[i] = 0;
    p[i] = ti;
    rr += ri * ri;
    rt += ri * ti;
    tt += ti * ti;
    T vr[KB > 0 ? KB : 1];
    vhat_row<KB, T>(V, n, k, i, vr);
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] += vr[j] * ti;
  }
  double v[W];
  v[0] = (double)rr;
  v[1] = (double)rt;
  v[2] = (double)tt;
#pragma unroll
  for (int j = 0; j < KB; ++j) v[3 + j] = (double)acc[j];
  __shared__ double tot[W];
  if (grid_sum<W>(v, 3 + k, part, ticket, tot)) {
    if (threadIdx.x < k) {
      S->s[threadIdx.x] = tot[3 + threadIdx.x];
      S->vt[threadIdx.x] = tot[3 + threadIdx.x];  // p0 = t0
      S->cs_[threadIdx.x] = S->c[threadIdx.x] * tot[3 + threadIdx.x];
    }
    if (threadIdx.x == 0) {
      S->its = 0;
      S->yy = tot[0];
      S->rr = tot[0];
      S->rho = tot[1];
      S->rho_par[0] = tot[1];
      S->status = 0;
      if (tot[0] == 0.0) {
        S->done = 1;  // y = 0: z = 0 is exact
      } else if (!(fabs(tot[1]) > S->eps * sqrt(tot[0]) * sqrt(tot[2]))) {
        S->status = 3;
        S->done = 1;
      } else {
        S->done = 0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// General M_cg (triangular sweeps, C C^T, SMW form): the preconditioner
// writes t; these kernels do the remaining CG pieces.
// ---------------------------------------------------------------------------

// r = y * inv_scale, z = 0, yy = r^T r
template <typename T, typename TY>
__global__ __launch_bounds__(MCG_BLOCK) void k_cg_init_r(int n, const TY *__restrict__ y,
                                                         T *__restrict__ z, T *__restrict__ r,
                                                         DevState *__restrict__ S, double *part,
                                                         unsigned *ticket) {
  const double inv_scale = S->inv_scale;
  T rr = 0;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    const T ri = (T)((double)y[i] * inv_scale);
    r[i] = ri;
    z[i] = 0;
    rr += ri * ri;
  }
  double v[1] = {(double)rr};
  __shared__ double tot[1];
  if (grid_sum<1>(v, 1, part, ticket, tot) && threadIdx.x == 0) {
    S->its = 0;
    S->yy = tot[0];
    S->rr = tot[0];
    S->status = 0;
    S->done = (tot[0] == 0.0) ? 1 : 0;
  }
}

// General M_cg, step 1 (no finalize before it): alpha = rho / pi from the
// M_mr apply's compact per-block pi; z += alpha p; r -= alpha q; per-block
// r^T r into rr_out (compact).  pi <= 0: NOT_SPD.
template <typename T>
__global__ __launch_bounds__(MCG_BLOCK) void k_cg_update_gen_f(
    int n, T *__restrict__ z, T *__restrict__ r, const T *__restrict__ p,
    const T *__restrict__ q, DevState *__restrict__ S, const double *__restrict__ pi_in,
    int nb_in, double *__restrict__ rr_out, int par) {
  if (S->done) return;
  double pi[1];
  block_sum_cols<1>(pi_in, nb_in, 1, pi);
  const bool spd = pi[0] > 0.0;
  const double alpha_d = spd ? S->rho_par[par] / pi[0] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S->pi = pi[0];
    S->alpha = alpha_d;
    if (!spd) {
      S->status = 4;  // MCG_NOT_SPD
      S->done = 1;
    }
  }
  if (!spd) return;
  const T alpha = (T)alpha_d;
  T rr = 0;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    const T zi = z[i] + alpha * p[i];
    const T ri = r[i] - alpha * q[i];
    z[i] = zi;
    r[i] = ri;
    rr += ri * ri;
  }
  double v[1] = {(double)rr};
  block_partials<1>(v, 1, rr_out);
}

// General M_cg, direction step (t = M_cg^{-1} r given): from the compact
// r^T t of the kernel that formed t (nb_rho blocks; rows of (r^T t, t^T t)
// for block 0) and the update's compact r^T r (nb_upd blocks): stop tests
// and breakdown guard (block 0 records its, rr, status/done, rho in the other
// parity slot), beta = r^T t / rho; p = t + beta p with block partials of
// Vhat^T p (FIN_VTP).  first = 1 starts a solve (beta = 0, no stop test).
template <typename T, int KB>
__global__ __launch_bounds__(MCG_BLOCK) void k_cg_dir_gf(
    int n, T *__restrict__ p, const T *__restrict__ t, const T *__restrict__ V, int k,
    DevState *__restrict__ S, const double *__restrict__ rt_in,
    const double *__restrict__ rows_in, int nb_rho, const double *__restrict__ rr_in,
    int nb_upd, double *__restrict__ part_out, int first, int par) {
  if (S->done) return;
  double rts[1];
  block_sum_cols<1>(rt_in, nb_rho, 1, rts);
  const double beta_d = first ? 0.0 : rts[0] / S->rho_par[par];
  if (blockIdx.x == 0) {
    double tot2[2];  // r^T t, t^T t
    block_sum_cols<2>(rows_in, nb_rho, 2, tot2);
    double rr1[1] = {0.0};
    if (!first) block_sum_cols<1>(rr_in, nb_upd, 1, rr1);
    if (threadIdx.x == 0) {
      bool stop = false;
      double rr = S->rr;
      if (!first) {
        rr = rr1[0];
        const int64_t its = S->its + 1;
        S->its = its;
        S->rr = rr;
        if (rr <= S->rtol2 * S->yy) {
          S->status = 0;
          stop = true;
        } else if (its >= S->maxit) {
          S->status = 1;
          stop = true;
        }
      }
      if (!stop && !(fabs(rts[0]) > S->eps * sqrt(rr) * sqrt(tot2[1]))) {
        S->status = 3;  // breakdown: rho' ~ 0
        stop = true;
      }
      if (stop) {
        S->done = 1;
      } else {
        S->beta = beta_d;
        S->rho = rts[0];
        S->rho_par[par ^ 1] = rts[0];
      }
    }
  }
  const T beta = (T)beta_d;
  constexpr int KW = KB > 0 ? KB : 1;
  T acc[KW];
#pragma unroll
  for (int j = 0; j < KW; ++j) acc[j] = 0;
  constexpr int U = 2;
  const int stride = gridDim.x * MCG_BLOCK;
  for (int base = blockIdx.x * MCG_BLOCK + threadIdx.x; base < n; base += U * stride) {
    T tv[U], pv[U], vr[U][KW];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = min(base + u * stride, n - 1);
      tv[u] = t[i];
      pv[u] = first ? (T)0 : p[i];
      vhat_row<KB, T>(V, n, k, i, vr[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * stride;
      if (i < n) {
        const T pi = tv[u] + beta * pv[u];
        p[i] = pi;
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] += vr[u][j] * pi;
      }
    }
  }
  if constexpr (KB == 0) {
    return;
  } else if constexpr (sizeof(T) == 4) {
    block_partials_f<KB>(acc, k, part_out);  // finished by k_finalize(FIN_VTP)
  } else {
    double v[KW];
#pragma unroll
    for (int j = 0; j < KW; ++j) v[j] = (double)acc[j];
    block_partials<KW>(v, k, part_out);  // finished by k_finalize(FIN_VTP)
  }
}

// r^T t and t^T t of a formed t (block partials: rows in part, r^T t also in
// compact), finished by k_cg_dir_gf.
template <typename T>
__global__ __launch_bounds__(MCG_BLOCK) void k_cg_rho(int n, const T *__restrict__ r,
                                                      const T *__restrict__ t,
                                                      DevState *__restrict__ S, double *part,
                                                      double *__restrict__ compact) {
  if (S->done) return;
  T rt = 0, tt = 0;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    const T ti = t[i];
    rt += r[i] * ti;
    tt += ti * ti;
  }
  double v[2] = {(double)rt, (double)tt};
  block_partials<2>(v, 2, part, compact);  // finished by k_cg_dir_gf
}

// ---------------------------------------------------------------------------
// a3/a4 with M_cg = C C^T (C lower triangular, the learned factor): after
// z += alpha p, r -= alpha q (k_cg_update_gen) and u = C^T r, one pass forms
// t = C u with r^T t and t^T t (finished by FIN_RHO); the direction kernel
// k_cg_dir then streams p = t + beta p together with Vhat^T p.  (Reading the
// Vhat rows inside this CSR-tile kernel made it latency-bound; the streaming
// direction pass reads them at full rate.)
// ---------------------------------------------------------------------------
template <int L, typename T>
__global__ __launch_bounds__(MCG_BLOCK) void k_cct_t(int n, const int32_t *__restrict__ c_rp,
                                                     const int32_t *__restrict__ c_ci,
                                                     const T *__restrict__ c_v,
                                                     const T *__restrict__ u, T *__restrict__ t,
                                                     const T *__restrict__ r,
                                                     const DevState *__restrict__ S,
                                                     double *__restrict__ part,
                                                     double *__restrict__ compact) {
  if (S->done) return;
  __shared__ T tile[MCG_BLOCK];
  T rt = 0, tt = 0;
  for (int row0 = blockIdx.x * MCG_BLOCK; row0 < n; row0 += gridDim.x * MCG_BLOCK) {
    const int row = row0 + threadIdx.x;
    const T rv = r[row < n ? row : n - 1];
    csr_tile<L, T, T>(n, row0, c_rp, c_ci, c_v, u, tile);
    __syncthreads();
    if (row < n) {
      const T ti = tile[threadIdx.x];
      t[row] = ti;
      rt += rv * ti;
      tt += ti * ti;
    }
    __syncthreads();
  }
  double v[2] = {(double)rt, (double)tt};
  block_partials<2>(v, 2, part, compact);  // finished by k_cg_dir_gf
}

// t = C u from the sliced copy of C, with the partials of r^T t and t^T t
// (the sliced counterpart of k_cct_t), two slices per wavefront
template <typename T, typename IDX, int G = 8, typename TV = T>
__global__ __launch_bounds__(MCG_BLOCK) void k_sell_cct_t(int n, int nslices,
                                                          const int64_t *__restrict__ off,
                                                          const IDX *__restrict__ col,
                                                          const TV *__restrict__ val,
                                                          const T *__restrict__ u,
                                                          T *__restrict__ t,
                                                          const T *__restrict__ r,
                                                          const DevState *__restrict__ S,
                                                          double *__restrict__ part,
                                                          double *__restrict__ compact) {
  if (S->done) return;
  const int lane = threadIdx.x & 63;
  T rt = 0, tt = 0;
  for (int wv = blockIdx.x * MCG_NWAVE + (threadIdx.x >> 6); 2 * wv < nslices;
       wv += gridDim.x * MCG_NWAVE) {
    const int s0 = 2 * wv, s1 = min(s0 + 1, nslices - 1);
    const int r0 = s0 * 64 + lane, r1 = (s0 + 1) * 64 + lane;
    const T rv0 = r[r0 < n ? r0 : n - 1], rv1 = r[r1 < n ? r1 : n - 1];
    T t0, t1;
    sell_rows2<T, IDX, G, TV>(off, col, val, u, s0, s1, lane, t0, t1);
    if (r0 < n) {
      t[r0] = t0;
      rt += rv0 * t0;
      tt += t0 * t0;
    }
    if (s0 + 1 < nslices && r1 < n) {
      t[r1] = t1;
      rt += rv1 * t1;
      tt += t1 * t1;
    }
  }
  double v[2] = {(double)rt, (double)tt};
  block_partials<2>(v, 2, part, compact);  // finished by k_cg_dir_gf
}

// MINRES-CG*: u = Vhat^T g (into S->u), then t += Vhat (smw o u)
template <typename T, int KB>
__global__ __launch_bounds__(MCG_BLOCK) void k_smw_vtg(int n, const T *__restrict__ g,
                                                       const T *__restrict__ V, int k,
                                                       DevState *__restrict__ S, double *part,
                                                       unsigned *ticket, int check_done) {
  if (check_done && S->done) return;
  T acc[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) acc[j] = 0;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    const T gi = g[i];
    T vr[KB];
    vhat_row<KB, T>(V, n, k, i, vr);
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] += vr[j] * gi;
  }
  double v[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) v[j] = (double)acc[j];
  block_partials<KB>(v, k, part);  // finished by k_finalize(FIN_SMW)
}

template <typename T, int KB>
__global__ __launch_bounds__(MCG_BLOCK) void k_smw_add(int n, T *__restrict__ t,
                                                       const T *__restrict__ V, int k,
                                                       const DevState *__restrict__ S,
                                                       int check_done) {
  if (check_done && S->done) return;
  __shared__ T u[KB];
  if (threadIdx.x < KB) u[threadIdx.x] = threadIdx.x < k ? (T)S->u[threadIdx.x] : (T)0;
  __syncthreads();
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    T vr[KB];
    vhat_row<KB, T>(V, n, k, i, vr);
    T acc = t[i];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc += vr[j] * u[j];
    t[i] = acc;
  }
}

// t = dinv o g (Jacobi / identity applied standalone or before the SMW term)
template <typename T>
__global__ __launch_bounds__(MCG_BLOCK) void k_diag_apply(int n, const T *__restrict__ dinv,
                                                          const T *__restrict__ g,
                                                          T *__restrict__ t,
                                                          const DevState *__restrict__ S,
                                                          int check_done) {
  if (check_done && S->done) return;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK)
    t[i] = dinv[i] * g[i];
}

// ---------------------------------------------------------------------------
// a6/a7: outer MINRES (FP64)
// ---------------------------------------------------------------------------

// rt = b - A x; rt2 = ||rt||^2, bb = ||b||^2
template <int L>
__global__ __launch_bounds__(MCG_BLOCK) void k_resid(int n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const double *__restrict__ va,
                                                     const double *__restrict__ x,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ rt,
                                                     DevState *__restrict__ S, double *part,
                                                     unsigned *ticket) {
  __shared__ double tile[MCG_BLOCK];
  double r2 = 0.0, b2 = 0.0;
  for (int row0 = blockIdx.x * MCG_BLOCK; row0 < n; row0 += gridDim.x * MCG_BLOCK) {
    csr_tile<L, double, double>(n, row0, rp, ci, va, x, tile);
    __syncthreads();
    const int row = row0 + threadIdx.x;
    if (row < n) {
      const double bi = b[row];
      const double ri = bi - tile[threadIdx.x];
      rt[row] = ri;
      r2 += ri * ri;
      b2 += bi * bi;
    }
    __syncthreads();
  }
  double v[2] = {r2, b2};
  __shared__ double tot[2];
  if (grid_sum<2>(v, 2, part, ticket, tot) && threadIdx.x == 0) {
    S->rt2 = tot[0];
    S->bb = tot[1];
  }
}

// Lanczos, first half: v = y / beta; r1 <- A v - (beta / oldb) r1 (the
// second term from the second iteration on); alfa = v^T r1.
template <int L>
__global__ __launch_bounds__(MCG_BLOCK) void k_lanczos_a(int n, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci,
                                                         const double *__restrict__ va,
                                                         const double *__restrict__ y,
                                                         double *__restrict__ v,
                                                         double *__restrict__ r1,
                                                         DevState *__restrict__ S,
                                                         double *part, unsigned *ticket,
                                                         int first) {
  __shared__ double tile[MCG_BLOCK];
  const double beta = S->beta_cur;
  const double sc = 1.0 / beta;
  const double f = first ? 0.0 : beta / S->oldb;
  double va_ = 0.0;
  for (int row0 = blockIdx.x * MCG_BLOCK; row0 < n; row0 += gridDim.x * MCG_BLOCK) {
    csr_tile<L, double, double>(n, row0, rp, ci, va, y, tile);
    __syncthreads();
    const int row = row0 + threadIdx.x;
    if (row < n) {
      const double vi = sc * y[row];
      v[row] = vi;
      double yi = sc * tile[threadIdx.x];
      if (!first) yi -= f * r1[row];
      r1[row] = yi;
      va_ += vi * yi;
    }
    __syncthreads();
  }
  double vv[1] = {va_};
  __shared__ double tot[1];
  if (grid_sum<1>(vv, 1, part, ticket, tot) && threadIdx.x == 0) S->alfa = tot[0];
}

// Lanczos, second half: r1 <- r1 - (alfa / beta) r2; ||r1||^2 gives the
// scale of the precision boundary (mixed) or 1 (FP64).
static __global__ __launch_bounds__(MCG_BLOCK) void k_lanczos_b(int n, double *__restrict__ r1,
                                                         const double *__restrict__ r2,
                                                         DevState *__restrict__ S, double *part,
                                                         unsigned *ticket, int scaled) {
  const double f = S->alfa / S->beta_cur;
  double nn = 0.0;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    const double yi = r1[i] - f * r2[i];
    r1[i] = yi;
    nn += yi * yi;
  }
  double v[1] = {nn};
  __shared__ double tot[1];
  if (grid_sum<1>(v, 1, part, ticket, tot) && threadIdx.x == 0) {
    const double s = sqrt(tot[0]);
    S->scale = scaled ? s : 1.0;
    S->inv_scale = scaled ? (s > 0.0 ? 1.0 / s : 0.0) : 1.0;
  }
}

// scale of the boundary for an arbitrary FP64 vector (first inner solve)
static __global__ __launch_bounds__(MCG_BLOCK) void k_set_scale(int n, const double *__restrict__ y,
                                                         DevState *__restrict__ S, double *part,
                                                         unsigned *ticket, int scaled) {
  double nn = 0.0;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    const double yi = y[i];
    nn += yi * yi;
  }
  double v[1] = {nn};
  __shared__ double tot[1];
  if (grid_sum<1>(v, 1, part, ticket, tot) && threadIdx.x == 0) {
    const double s = sqrt(tot[0]);
    S->scale = scaled ? s : 1.0;
    S->inv_scale = scaled ? (s > 0.0 ? 1.0 / s : 0.0) : 1.0;
  }
}

// After an inner solve: y = scale * z (back to FP64), beta^2 = r2^T y, then
// either start the Givens recurrences (first) or apply the previous
// rotation and build the new one; also records the inner iteration count.
template <typename T>
__global__ __launch_bounds__(MCG_BLOCK) void k_outer_post(int n, const T *__restrict__ z,
                                                          double *__restrict__ y,
                                                          const double *__restrict__ r2,
                                                          DevState *__restrict__ S,
                                                          double *part, unsigned *ticket,
                                                          int first, int64_t *hist, int idx) {
  const double scale = S->scale;
  double b2 = 0.0;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    const double yi = scale * (double)z[i];
    y[i] = yi;
    b2 += r2[i] * yi;
  }
  double v[1] = {b2};
  __shared__ double tot[1];
  if (grid_sum<1>(v, 1, part, ticket, tot) && threadIdx.x == 0) {
    if (hist) hist[idx] = S->its;
    const double beta2 = tot[0];
    S->beta2 = beta2;
    if (!(beta2 >= 0.0)) {
      S->outer_flag = 1;  // M^{-1} not positive along r2, or NaN
      return;
    }
    const double beta = sqrt(beta2);
    if (first) {
      S->beta_cur = beta;
      S->oldb = 0.0;
      S->dbar = 0.0;
      S->epsln = 0.0;
      S->phibar = beta;
      S->cs = -1.0;
      S->sn = 0.0;
    } else {
      S->oldb = S->beta_cur;
      S->beta_cur = beta;
      const double alfa = S->alfa, cs = S->cs, sn = S->sn, dbar = S->dbar;
      S->oldeps = S->epsln;
      S->delta = cs * dbar + sn * alfa;
      const double gbar = sn * dbar - cs * alfa;
      S->epsln = sn * beta;
      S->dbar = -cs * beta;
      double gamma = hypot(gbar, beta);
      if (gamma < 2.220446049250313e-16) gamma = 2.220446049250313e-16;
      S->gamma = gamma;
      S->cs = gbar / gamma;
      S->sn = beta / gamma;
      S->phi = S->cs * S->phibar;
      S->phibar = S->sn * S->phibar;
    }
  }
}

// w = (v - oldeps w1 - delta w2) / gamma;  x += phi w
static __global__ __launch_bounds__(MCG_BLOCK) void k_outer_update(int n, double *__restrict__ w,
                                                            const double *__restrict__ w1,
                                                            const double *__restrict__ w2,
                                                            const double *__restrict__ v,
                                                            double *__restrict__ x,
                                                            const DevState *__restrict__ S) {
  const double oldeps = S->oldeps, delta = S->delta, ig = 1.0 / S->gamma, phi = S->phi;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    const double wi = (v[i] - oldeps * w1[i] - delta * w2[i]) * ig;
    w[i] = wi;
    x[i] += phi * wi;
  }
}

// ---------------------------------------------------------------------------
// Finalize kernels of the CG iteration: one block sums the partials that the
// preceding kernel wrote (the kernel boundary makes them visible, so no
// block of the streaming kernels needs a device-scope fence) and updates the
// device-resident scalars.
// ---------------------------------------------------------------------------
enum FinKind {
  FIN_REFRESH = 2,      // Vhat^T p, Vhat^T t recomputed                    [2 KB]
  FIN_VTP = 3,          // Vhat^T p                                          [k]
  FIN_SMW = 6           // Vhat^T g -> u = (-2/lambda) o Vhat^T g            [k]
};

static __global__ __launch_bounds__(1024) void k_finalize(int kind, DevState *__restrict__ S,
                                                   const double *__restrict__ part, int nb,
                                                   int w, int a, int check_done) {
  if (check_done && S->done) return;
  __shared__ double tot[2 * MCG_KMAX + 4];
  sum_partials(part, nb, w, tot);
  const int t = threadIdx.x;
  switch (kind) {
    case FIN_REFRESH: {  // layout [s_0..s_{KB-1}, vt_0..vt_{KB-1}], a = k
      const int KBv = w / 2;
      if (t < a) {
        S->s[t] = tot[t];
        S->cs_[t] = S->c[t] * tot[t];
        S->vt[t] = tot[KBv + t];
      }
      break;
    }
    case FIN_VTP:
      if (t < w) {
        S->s[t] = tot[t];
        S->cs_[t] = S->c[t] * tot[t];
      }
      break;
    case FIN_SMW:
      if (t < w) S->u[t] = S->smw[t] * tot[t];
      break;
  }
}

// ---------------------------------------------------------------------------
// setup helpers
// ---------------------------------------------------------------------------

// dinv[i] = 1 / a_ii (identity: ones); bad[0] counts missing / zero diagonals
template <typename T>
__global__ void k_jacobi_setup(int n, const int32_t *__restrict__ rp,
                               const int32_t *__restrict__ ci, const double *__restrict__ va,
                               T *__restrict__ dinv, int identity, unsigned *bad) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (identity) {
      dinv[i] = (T)1;
      continue;
    }
    double d = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p)
      if (ci[p] == i) d = va[p];
    if (d == 0.0 || !isfinite(d)) {
      atomicAdd(bad, 1u);
      dinv[i] = (T)0;
    } else {
      dinv[i] = (T)(1.0 / d);
    }
  }
}

template <typename T>
__global__ void k_fill(int64_t n, T value, T *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = value;
}

template <typename TO, typename TI>
__global__ void k_convert(int64_t n, const TI *__restrict__ in, TO *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (TO)in[i];
}

// count non-finite values
static __global__ void k_count_nonfinite(int64_t n, const double *__restrict__ a, unsigned *bad) {
  unsigned c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(a[i])) ++c;
  if (c) atomicAdd(bad, c);
}
