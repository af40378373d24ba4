// Host side of the solver (handles, inner and outer solve loops) and the C ABI of
// libminrescg.so (see include/minres_cg.h).
//
// One solver handle owns: the CSR copy of A (FP64, plus an FP32 shadow in
// mixed precision), Vhat (same), the solve workspace, device-resident
// scalars (DevState), reduction partials and pinned host mirrors used to
// poll the inner stop flag.  Nothing is allocated inside a solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "mcg_internal.h"

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) {                             \
      mcg_last_hip_error = e_;                          \
      return e_ == hipErrorOutOfMemory ? MCG_ENOMEM : MCG_EHIP; \
    }                                                   \
  } while (0)

std::atomic<hipError_t> mcg_last_hip_error{hipSuccess};

static inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Vhat column buckets: kernels are instantiated for these widths; a k below
// its bucket re-reads column k-1 (cache hits) for the padding columns.
int mcg_kb_bucket(int k) {
  static const int buckets[] = {4, 8, 12, 16, 20, 24, 32, 40, 48, 64};
  if (k <= 0) return 0;
  for (int b : buckets)
    if (k <= b) return b;
  return 64;
}

static int lanes_heuristic(int64_t nnz, int n) {
  double mean = n > 0 ? (double)nnz / n : 1.0;
  int L = 2;
  while (L < 64 && L < mean) L *= 2;
  return L;
}

int mcg_grid_tile(const mcg_solver *h) { return std::max(1, std::min(ceil_div(h->n, MCG_BLOCK), h->grid_tile_max)); }
int mcg_grid_stream(const mcg_solver *h) { return std::max(1, std::min(ceil_div(h->n, MCG_BLOCK), h->grid_stream_max)); }

template <typename T>
static int dev_alloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  HIP_TRY(hipMalloc((void **)p, count * sizeof(T)));
  return MCG_OK;
}

static void dev_free(void *p) {
  if (p) (void)hipFree(p);
}

// ---------------------------------------------------------------------------
// kernel dispatch (lanes L, Vhat bucket KB, precision T)
// ---------------------------------------------------------------------------
#define MCG_SWITCH_L(Lv, ...)                             \
  switch (Lv) {                                           \
    case 1: { constexpr int L = 1; __VA_ARGS__; } break;  \
    case 2: { constexpr int L = 2; __VA_ARGS__; } break;  \
    case 4: { constexpr int L = 4; __VA_ARGS__; } break;  \
    case 8: { constexpr int L = 8; __VA_ARGS__; } break;  \
    case 16: { constexpr int L = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int L = 32; __VA_ARGS__; } break; \
    default: { constexpr int L = 64; __VA_ARGS__; } break; \
  }

#define MCG_SWITCH_KB(KBv, ...)                            \
  switch (KBv) {                                           \
    case 0: { constexpr int KB = 0; __VA_ARGS__; } break;  \
    case 4: { constexpr int KB = 4; __VA_ARGS__; } break;  \
    case 8: { constexpr int KB = 8; __VA_ARGS__; } break;  \
    case 12: { constexpr int KB = 12; __VA_ARGS__; } break; \
    case 16: { constexpr int KB = 16; __VA_ARGS__; } break; \
    case 20: { constexpr int KB = 20; __VA_ARGS__; } break; \
    case 24: { constexpr int KB = 24; __VA_ARGS__; } break; \
    case 32: { constexpr int KB = 32; __VA_ARGS__; } break; \
    case 40: { constexpr int KB = 40; __VA_ARGS__; } break; \
    case 48: { constexpr int KB = 48; __VA_ARGS__; } break; \
    default: { constexpr int KB = 64; __VA_ARGS__; } break; \
  }

template <typename T>
static const T *valsT(const mcg_solver *h);
template <>
const double *valsT<double>(const mcg_solver *h) { return h->va; }
template <>
const float *valsT<float>(const mcg_solver *h) { return h->va32; }
template <typename T>
static const T *VT(const mcg_solver *h);
template <>
const double *VT<double>(const mcg_solver *h) { return h->V; }
template <>
const float *VT<float>(const mcg_solver *h) { return h->V32; }
template <typename T>
static const T *dinvT(const mcg_pc *p);
template <>
const double *dinvT<double>(const mcg_pc *p) { return p->dinv64; }
template <>
const float *dinvT<float>(const mcg_pc *p) { return p->dinv32; }

template <typename T>
static const T *bsr_valsT(const mcg_solver *h);
template <>
const double *bsr_valsT<double>(const mcg_solver *h) { return h->b_v; }
template <>
const float *bsr_valsT<float>(const mcg_solver *h) { return h->b_v32; }

// y = A x with the block CSR copy (h->bsr_bs > 0); S != nullptr: done check
template <typename T>
static void launch_bsr(const mcg_solver *h, const T *x, T *y, const DevState *S, hipStream_t s) {
  if (h->bsa.bs) {  // sliced copy of the blocks (the kernel writes S only when folding)
    mcg_bsell_spmv<T>(h->bsa, x, y, const_cast<DevState *>(S), s);
    return;
  }
  constexpr int G = 16;  // lanes per block row (two blocks each in flight: 32 blocks)
  const int g = std::max(1, std::min(ceil_div(h->nbr, MCG_BLOCK / G), 4096));
  const T *bv = bsr_valsT<T>(h);
  switch (h->bsr_bs) {
    case 2:
      k_bsr_spmv<2, G, T><<<g, MCG_BLOCK, 0, s>>>(h->nbr, h->b_rp, h->b_ci, bv, x, y, S);
      break;
    case 3:
      k_bsr_spmv<3, G, T><<<g, MCG_BLOCK, 0, s>>>(h->nbr, h->b_rp, h->b_ci, bv, x, y, S);
      break;
    default:
      k_bsr_spmv<4, G, T><<<g, MCG_BLOCK, 0, s>>>(h->nbr, h->b_rp, h->b_ci, bv, x, y, S);
      break;
  }
}

// column type of the sliced ELL copy
#define MCG_SWITCH_IDX(bits, ...)                         \
  if ((bits) == 16) {                                     \
    using IDX = int16_t;                                  \
    __VA_ARGS__;                                          \
  } else {                                                \
    using IDX = int32_t;                                  \
    __VA_ARGS__;                                          \
  }

// y = A x with the sliced ELL copy (h->sa.bits > 0); S != nullptr: done check
template <typename T>
static void launch_sell(const mcg_solver *h, const T *x, T *y, const DevState *S, hipStream_t s) {
  mcg_sell_spmv<T>(h->sa, x, y, S, s);
}

// Grid of the one-pass M_mr apply over the sliced copy: a wavefront per
// slice, at most grid_tile_max blocks (their partials are summed by the
// consumer kernels).
static int sell_grid(const mcg_solver *h, const mcg_sell &A, int slices_per_wave = 1) {
  return std::max(1, std::min(ceil_div(A.nslices, MCG_NWAVE * slices_per_wave), h->grid_tile_max));
}

template <typename T, bool WQ>
static int launch_sell_mmr(const mcg_solver *h, const T *p, T *q, const T *dinv, DevState *S,
                           int stage, hipStream_t s, double *pi_compact) {
  const int g = sell_grid(h, h->sa);
  MCG_SWITCH_IDX(h->sa.bits, MCG_SWITCH_KB(h->kb, (k_sell_mmr<T, IDX, KB, WQ><<<g, MCG_BLOCK, 0, s>>>(
                                                   h->n, h->sa.nslices, h->sa.off,
                                                   (const IDX *)h->sa.col, mcg_sell_vals<T>(h->sa), p, q,
                                                   dinv, VT<T>(h), h->k, S, stage, h->part,
                                                   pi_compact))));
  return g;
}

template <typename T>
void mcg_launch_spmv(const mcg_solver *h, const T *x, T *y, hipStream_t s) {
  if (h->bsr_bs) {
    launch_bsr<T>(h, x, y, nullptr, s);
    return;
  }
  if (h->sa.bits) {
    launch_sell<T>(h, x, y, nullptr, s);
    return;
  }
  mcg_launch_spmv_csr<T>(h, x, y, s);
}

template <typename T>
void mcg_launch_spmv_csr(const mcg_solver *h, const T *x, T *y, hipStream_t s) {
  const int g = mcg_grid_tile(h);
  MCG_SWITCH_L(h->lanes, (k_spmv<L, T><<<g, MCG_BLOCK, 0, s>>>(h->n, h->rp, h->ci, valsT<T>(h), x, y)));
}

// M_mr apply with p^T q partials (stage_alpha = 1) or q only (0); returns
// the number of blocks that wrote partials
template <typename T>
static int launch_mmr(const mcg_solver *h, const T *p, T *q, DevState *S, int stage_alpha,
                      hipStream_t s, double *pi_compact = nullptr) {
  if (h->sa.bits)
    return launch_sell_mmr<T, false>(h, p, q, nullptr, S, stage_alpha, s, pi_compact);
  const int g = mcg_grid_tile(h);
  const T *V = VT<T>(h);
  MCG_SWITCH_L(h->lanes, MCG_SWITCH_KB(h->kb, (k_mmr<L, T, KB><<<g, MCG_BLOCK, 0, s>>>(
                                                   h->n, h->rp, h->ci, valsT<T>(h), p, q, V, h->k,
                                                   S, h->part, h->ticket, stage_alpha, nullptr,
                                                   pi_compact))));
  return g;
}

// partial-sum regions inside h->part2
static double *part_rows(const mcg_solver *h) { return h->part2; }
static double *pi_compact(const mcg_solver *h) { return h->part2 + 3 * (size_t)h->grid_tile_max; }
static double *rt_compact(const mcg_solver *h) { return h->part2 + 4 * (size_t)h->grid_tile_max; }
static double *rr_compact(const mcg_solver *h) { return h->part2 + 5 * (size_t)h->grid_tile_max; }

// Grid of the general direction kernel k_cg_dir_gf: at most 512 blocks (its
// k-wide closing reduction is paid once per block).
static int dir_grid(const mcg_solver *h) {
  return std::max(1, std::min(ceil_div(h->n, MCG_BLOCK), 512));
}

// With the split form over a sliced copy, the SpMV of the next M_mr apply
// finishes the direction kernel's Vhat^T p reduction (no finalize launch).
static bool fold_vtp(const mcg_solver *h) {
  return (h->sa.bits || h->bsa.bs) && h->mmr_split && h->k > 0;
}

// Ap = A p over the sliced copy (scalar or block) with per-block p^T A p in
// pap (compact); fold: also finish the direction kernel's Vhat^T p reduction.
// Returns the number of blocks that wrote pap.
template <typename T>
static int launch_spmv_pap(const mcg_solver *h, const T *p, T *Ap, bool fold, double *pap,
                           hipStream_t s) {
  if (h->bsa.bs)
    return mcg_bsell_spmv<T>(h->bsa, p, Ap, h->S, s, true, p, part_rows(h), pap,
                             fold ? h->part : nullptr, dir_grid(h), h->k);
  const mcg_sell &A = h->sa;
  const int g = std::max(1, std::min(ceil_div(A.nslices, 2 * MCG_NWAVE), 2048));
  MCG_SWITCH_IDX(A.bits, (k_sell_spmv_vtp<T, IDX><<<g, MCG_BLOCK, 0, s>>>(
                             h->n, A.nslices, A.off, (const IDX *)A.col, mcg_sell_vals<T>(A), p,
                             Ap, h->S, fold ? h->part : nullptr, dir_grid(h), h->k, pap)));
  return g;
}

// Grid of k_cg_update_v with the Jacobi (1 + k)-wide closing reduction: at
// most 384 blocks (measured fastest of 256..2048 on the 128^3 Laplacian)
static int update_v_grid(const mcg_solver *h) {
  return std::max(1, std::min(ceil_div(h->n, MCG_BLOCK), 384));
}

// M_mr apply of a general-M_cg iteration (q and p^T q): the split form
// (SpMV + streaming rank-k pass) when the autotuner chose it, else fused.
// Returns the number of blocks whose pi values the update kernel sums.
template <typename T>
static int launch_mmr_gen(const mcg_solver *h, const T *p, T *q, DevState *S, hipStream_t s,
                          double *pi_compact) {
  if (h->sa.bits && !h->mmr_split) return launch_sell_mmr<T, false>(h, p, q, nullptr, S, 1, s, pi_compact);
  if (h->mmr_split && h->k > 0) {
    const int gt = mcg_grid_tile(h), gs = mcg_grid_stream(h);
    if (h->bsa.bs) {
      mcg_bsell_spmv<T>(h->bsa, p, q, S, s, false, nullptr, nullptr, nullptr,
                        fold_vtp(h) ? h->part : nullptr, dir_grid(h), h->k);
    } else if (h->bsr_bs) {
      launch_bsr<T>(h, p, q, S, s);
    } else if (fold_vtp(h)) {
      const mcg_sell &A = h->sa;
      const int g = std::max(1, std::min(ceil_div(A.nslices, 2 * MCG_NWAVE), 2048));
      MCG_SWITCH_IDX(A.bits, (k_sell_spmv_vtp<T, IDX><<<g, MCG_BLOCK, 0, s>>>(
                                 h->n, A.nslices, A.off, (const IDX *)A.col, mcg_sell_vals<T>(A),
                                 p, q, S, h->part, dir_grid(h), h->k, nullptr)));
    } else if (h->sa.bits) {
      launch_sell<T>(h, p, q, S, s);
    } else {
      MCG_SWITCH_L(h->lanes, (k_spmv_chk<L, T><<<gt, MCG_BLOCK, 0, s>>>(h->n, h->rp, h->ci,
                                                                       valsT<T>(h), p, q, S)));
    }
    MCG_SWITCH_KB(h->kb, if constexpr (KB > 0) {
      k_mmr_vpart<T, KB, false><<<gs, MCG_BLOCK, 0, s>>>(h->n, p, q, nullptr, VT<T>(h), h->k, S,
                                                         h->part, pi_compact);
    });
    return gs;
  }
  return launch_mmr<T>(h, p, q, S, 1, s, pi_compact);
}

// one-block reduction of the partials of the previous kernel (nb blocks, w
// values each) and the scalar update that depends on them
static void fin(const mcg_solver *h, int kind, DevState *S, int nb, int w, int a, int check_done,
                hipStream_t s) {
  if (w <= 0) return;
  k_finalize<<<1, 1024, 0, s>>>(kind, S, h->part, nb, w, a, check_done);
}

template <typename T>
int mcg_launch_mmr_diag(const mcg_solver *h, const T *p, T *q, const T *dinv, DevState *S,
                        hipStream_t s, double *pi_compact) {
  if (h->sa.bits && !h->mmr_split) return launch_sell_mmr<T, true>(h, p, q, dinv, S, 1, s, pi_compact);
  const int gt = mcg_grid_tile(h);
  if (h->mmr_split) {
    const int gs = mcg_grid_stream(h);
    if (h->bsr_bs)
      launch_bsr<T>(h, p, q, S, s);
    else if (h->sa.bits)
      launch_sell<T>(h, p, q, S, s);
    else
      MCG_SWITCH_L(h->lanes, (k_spmv_chk<L, T><<<gt, MCG_BLOCK, 0, s>>>(h->n, h->rp, h->ci,
                                                                       valsT<T>(h), p, q, S)));
    // fewer, longer-lived blocks for the pass with the wide (1 + k) block
    // reduction: its closing reduction is paid once per block
    const int gv = std::max(1, std::min(ceil_div(h->n, MCG_BLOCK), 512));
    MCG_SWITCH_KB(h->kb, if constexpr (KB > 0) {
      k_mmr_vpart<T, KB><<<gv, MCG_BLOCK, 0, s>>>(h->n, p, q, dinv, VT<T>(h), h->k, S, h->part,
                                                  pi_compact);
    });
    return gv;
  } else {
    MCG_SWITCH_L(h->lanes, MCG_SWITCH_KB(h->kb, (k_mmr<L, T, KB, true><<<gt, MCG_BLOCK, 0, s>>>(
                                                     h->n, h->rp, h->ci, valsT<T>(h), p, q,
                                                     VT<T>(h), h->k, S, h->part, h->ticket, 1,
                                                     dinv, pi_compact))));
  }
  return gt;
}
template int mcg_launch_mmr_diag<double>(const mcg_solver *, const double *, double *,
                                         const double *, DevState *, hipStream_t, double *);
template int mcg_launch_mmr_diag<float>(const mcg_solver *, const float *, float *,
                                        const float *, DevState *, hipStream_t, double *);

template <typename T>
static void launch_vtu(const mcg_solver *h, const T *u, DevState *S, hipStream_t s) {
  if (h->k == 0) return;
  const int g = mcg_grid_stream(h);
  MCG_SWITCH_KB(h->kb, if constexpr (KB > 0) {
    k_vtu<T, KB><<<g, MCG_BLOCK, 0, s>>>(h->n, u, VT<T>(h), h->k, S, h->part, h->ticket);
  });
}

// ---------------------------------------------------------------------------
// preconditioner application inside the inner loop (general path): t = M^{-1} r
// ---------------------------------------------------------------------------
template <typename T>
static void launch_pc_apply(const mcg_pc *pc, const T *g, T *t, DevState *S, int check_done,
                            hipStream_t s) {
  const mcg_solver *h = pc->h;
  const int gs = mcg_grid_stream(h);
  switch (pc->base) {
    case MCG_PC_NONE:
    case MCG_PC_JACOBI:
      k_diag_apply<T><<<gs, MCG_BLOCK, 0, s>>>(h->n, dinvT<T>(pc), g, t, S, check_done);
      break;
    case MCG_PC_ILDL0:
      mcg_ildl0_apply<T>(pc, g, t, S, check_done, s);
      break;
    case MCG_PC_CCT:
      mcg_cct_apply<T>(pc, g, t, S, check_done, s);
      break;
    case MCG_PC_ILDLP:
      mcg_ildlp_apply<T>(pc, g, t, S, check_done, s);
      break;
  }
  if (pc->smw && h->k > 0) {
    MCG_SWITCH_KB(h->kb, if constexpr (KB > 0) {
      k_smw_vtg<T, KB><<<gs, MCG_BLOCK, 0, s>>>(h->n, g, VT<T>(h), h->k, S, h->part, h->ticket,
                                                check_done);
      fin(h, FIN_SMW, S, gs, h->k, 0, check_done, s);
      k_smw_add<T, KB><<<gs, MCG_BLOCK, 0, s>>>(h->n, t, VT<T>(h), h->k, S, check_done);
    });
  }
}

// ---------------------------------------------------------------------------
// inner solve: z = PCG(M_mr, M_cg; y * inv_scale), z0 = 0
// ---------------------------------------------------------------------------
__global__ void k_inner_params(DevState *S, int64_t maxit, double rtol2, double eps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    S->maxit = maxit;
    S->rtol2 = rtol2;
    S->eps = eps;
    S->done = 0;
    S->status = 0;
    S->its = 0;
  }
}

// Scalar hand-off between the inner-iteration kernels (no finalize
// launches): h->part2 holds rows of up to 3 partials per block, then compact
// per-block arrays of pi (M_mr apply), r^T t and r^T r.

// General M_cg, direction step: p = t + beta p, Vhat^T p (FIN_VTP)
template <typename T>
static void dir_general(mcg_solver *h, T *p, const T *t, int nb_rho, int first, int par,
                        hipStream_t s) {
  const int gs = mcg_grid_stream(h);
  const int gd = dir_grid(h);
  MCG_SWITCH_KB(h->kb, (k_cg_dir_gf<T, KB><<<gd, MCG_BLOCK, 0, s>>>(
                           h->n, p, t, VT<T>(h), h->k, h->S, rt_compact(h), part_rows(h), nb_rho,
                           rr_compact(h), gs, h->part, first, par)));
  if (!fold_vtp(h)) fin(h, FIN_VTP, h->S, gd, h->k, 0, 1, s);
}

// C C^T second level: u = C^T r; t = C u with r^T t, t^T t; then the
// direction step.  first = 1 starts a solve.
template <typename T>
static void cct_tail(mcg_solver *h, const mcg_cct_view &v, const T *r, T *t, T *p, int first,
                     int par, hipStream_t s) {
  T *u = (T *)v.tmp;
  const int gt = mcg_grid_tile(h), gs = mcg_grid_stream(h);
  if (v.c_bsell && v.ct_bsell) {
    // u = C^T r, then t = C u with the r^T t, t^T t partials
    mcg_bsell_spmv<T>(*v.ct_bsell, r, u, h->S, s);
    const int g = mcg_bsell_spmv<T>(*v.c_bsell, u, t, h->S, s, true, r, part_rows(h),
                                    rt_compact(h));
    dir_general<T>(h, p, t, g, first, par, s);
    return;
  }
  if (v.bsr) {
    constexpr int G = 16;
    const int g = std::max(1, std::min(ceil_div(v.nbr, MCG_BLOCK / G), 2048));
    const T *cbv = (const T *)v.cb_v, *ctbv = (const T *)v.ctb_v;
#define MCG_CCT_BSR(BSV)                                                                        \
  case BSV:                                                                                     \
    k_bsr_spmv<BSV, G, T><<<g, MCG_BLOCK, 0, s>>>(v.nbr, v.ctb_rp, v.ctb_ci, ctbv, r, u, h->S);  \
    k_bsr_spmv<BSV, G, T, true><<<g, MCG_BLOCK, 0, s>>>(v.nbr, v.cb_rp, v.cb_ci, cbv, u, t, h->S, \
                                                       r, part_rows(h), rt_compact(h));         \
    break;
    switch (v.bsr) {
      MCG_CCT_BSR(2)
      MCG_CCT_BSR(3)
      default:
      MCG_CCT_BSR(4)
    }
#undef MCG_CCT_BSR
    dir_general<T>(h, p, t, g, first, par, s);
    return;
  }
  if (v.c_sell) {
    // u = C^T r, then t = C u with the r^T t, t^T t partials
    mcg_sell_spmv<T>(*v.ct_sell, r, u, h->S, s);
    const mcg_sell &Cs = *v.c_sell;
    const int g = sell_grid(h, Cs, 2);
    bool done16 = false;
    if constexpr (sizeof(T) == 4) {
      if (Cs.v16) {  // FP16 values of C, FP32 arithmetic
        if (Cs.maxw <= 4) {
          MCG_SWITCH_IDX(Cs.bits, (k_sell_cct_t<T, IDX, 4, _Float16><<<g, MCG_BLOCK, 0, s>>>(
                                      h->n, Cs.nslices, Cs.off, (const IDX *)Cs.col, Cs.v16, u,
                                      t, r, h->S, part_rows(h), rt_compact(h))));
        } else {
          MCG_SWITCH_IDX(Cs.bits, (k_sell_cct_t<T, IDX, 8, _Float16><<<g, MCG_BLOCK, 0, s>>>(
                                      h->n, Cs.nslices, Cs.off, (const IDX *)Cs.col, Cs.v16, u,
                                      t, r, h->S, part_rows(h), rt_compact(h))));
        }
        done16 = true;
      }
    }
    if (done16) {
    } else if (Cs.maxw <= 4) {
      MCG_SWITCH_IDX(Cs.bits, (k_sell_cct_t<T, IDX, 4><<<g, MCG_BLOCK, 0, s>>>(
                                  h->n, Cs.nslices, Cs.off, (const IDX *)Cs.col,
                                  mcg_sell_vals<T>(Cs), u, t, r, h->S, part_rows(h),
                                  rt_compact(h))));
    } else {
      MCG_SWITCH_IDX(Cs.bits, (k_sell_cct_t<T, IDX, 8><<<g, MCG_BLOCK, 0, s>>>(
                                  h->n, Cs.nslices, Cs.off, (const IDX *)Cs.col,
                                  mcg_sell_vals<T>(Cs), u, t, r, h->S, part_rows(h),
                                  rt_compact(h))));
    }
    dir_general<T>(h, p, t, g, first, par, s);
    return;
  }
  mcg_csr_apply<T>(v.lanes, h->n, v.ct_rp, v.ct_ci, (const T *)v.ct_v, r, u, h->S, 1, s);
  double *rows = part_rows(h), *rtc = rt_compact(h);
  if (v.lanes <= 4)
    k_cct_t<4, T><<<gt, MCG_BLOCK, 0, s>>>(h->n, v.c_rp, v.c_ci, (const T *)v.c_v, u, t, r, h->S,
                                           rows, rtc);
  else if (v.lanes <= 16)
    k_cct_t<16, T><<<gt, MCG_BLOCK, 0, s>>>(h->n, v.c_rp, v.c_ci, (const T *)v.c_v, u, t, r,
                                            h->S, rows, rtc);
  else
    k_cct_t<32, T><<<gt, MCG_BLOCK, 0, s>>>(h->n, v.c_rp, v.c_ci, (const T *)v.c_v, u, t, r,
                                            h->S, rows, rtc);
  (void)gs;
  dir_general<T>(h, p, t, gt, first, par, s);
}

template <typename T, typename TY>
static void enqueue_inner_init(mcg_solver *h, const mcg_pc *pc, const TY *y, hipStream_t s) {
  T *z = (T *)h->z, *r = (T *)h->r, *p = (T *)h->p, *t = (T *)h->t;
  const int gs = mcg_grid_stream(h);
  if (pc->diag_path) {
    MCG_SWITCH_KB(h->kb, (k_cg_init_diag<T, TY, KB><<<gs, MCG_BLOCK, 0, s>>>(
                             h->n, y, z, r, p, dinvT<T>(pc), VT<T>(h), h->k, h->S, h->part,
                             h->ticket)));
  } else if (mcg_cct_view v; !pc->smw && mcg_cct_view_get(pc, sizeof(T) == 4, &v)) {
    // the start writes rho into parity slot 0 (par = 1), read by iteration 0
    k_cg_init_r<T, TY><<<gs, MCG_BLOCK, 0, s>>>(h->n, y, z, r, h->S, h->part, h->ticket);
    cct_tail<T>(h, v, r, t, p, 1, 1, s);
  } else {
    k_cg_init_r<T, TY><<<gs, MCG_BLOCK, 0, s>>>(h->n, y, z, r, h->S, h->part, h->ticket);
    launch_pc_apply<T>(pc, r, t, h->S, 1, s);
    k_cg_rho<T><<<gs, MCG_BLOCK, 0, s>>>(h->n, r, t, h->S, part_rows(h), rt_compact(h));
    dir_general<T>(h, p, t, gs, 1, 1, s);
  }
}

// Diagonal M_cg: Vhat^T p and Vhat^T t advance by k-vector recurrences (one
// pass over Vhat per iteration, inside the M_mr kernel); every
// kRefreshPeriod-th iteration recomputes both directly to bound their drift.
static constexpr int64_t kRefreshPeriod = 32;

template <typename T>
static void enqueue_inner_iteration(mcg_solver *h, const mcg_pc *pc, hipStream_t s,
                                    hipEvent_t *prof_pair, int64_t iter) {
  T *z = (T *)h->z, *r = (T *)h->r, *p = (T *)h->p, *q = (T *)h->q, *t = (T *)h->t;
  const int gs = mcg_grid_stream(h);
  if (prof_pair) (void)hipEventRecord(prof_pair[0], s);
  const int gt = mcg_grid_tile(h);
  mcg_cct_view cv;
  const bool cct = !pc->diag_path && !pc->smw && mcg_cct_view_get(pc, sizeof(T) == 4, &cv);
  const int par = (int)(iter & 1);
  if (!pc->diag_path) {
    if (fold_vtp(h)) {
      // Ap with p^T A p (finishing Vhat^T p), then the update forms q itself
      const int nb = launch_spmv_pap<T>(h, p, q, true, pi_compact(h), s);
      if (prof_pair && h->opt.profile == 2) (void)hipEventRecord(prof_pair[1], s);
      MCG_SWITCH_KB(h->kb, if constexpr (KB > 0) {
        k_cg_update_v<T, KB, false><<<gs, MCG_BLOCK, 0, s>>>(
            h->n, z, r, p, q, nullptr, VT<T>(h), h->k, h->S, pi_compact(h), nb, nullptr, nullptr,
            nullptr, rr_compact(h), par);
      });
      if (prof_pair && h->opt.profile != 2) (void)hipEventRecord(prof_pair[1], s);
    } else {
      const int nb = launch_mmr_gen<T>(h, p, q, h->S, s, pi_compact(h));
      if (prof_pair) (void)hipEventRecord(prof_pair[1], s);
      k_cg_update_gen_f<T><<<gs, MCG_BLOCK, 0, s>>>(h->n, z, r, p, q, h->S, pi_compact(h), nb,
                                                     rr_compact(h), par);
    }
    if (cct) {
      cct_tail<T>(h, cv, r, t, p, 0, par, s);
    } else {
      launch_pc_apply<T>(pc, r, t, h->S, 1, s);
      k_cg_rho<T><<<gs, MCG_BLOCK, 0, s>>>(h->n, r, t, h->S, part_rows(h), rt_compact(h));
      dir_general<T>(h, p, t, gs, 0, par, s);
    }
    return;
  }
  // Jacobi (diagonal M_cg)
  double *pi_c = pi_compact(h), *rt_c = rt_compact(h);
  const bool refresh = h->k > 0 && (iter % kRefreshPeriod) == kRefreshPeriod - 1;
  if (fold_vtp(h)) {
    // Ap with p^T A p; the update streams Vhat, forms q, updates z and r and
    // reduces (r^T t, r^T r, t^T t) and w = Vhat^T D^-1 q; the profiled unit
    // is that update kernel (the SpMV is timed on its own by the bench)
    const int nb = launch_spmv_pap<T>(h, p, q, false, pi_c, s);
    const int gv = update_v_grid(h);
    if (prof_pair && h->opt.profile == 2) (void)hipEventRecord(prof_pair[1], s);
    if (prof_pair && h->opt.profile != 2) (void)hipEventRecord(prof_pair[0], s);
    MCG_SWITCH_KB(h->kb, if constexpr (KB > 0) {
      k_cg_update_v<T, KB, true><<<gv, MCG_BLOCK, 0, s>>>(
          h->n, z, r, p, q, dinvT<T>(pc), VT<T>(h), h->k, h->S, pi_c, nb, h->part2, rt_c, h->part,
          nullptr, par);
    });
    if (prof_pair && h->opt.profile != 2) (void)hipEventRecord(prof_pair[1], s);
    if (refresh) {
      MCG_SWITCH_KB(h->kb, (k_cg_dir_f<T, KB, true><<<gs, MCG_BLOCK, 0, s>>>(
                               h->n, p, r, dinvT<T>(pc), VT<T>(h), h->k, h->S, h->part2, gv,
                               h->part, gv, h->part, rt_c, par)));
      fin(h, FIN_REFRESH, h->S, gs, 2 * h->kb, h->k, 1, s);
    } else {
      MCG_SWITCH_KB(h->kb, (k_cg_dir_f<T, KB, false><<<gs, MCG_BLOCK, 0, s>>>(
                               h->n, p, r, dinvT<T>(pc), VT<T>(h), h->k, h->S, h->part2, gv,
                               h->part, gv, h->part, rt_c, par)));
    }
    return;
  }
  const int nb_mmr = h->k > 0 ? mcg_launch_mmr_diag<T>(h, p, q, dinvT<T>(pc), h->S, s, pi_c)
                              : launch_mmr<T>(h, p, q, h->S, 1, s, pi_c);
  if (prof_pair) (void)hipEventRecord(prof_pair[1], s);
  {
    // the M_mr partials (pi, w) stay in h->part for both kernels below; the
    // update's partials go to h->part2
    k_cg_update_diag_f<T><<<gs, MCG_BLOCK, 0, s>>>(h->n, z, r, p, q, dinvT<T>(pc), h->S, pi_c,
                                                    nb_mmr, h->part2, rt_c, par);
    if (refresh) {
      MCG_SWITCH_KB(h->kb, (k_cg_dir_f<T, KB, true><<<gs, MCG_BLOCK, 0, s>>>(
                               h->n, p, r, dinvT<T>(pc), VT<T>(h), h->k, h->S, h->part2, gs,
                               h->part, nb_mmr, h->part, rt_c, par)));
      fin(h, FIN_REFRESH, h->S, gs, 2 * h->kb, h->k, 1, s);
    } else {
      MCG_SWITCH_KB(h->kb, (k_cg_dir_f<T, KB, false><<<gs, MCG_BLOCK, 0, s>>>(
                               h->n, p, r, dinvT<T>(pc), VT<T>(h), h->k, h->S, h->part2, gs,
                               h->part, nb_mmr, h->part, rt_c, par)));
    }
  }
}

// Adds the durations of the M_mr launches of a finished chunk that did work
// (iteration index below the inner iteration count reached).
static void prof_accumulate(mcg_solver *h, int slot, int64_t its) {
  const int used = h->prof_used[slot];
  for (int j = 0; j < used; ++j) {
    if (h->prof_first_iter[slot] + j >= its) break;
    float ms = 0.f;
    hipEvent_t *e = &h->prof_ev[2 * (slot * mcg_solver::kProfSlots + j)];
    if (hipEventElapsedTime(&ms, e[0], e[1]) == hipSuccess) {
      h->prof_ms += ms;
      h->prof_launches += 1;
    }
  }
  h->prof_used[slot] = 0;
}

// 32 inner iterations (one full period of the kernel sequence: parity slots
// alternate, the direct Vhat refresh comes every 32nd iteration) captured
// once per (handle, preconditioner, precision) on a private stream; nullptr
// if capture is not possible (the caller then launches eagerly).  Launches
// after the inner stop return at once, as in the eager path.
static constexpr int kGraphIters = 32;
// largest M_cg apply (kernel launches) that the 32-iteration graph captures
static constexpr int kMaxApplyLaunchesInGraph = 128;
static_assert(kGraphIters % kRefreshPeriod == 0, "graph must hold whole refresh periods");
template <typename T>
static hipGraphExec_t inner_graph(mcg_solver *h, const mcg_pc *pc_c) {
  mcg_pc *pc = const_cast<mcg_pc *>(pc_c);
  const int idx = sizeof(T) == 4 ? 1 : 0;
  if (pc->graph32[idx] || pc->graph_failed[idx]) return pc->graph32[idx];
  // no graph for a second level that launches many kernels per apply: the
  // captured period would hold kGraphIters times that many nodes
  if (pc->apply_launches > kMaxApplyLaunchesInGraph) {
    pc->graph_failed[idx] = true;
    return nullptr;
  }
  hipStream_t cs = nullptr;
  hipGraph_t g = nullptr;
  bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
            hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    for (int64_t i = 0; i < kGraphIters; ++i) enqueue_inner_iteration<T>(h, pc, cs, nullptr, i);
    ok = hipStreamEndCapture(cs, &g) == hipSuccess && g != nullptr;
  }
  if (ok) ok = hipGraphInstantiate(&pc->graph32[idx], g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (cs) (void)hipStreamDestroy(cs);
  (void)hipGetLastError();  // a failed capture leaves the eager path usable
  if (!ok) {
    pc->graph32[idx] = nullptr;
    pc->graph_failed[idx] = true;
  }
  return pc->graph32[idx];
}

// Runs the inner solve to completion (device decides when to stop; the host
// polls the stop flag after every chunk, keeping one chunk in flight).
template <typename T, typename TY>
static int run_inner(mcg_solver *h, const mcg_pc *pc, const TY *y, double rtol, int64_t maxit,
                     hipStream_t s, DevPoll *out) {
  const double eps = sizeof(T) == 8 ? 2.220446049250313e-16 : 1.1920928955078125e-07;
  k_inner_params<<<1, 64, 0, s>>>(h->S, maxit, rtol * rtol, eps);
  if (maxit <= 0) {
    // no iteration allowed: z = 0 (the start iterate) and the cap status,
    // so that nothing downstream reads a stale z
    k_fill<T><<<mcg_grid_stream(h), MCG_BLOCK, 0, s>>>(h->n, T(0), (T *)h->z);
    HIP_TRY(hipMemcpyAsync(&h->poll[0], h->S, sizeof(DevPoll), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *out = h->poll[0];
    out->status = MCG_MAXIT;
    out->its = 0;
    out->done = 1;
    h->last_inner_its = 0;
    return MCG_OK;
  }
  enqueue_inner_init<T, TY>(h, pc, y, s);
  int64_t chunk = h->opt.chunk > 0 ? h->opt.chunk
                                   : std::max<int64_t>(4, std::min<int64_t>(64, h->last_inner_its / 6));
  const bool prof = h->opt.profile != 0;
  if (prof) chunk = std::min<int64_t>(chunk, mcg_solver::kProfSlots);
  hipGraphExec_t graph = (!prof && !h->opt.eager) ? inner_graph<T>(h, pc) : nullptr;
  if (graph) chunk = std::max<int64_t>(1, (chunk + kGraphIters / 2) / kGraphIters) * kGraphIters;
  int slot = 0;
  bool have_prev = false;
  int64_t enqueued = 0;
  for (;;) {
    const int64_t c = std::min<int64_t>(chunk, std::max<int64_t>(1, maxit - enqueued));
    h->prof_first_iter[slot] = enqueued;
    h->prof_used[slot] = prof ? (int)c : 0;
    if (graph) {  // whole periods: iteration indices stay aligned to 32
      const int64_t reps = (c + kGraphIters - 1) / kGraphIters;
      for (int64_t r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(graph, s));
      enqueued += reps * kGraphIters;
    } else {
      for (int64_t i = 0; i < c; ++i)
        enqueue_inner_iteration<T>(h, pc, s,
                                   prof ? &h->prof_ev[2 * (slot * mcg_solver::kProfSlots + i)]
                                        : nullptr,
                                   enqueued + i);
      enqueued += c;
    }
    HIP_TRY(hipMemcpyAsync(&h->poll[slot], h->S, sizeof(DevPoll), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(h->ev[slot], s));
    if (have_prev) {
      HIP_TRY(hipEventSynchronize(h->ev[slot ^ 1]));
      prof_accumulate(h, slot ^ 1, h->poll[slot ^ 1].its);
      if (h->poll[slot ^ 1].done) {
        HIP_TRY(hipEventSynchronize(h->ev[slot]));
        prof_accumulate(h, slot, h->poll[slot].its);
        *out = h->poll[slot];
        break;
      }
    }
    if (enqueued >= maxit) {
      HIP_TRY(hipEventSynchronize(h->ev[slot]));
      prof_accumulate(h, slot, h->poll[slot].its);
      *out = h->poll[slot];
      break;
    }
    have_prev = true;
    slot ^= 1;
  }
  h->last_inner_its = out->its;
  return MCG_OK;
}

// ---------------------------------------------------------------------------
// handle lifecycle
// ---------------------------------------------------------------------------
extern "C" void minres_cg_default_options(mcg_options_t *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = MCG_PREC_FP64;
  opt->stag_window = 10;
  opt->keep_best = 1;
  opt->block_size = 1;
}

static int validate_csr_host(int n, int64_t nnz, const std::vector<int32_t> &rp,
                             const std::vector<int32_t> &ci) {
  if (rp[0] != 0 || rp[n] != nnz) return MCG_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return MCG_EINVAL;
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
      if (ci[p] < 0 || ci[p] >= n) return MCG_EINVAL;
      if (p > rp[i] && ci[p] <= ci[p - 1]) return MCG_EINVAL;
    }
  }
  return MCG_OK;
}

static void free_solver(mcg_solver *h) {
  if (!h) return;
  void *bufs[] = {h->rp, h->ci, h->va, h->va32, h->V, h->V32, h->r1, h->r2, h->y, h->v, h->w,
                  h->w1, h->w2, h->rt, h->xbest, h->z, h->r, h->p, h->q, h->t, h->S, h->Saux,
                  h->part, h->part2, h->ticket, h->hist, h->badcount, h->b_rp, h->b_ci, h->b_v,
                  h->b_v32};
  for (void *b : bufs) dev_free(b);
  mcg_sell_free(&h->sa);
  mcg_bsell_free(&h->bsa);
  if (h->poll) (void)hipHostFree(h->poll);
  if (h->hstate) (void)hipHostFree(h->hstate);
  for (int i = 0; i < 2; ++i)
    if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
  for (hipEvent_t e : h->prof_ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
}

extern "C" void minres_cg_free(mcg_handle_t h) { free_solver(h); }

// Block CSR copy of A for opt.block_size = bs in 2..4: kept only if every
// nonzero block is dense (each row of a block row has the same block
// columns, each with its bs consecutive entries); otherwise CSR alone is used.
static int build_bsr(mcg_solver *h, hipStream_t s) {
  const int bs = h->opt.block_size, n = h->n;
  if (bs < 2 || bs > 4 || n % bs != 0 || h->nnz == 0 || h->opt.spmv_format != 0) return MCG_OK;
  const int N = n / bs;
  const std::vector<int32_t> &rp = h->h_rp, &ci = h->h_ci;
  std::vector<int32_t> brp(N + 1, 0), bci;
  bci.reserve((size_t)(h->nnz / (bs * bs)) + 1);
  for (int I = 0; I < N; ++I) {
    const int r0 = I * bs;
    const int len = rp[r0 + 1] - rp[r0];
    if (len % bs) return MCG_OK;
    for (int a = 1; a < bs; ++a)
      if (rp[r0 + a + 1] - rp[r0 + a] != len) return MCG_OK;
    for (int t = 0; t < len; t += bs) {
      const int c0 = ci[rp[r0] + t];
      if (c0 % bs) return MCG_OK;
      for (int a = 0; a < bs; ++a)
        for (int b = 0; b < bs; ++b)
          if (ci[rp[r0 + a] + t + b] != c0 + b) return MCG_OK;
      bci.push_back(c0 / bs);
    }
    brp[I + 1] = (int32_t)bci.size();
  }
  const int64_t nb = (int64_t)bci.size();
  std::vector<double> v(h->nnz), bv((size_t)nb * bs * bs);
  HIP_TRY(hipMemcpy(v.data(), h->va, sizeof(double) * h->nnz, hipMemcpyDeviceToHost));
  for (int I = 0; I < N; ++I)
    for (int a = 0; a < bs; ++a) {
      const int r = I * bs + a;
      for (int t = 0; t < rp[r + 1] - rp[r]; ++t) {
        const int64_t blk = brp[I] + t / bs;
        bv[((size_t)blk * bs + a) * bs + (t % bs)] = v[rp[r] + t];
      }
    }
  int rc;
  if ((rc = dev_alloc(&h->b_rp, N + 1)) || (rc = dev_alloc(&h->b_ci, nb)) ||
      (rc = dev_alloc(&h->b_v, (size_t)nb * bs * bs)))
    return rc;
  HIP_TRY(hipMemcpy(h->b_rp, brp.data(), sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->b_ci, bci.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->b_v, bv.data(), sizeof(double) * bv.size(), hipMemcpyHostToDevice));
  if (h->opt.precision == MCG_PREC_MIXED) {
    if ((rc = dev_alloc(&h->b_v32, (size_t)nb * bs * bs))) return rc;
    k_convert<float, double><<<2048, 256, 0, s>>>((int64_t)bv.size(), h->b_v, h->b_v32);
    HIP_TRY(hipStreamSynchronize(s));
  }
  // sliced copy of the blocks for the inner products (padding <= 25 %)
  if ((rc = mcg_bsell_build(&h->bsa, bs, N, brp, bci, bv, 0.25,
                            h->opt.precision == MCG_PREC_MIXED, s, false, h->opt.xcd_order)))
    return rc;
  h->bsr_bs = bs;
  h->nbr = N;
  h->nnzb = nb;
  return MCG_OK;
}

// Sliced ELL copy (layout at k_sell_spmv).  Automatic (spmv_format 0): only
// without a block copy, without an explicit lanes-per-row request, and when
// padding adds at most 25 % to nnz; 16-bit column offsets when every offset
// fits.  spmv_format 2: always, 32-bit columns.
static int build_sell(mcg_solver *h, hipStream_t s) {
  const int fmt = h->opt.spmv_format;
  if (h->bsr_bs || h->nnz == 0 || h->n == 0 || fmt == 1) return MCG_OK;
  if (fmt == 0 && h->opt.spmv_lanes > 0) return MCG_OK;
  std::vector<double> v(h->nnz);
  HIP_TRY(hipMemcpy(v.data(), h->va, sizeof(double) * h->nnz, hipMemcpyDeviceToHost));
  return mcg_sell_build(&h->sa, h->n, h->h_rp, h->h_ci, v.data(), fmt == 0, fmt == 0 ? 0.25 : -1.0,
                        h->opt.precision == MCG_PREC_MIXED, s);
}

static int create_impl(mcg_solver *h, const mcg_csr_t *A, int32_t k, const double *Vhat,
                       const double *lam, hipStream_t s) {
  const int n = A->n;
  const int64_t nnz = A->nnz;
  // structure check on the host (setup only)
  h->h_rp.resize(n + 1);
  h->h_ci.resize(nnz);
  HIP_TRY(hipMemcpy(h->h_rp.data(), A->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
  if (nnz) HIP_TRY(hipMemcpy(h->h_ci.data(), A->col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  if (validate_csr_host(n, nnz, h->h_rp, h->h_ci) != MCG_OK) return MCG_EINVAL;
  std::vector<double> hlam(k);
  if (k) HIP_TRY(hipMemcpy(hlam.data(), lam, sizeof(double) * k, hipMemcpyDeviceToHost));
  for (int j = 0; j < k; ++j)
    if (!(hlam[j] < 0.0) || !std::isfinite(hlam[j])) return MCG_EINVAL;

  int rc;
  if ((rc = dev_alloc(&h->rp, n + 1)) || (rc = dev_alloc(&h->ci, nnz)) ||
      (rc = dev_alloc(&h->va, nnz)) || (rc = dev_alloc(&h->badcount, 4)))
    return rc;
  HIP_TRY(hipMemcpyAsync(h->rp, A->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->ci, A->col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->va, A->val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
  const size_t nk = (size_t)n * k;
  const size_t nkb = (size_t)((n + MCG_VBLK - 1) / MCG_VBLK) * MCG_VBLK * k;  // blocked layout
  if ((rc = dev_alloc(&h->V, nkb))) return rc;
  if (k) k_vhat_to_blocked<double><<<2048, 256, 0, s>>>(n, k, Vhat, h->V);
  // non-finite values in A or Vhat
  HIP_TRY(hipMemsetAsync(h->badcount, 0, 4 * sizeof(unsigned), s));
  k_count_nonfinite<<<1024, 256, 0, s>>>(nnz, h->va, h->badcount);
  if (k) k_count_nonfinite<<<1024, 256, 0, s>>>((int64_t)nk, Vhat, h->badcount);
  unsigned bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, h->badcount, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (bad) return MCG_EINVAL;

  const bool mixed = h->opt.precision == MCG_PREC_MIXED;
  if (mixed) {
    if ((rc = dev_alloc(&h->va32, nnz)) || (rc = dev_alloc(&h->V32, nkb))) return rc;
    k_convert<float, double><<<2048, 256, 0, s>>>(nnz, h->va, h->va32);
    if (k) k_vhat_to_blocked<float><<<2048, 256, 0, s>>>(n, k, Vhat, h->V32);
  }
  // workspace: outer FP64 vectors, inner vectors in the inner precision
  double **outer[] = {&h->r1, &h->r2, &h->y, &h->v, &h->w, &h->w1, &h->w2, &h->rt, &h->xbest};
  for (double **b : outer)
    if ((rc = dev_alloc(b, n))) return rc;
  const size_t es = mixed ? sizeof(float) : sizeof(double);
  void **inner[] = {&h->z, &h->r, &h->p, &h->q, &h->t};
  for (void **b : inner) {
    HIP_TRY(hipMalloc(b, std::max<size_t>(1, (size_t)n) * es));
  }
  h->grid_tile_max = 2048;
  h->grid_stream_max = 1024;
  const int gmax = std::max(h->grid_tile_max, h->grid_stream_max);
  if ((rc = dev_alloc(&h->part, (size_t)gmax * (MCG_KMAX + 4))) ||
      (rc = dev_alloc(&h->part2, (size_t)h->grid_tile_max * 6)) ||
      (rc = dev_alloc(&h->ticket, 16)) ||
      (rc = dev_alloc(&h->S, 1)) || (rc = dev_alloc(&h->Saux, 1)))
    return rc;
  HIP_TRY(hipMemsetAsync(h->ticket, 0, 16 * sizeof(unsigned), s));
  DevState init;
  std::memset(&init, 0, sizeof(init));
  for (int j = 0; j < k; ++j) {
    init.c[j] = 2.0 * std::fabs(hlam[j]);
    init.smw[j] = -2.0 / hlam[j];
  }
  init.scale = init.inv_scale = 1.0;
  HIP_TRY(hipMemcpyAsync(h->S, &init, sizeof(DevState), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->Saux, &init, sizeof(DevState), hipMemcpyHostToDevice, s));
  HIP_TRY(hipHostMalloc((void **)&h->poll, 2 * sizeof(DevPoll), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void **)&h->hstate, sizeof(DevState), hipHostMallocDefault));
  for (int i = 0; i < 2; ++i) HIP_TRY(hipEventCreateWithFlags(&h->ev[i], hipEventDisableTiming));
  if (h->opt.profile)
    for (hipEvent_t &e : h->prof_ev) HIP_TRY(hipEventCreate(&e));
  h->hist_cap = 0;
  h->lanes = h->opt.spmv_lanes > 0 ? h->opt.spmv_lanes : lanes_heuristic(nnz, n);
  h->mmr_split = h->opt.mmr_form == 2 ? 1 : 0;
  HIP_TRY(hipStreamSynchronize(s));
  if ((rc = build_bsr(h, s))) return rc;
  // the block copy serves the split M_mr apply (unless the fused CSR form was asked for)
  if (h->bsr_bs && h->opt.mmr_form != 1) h->mmr_split = 1;
  if ((rc = build_sell(h, s))) return rc;
  // with a sliced copy: split form unless the one-pass kernel was asked for
  // (the autotuner below times both)
  if (h->sa.bits && h->opt.mmr_form != 1) h->mmr_split = 1;
  if (h->opt.autotune) {
    rc = mcg_autotune_lanes(h, s);
    if (rc) return rc;
  }
  return MCG_OK;
}

extern "C" int minres_cg_create(mcg_handle_t *out, const mcg_csr_t *A, int32_t k,
                                const double *Vhat, const double *lam,
                                const mcg_options_t *opt, void *stream) {
  if (!out || !A) return MCG_EINVAL;
  *out = nullptr;
  if (A->n <= 0 || A->nnz < 0 || A->nnz >= ((int64_t)1 << 31) || !A->row_ptr ||
      (A->nnz > 0 && (!A->col || !A->val)))
    return MCG_EINVAL;
  if (k < 0 || k > MCG_KMAX || (k > 0 && (!Vhat || !lam))) return MCG_EINVAL;
  if ((int64_t)A->n * k >= ((int64_t)1 << 31)) return MCG_EINVAL;
  mcg_solver *h = new (std::nothrow) mcg_solver();
  if (!h) return MCG_ENOMEM;
  if (opt) h->opt = *opt; else minres_cg_default_options(&h->opt);
  if (h->opt.precision != MCG_PREC_FP64 && h->opt.precision != MCG_PREC_MIXED) { delete h; return MCG_EINVAL; }
  if (h->opt.spmv_lanes < 0 || h->opt.spmv_lanes > 64 ||
      (h->opt.spmv_lanes & (h->opt.spmv_lanes - 1))) { delete h; return MCG_EINVAL; }
  if (h->opt.block_size <= 0) h->opt.block_size = 1;
  if (h->opt.mmr_form < 0 || h->opt.mmr_form > 2) { delete h; return MCG_EINVAL; }
  if (h->opt.xcd_order < 0 || h->opt.xcd_order > 2) { delete h; return MCG_EINVAL; }
  h->n = A->n;
  h->nnz = A->nnz;
  h->k = k;
  h->kb = mcg_kb_bucket(k);
  int rc = create_impl(h, A, k, Vhat, lam, (hipStream_t)stream);
  if (rc != MCG_OK) {
    free_solver(h);
    return rc;
  }
  *out = h;
  return MCG_OK;
}

// ---------------------------------------------------------------------------
// preconditioner handles
// ---------------------------------------------------------------------------
static void free_pc(mcg_pc *p) {
  if (!p) return;
  for (hipGraphExec_t &g : p->graph32)
    if (g) (void)hipGraphExecDestroy(g);
  mcg_pc_release_extra(p);
  dev_free(p->dinv64);
  dev_free(p->dinv32);
  delete p;
}

extern "C" void minres_cg_precond_free(mcg_precond_t p) { free_pc(p); }

extern "C" int minres_cg_precond_create(mcg_precond_t *out, mcg_handle_t h, int32_t kind,
                                        const void *params, void *stream) {
  if (!out || !h) return MCG_EINVAL;
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  const int base = kind & 0xff;
  const bool smw = (kind & MCG_PC_SMW) != 0;
  if ((kind & ~(0xff | MCG_PC_SMW)) != 0) return MCG_EINVAL;
  if (base != MCG_PC_NONE && base != MCG_PC_JACOBI && base != MCG_PC_ILDL0 &&
      base != MCG_PC_ILDLP && base != MCG_PC_CCT)
    return MCG_EINVAL;
  mcg_pc *p = new (std::nothrow) mcg_pc();
  if (!p) return MCG_ENOMEM;
  p->h = h;
  p->base = base;
  p->smw = smw;
  p->diag_path = (base == MCG_PC_NONE || base == MCG_PC_JACOBI) && !smw;
  int rc = MCG_OK;
  if (base == MCG_PC_NONE || base == MCG_PC_JACOBI) {
    if ((rc = dev_alloc(&p->dinv64, h->n))) { free_pc(p); return rc; }
    if (hipMemsetAsync(h->badcount, 0, sizeof(unsigned), s) != hipSuccess) { free_pc(p); return MCG_EHIP; }
    k_jacobi_setup<double><<<1024, 256, 0, s>>>(h->n, h->rp, h->ci, h->va, p->dinv64,
                                                 base == MCG_PC_NONE, h->badcount);
    if (h->opt.precision == MCG_PREC_MIXED) {
      if ((rc = dev_alloc(&p->dinv32, h->n))) { free_pc(p); return rc; }
      k_convert<float, double><<<1024, 256, 0, s>>>(h->n, p->dinv64, p->dinv32);
    }
    unsigned bad = 0;
    if (hipMemcpyAsync(&bad, h->badcount, sizeof(unsigned), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { free_pc(p); return MCG_EHIP; }
    if (bad) { free_pc(p); return MCG_EINVAL; }
  } else if (base == MCG_PC_ILDL0) {
    const double pivtol = params ? *(const double *)params : 1e-8;
    rc = mcg_ildl0_create(p, pivtol, s);
  } else if (base == MCG_PC_ILDLP) {
    mcg_ildlp_params_t prm{3.0, 1e-3, 0};
    if (params) prm = *(const mcg_ildlp_params_t *)params;
    rc = mcg_ildlp_create(p, prm.fill, prm.drop, prm.sweeps, s);
  } else {
    rc = mcg_cct_create(p, (const mcg_csr_t *)params, s);
  }
  if (rc != MCG_OK) { free_pc(p); return rc; }
  *out = p;
  return MCG_OK;
}

// ---------------------------------------------------------------------------
// the solve
// ---------------------------------------------------------------------------
static int read_state(mcg_solver *h, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(h->hstate, h->S, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MCG_OK;
}

// Optional record of the inner solves (minres_cg_solve_record): column i of Y
// gets the right-hand side of inner solve i, column i of Z its result.
struct InnerRecord {
  double *Y = nullptr, *Z = nullptr;
  int32_t cap = 0, count = 0;
};

static int record_inner(mcg_solver *h, InnerRecord *rec, const double *y_in, hipStream_t s) {
  if (!rec || rec->count >= rec->cap) return MCG_OK;
  const size_t off = (size_t)rec->count * h->n, bytes = sizeof(double) * (size_t)h->n;
  HIP_TRY(hipMemcpyAsync(rec->Y + off, y_in, bytes, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(rec->Z + off, h->y, bytes, hipMemcpyDeviceToDevice, s));
  rec->count += 1;
  return MCG_OK;
}

template <typename T>
static int solve_impl(mcg_solver *h, const mcg_pc *pc, const double *b, double *x,
                      double rtol_out, double rtol_in, int32_t maxit_out,
                      int64_t maxit_inner_total, mcg_stats_t *st, hipStream_t s,
                      InnerRecord *rec = nullptr) {
  const int n = h->n;
  const int gs = mcg_grid_stream(h), gt = mcg_grid_tile(h);
  const int scaled = sizeof(T) == 4;
  int rc;
  DevState *S = h->S;
  int64_t budget = maxit_inner_total;
  int64_t inner_total = 0;
  h->last_inner_its = 16 * 6;
  auto record = [&](int idx, double rel, double phib, int64_t its) {
    if (!st || !st->hist_cap || idx >= st->hist_cap) return;
    if (st->relres) st->relres[idx] = rel;
    if (st->phibar) st->phibar[idx] = phib;
    if (st->inner_its) st->inner_its[idx] = its;
  };
  // r1 = b - A x0
  MCG_SWITCH_L(h->lanes, (k_resid<L><<<gt, MCG_BLOCK, 0, s>>>(n, h->rp, h->ci, h->va, x, b, h->r1,
                                                             S, h->part, h->ticket)));
  // w, w1, w2 = 0: the first two direction updates scale w1 and w2 by zero,
  // which must not meet stale NaN bit patterns in the workspace
  for (double *wv : {h->w, h->w1, h->w2}) k_fill<double><<<gs, MCG_BLOCK, 0, s>>>(n, 0.0, wv);
  if ((rc = read_state(h, s))) return rc;
  const double bb = h->hstate->bb, r0 = h->hstate->rt2;
  if (!std::isfinite(bb) || !std::isfinite(r0)) return MCG_EINVAL;
  const double bnorm = std::sqrt(bb);
  double rnorm = std::sqrt(r0);
  double best = rnorm;
  if (st) { st->bnorm = bnorm; st->outer_its = 0; st->inner_its_total = 0; }
  if (bb == 0.0) {
    HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (st) { st->status = MCG_OK; st->final_relres = 0.0; }
    record(0, 0.0, 0.0, 0);
    return MCG_OK;
  }
  HIP_TRY(hipMemcpyAsync(h->xbest, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  record(0, rnorm / bnorm, rnorm, 0);
  if (rnorm <= rtol_out * bnorm) {
    HIP_TRY(hipStreamSynchronize(s));
    if (st) { st->status = MCG_OK; st->final_relres = rnorm / bnorm; }
    return MCG_OK;
  }
  // y = M^{-1} r1 (first inner solve), beta1 = sqrt(r1^T y)
  k_set_scale<<<gs, MCG_BLOCK, 0, s>>>(n, h->r1, S, h->part, h->ticket, scaled);
  DevPoll poll;
  if ((rc = run_inner<T, double>(h, pc, h->r1, rtol_in, std::min<int64_t>(n, budget), s, &poll))) return rc;
  budget -= poll.its;
  inner_total += poll.its;
  k_outer_post<T><<<gs, MCG_BLOCK, 0, s>>>(n, (const T *)h->z, h->y, h->r1, S, h->part, h->ticket,
                                           1, nullptr, 0);
  if (poll.its > 0 && (rc = record_inner(h, rec, h->r1, s))) return rc;
  if ((rc = read_state(h, s))) return rc;
  if (st && st->hist_cap > 0 && st->inner_its) st->inner_its[0] = poll.its;
  int status = MCG_MAXIT;
  if (poll.status == MCG_NOT_SPD || poll.status == MCG_BREAKDOWN) {
    status = poll.status;
  } else if (poll.status == MCG_MAXIT && budget <= 0) {
    status = MCG_MAXIT;
  } else if (h->hstate->outer_flag || !(h->hstate->beta2 > 0.0)) {
    status = MCG_BREAKDOWN;
  } else {
    if (st && st->hist_cap > 0 && st->phibar) st->phibar[0] = h->hstate->beta_cur;
    HIP_TRY(hipMemcpyAsync(h->r2, h->r1, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    int since_best = 0;
    status = MCG_MAXIT;
    for (int itn = 1; itn <= maxit_out; ++itn) {
      MCG_SWITCH_L(h->lanes, (k_lanczos_a<L><<<gt, MCG_BLOCK, 0, s>>>(
                                 n, h->rp, h->ci, h->va, h->y, h->v, h->r1, S, h->part,
                                 h->ticket, itn == 1)));
      k_lanczos_b<<<gs, MCG_BLOCK, 0, s>>>(n, h->r1, h->r2, S, h->part, h->ticket, scaled);
      std::swap(h->r1, h->r2);  // r1 <- old r2, r2 <- new Lanczos vector
      const int64_t cap = std::min<int64_t>(n, budget);
      if ((rc = run_inner<T, double>(h, pc, h->r2, rtol_in, cap, s, &poll))) return rc;
      budget -= poll.its;
      inner_total += poll.its;
      k_outer_post<T><<<gs, MCG_BLOCK, 0, s>>>(n, (const T *)h->z, h->y, h->r2, S, h->part,
                                               h->ticket, 0, nullptr, 0);
      if (poll.its > 0 && (rc = record_inner(h, rec, h->r2, s))) return rc;
      double *tmp = h->w1;
      h->w1 = h->w2;
      h->w2 = h->w;
      h->w = tmp;
      k_outer_update<<<gs, MCG_BLOCK, 0, s>>>(n, h->w, h->w1, h->w2, h->v, x, S);
      MCG_SWITCH_L(h->lanes, (k_resid<L><<<gt, MCG_BLOCK, 0, s>>>(n, h->rp, h->ci, h->va, x, b,
                                                                 h->rt, S, h->part, h->ticket)));
      if ((rc = read_state(h, s))) return rc;
      const DevState &hs = *h->hstate;
      if (st) st->outer_its = itn;
      if (poll.status == MCG_NOT_SPD || poll.status == MCG_BREAKDOWN) { status = poll.status; break; }
      if (hs.outer_flag) { status = MCG_BREAKDOWN; break; }
      rnorm = std::sqrt(hs.rt2);
      record(itn, rnorm / bnorm, hs.phibar, poll.its);
      if (!std::isfinite(rnorm)) { status = MCG_BREAKDOWN; break; }
      if (rnorm < best) {
        since_best = (rnorm < best * (1.0 - 1e-3)) ? 0 : since_best + 1;
        best = rnorm;
        HIP_TRY(hipMemcpyAsync(h->xbest, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      } else {
        ++since_best;
      }
      if (rnorm <= rtol_out * bnorm) { status = MCG_OK; break; }
      if ((poll.status == MCG_MAXIT && budget <= 0) || budget <= 0) { status = MCG_MAXIT; break; }
      if (h->opt.stag_window > 0 && since_best >= h->opt.stag_window) { status = MCG_STAGNATION; break; }
      if (hs.beta_cur == 0.0) { status = MCG_BREAKDOWN; break; }
    }
  }
  double final_rel = rnorm / bnorm;
  if (status != MCG_OK && h->opt.keep_best) {
    HIP_TRY(hipMemcpyAsync(x, h->xbest, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    final_rel = best / bnorm;
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (st) {
    st->status = status;
    st->inner_its_total = inner_total;
    st->final_relres = final_rel;
  }
  return status;
}

extern "C" int minres_cg_solve(mcg_handle_t h, mcg_precond_t p, const double *b, double *x,
                               int32_t nrhs, double rtol_out, double rtol_in, int32_t maxit_out,
                               int64_t maxit_inner_total, mcg_stats_t *stats, void *stream) {
  if (!h || !p || !b || !x || p->h != h) return MCG_EINVAL;
  if (nrhs < 1) return MCG_EINVAL;
  if (!(rtol_out >= 0.0) || !(rtol_in >= 0.0) || maxit_out < 0 || maxit_inner_total < 0)
    return MCG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  // the right-hand sides one after the other, on the same handle and graphs
  int worst = MCG_OK;
  for (int32_t j = 0; j < nrhs; ++j) {
    const size_t off = (size_t)j * h->n;
    mcg_stats_t *st = stats ? stats + j : nullptr;
    const int rc =
        h->opt.precision == MCG_PREC_MIXED
            ? solve_impl<float>(h, p, b + off, x + off, rtol_out, rtol_in, maxit_out,
                                maxit_inner_total, st, s)
            : solve_impl<double>(h, p, b + off, x + off, rtol_out, rtol_in, maxit_out,
                                 maxit_inner_total, st, s);
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
  }
  return worst;
}

extern "C" int minres_cg_solve_record(mcg_handle_t h, mcg_precond_t p, const double *b, double *x,
                                      double rtol_out, double rtol_in, int32_t maxit_out,
                                      int64_t maxit_inner_total, double *Y, double *Z,
                                      int32_t cap, int32_t *count, mcg_stats_t *stats,
                                      void *stream) {
  if (!h || !p || !b || !x || p->h != h || cap < 0 || (cap > 0 && (!Y || !Z))) return MCG_EINVAL;
  if (!(rtol_out >= 0.0) || !(rtol_in >= 0.0) || maxit_out < 0 || maxit_inner_total < 0)
    return MCG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  InnerRecord rec;
  rec.Y = Y;
  rec.Z = Z;
  rec.cap = cap;
  const int rc = h->opt.precision == MCG_PREC_MIXED
                     ? solve_impl<float>(h, p, b, x, rtol_out, rtol_in, maxit_out,
                                         maxit_inner_total, stats, s, &rec)
                     : solve_impl<double>(h, p, b, x, rtol_out, rtol_in, maxit_out,
                                          maxit_inner_total, stats, s, &rec);
  if (count) *count = rec.count;
  return rc;
}

// ---------------------------------------------------------------------------
// steps exposed one by one
// ---------------------------------------------------------------------------
extern "C" int mcg_spmv(mcg_handle_t h, int32_t precision, const void *x, void *y, void *stream) {
  if (!h || !x || !y) return MCG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (precision == MCG_PREC_FP64) {
    mcg_launch_spmv<double>(h, (const double *)x, (double *)y, s);
  } else if (precision == MCG_PREC_MIXED && h->va32) {
    mcg_launch_spmv<float>(h, (const float *)x, (float *)y, s);
  } else {
    return MCG_EINVAL;
  }
  HIP_TRY(hipGetLastError());
  return MCG_OK;
}

template <typename T>
static int mmr_apply_impl(mcg_solver *h, const T *u, T *q, hipStream_t s) {
  launch_vtu<T>(h, u, h->Saux, s);
  launch_mmr<T>(h, u, q, h->Saux, 0, s);
  HIP_TRY(hipGetLastError());
  return MCG_OK;
}

extern "C" int mcg_mmr_apply(mcg_handle_t h, int32_t precision, const void *u, void *q,
                             void *stream) {
  if (!h || !u || !q) return MCG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (precision == MCG_PREC_FP64) return mmr_apply_impl<double>(h, (const double *)u, (double *)q, s);
  if (precision == MCG_PREC_MIXED && h->va32) return mmr_apply_impl<float>(h, (const float *)u, (float *)q, s);
  return MCG_EINVAL;
}

extern "C" int mcg_precond_apply(mcg_precond_t p, int32_t precision, const void *g, void *t,
                                 void *stream) {
  if (!p || !g || !t) return MCG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (precision == MCG_PREC_FP64) {
    if (p->base == MCG_PC_ILDL0 && !p->has64) return MCG_EINVAL;
    launch_pc_apply<double>(p, (const double *)g, (double *)t, p->h->Saux, 0, s);
  } else if (precision == MCG_PREC_MIXED && p->h->va32) {
    launch_pc_apply<float>(p, (const float *)g, (float *)t, p->h->Saux, 0, s);
  } else {
    return MCG_EINVAL;
  }
  HIP_TRY(hipGetLastError());
  return MCG_OK;
}

template <typename T>
__global__ void k_scale_back(int n, const T *__restrict__ z, const DevState *__restrict__ S,
                             double *__restrict__ out) {
  const double sc = S->scale;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = sc * (double)z[i];
}

template <typename T>
static int pcg_impl(mcg_solver *h, const mcg_pc *p, const double *y, double *z, double rtol,
                    int64_t maxit, int64_t *its, hipStream_t s) {
  const int gs = mcg_grid_stream(h);
  k_set_scale<<<gs, MCG_BLOCK, 0, s>>>(h->n, y, h->S, h->part, h->ticket, sizeof(T) == 4);
  DevPoll poll;
  h->last_inner_its = 16 * 6;
  int rc = run_inner<T, double>(h, p, y, rtol, maxit, s, &poll);
  if (rc) return rc;
  k_scale_back<T><<<gs, MCG_BLOCK, 0, s>>>(h->n, (const T *)h->z, h->S, z);
  HIP_TRY(hipStreamSynchronize(s));
  if (its) *its = poll.its;
  return poll.status;
}

extern "C" int mcg_pcg_solve(mcg_handle_t h, mcg_precond_t p, const double *y, double *z,
                             double rtol_in, int64_t maxit, int64_t *its, void *stream) {
  if (!h || !p || !y || !z || p->h != h || !(rtol_in >= 0.0) || maxit < 0) return MCG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (h->opt.precision == MCG_PREC_MIXED) return pcg_impl<float>(h, p, y, z, rtol_in, maxit, its, s);
  return pcg_impl<double>(h, p, y, z, rtol_in, maxit, its, s);
}

extern "C" int minres_cg_kernel_time(mcg_handle_t h, double *ms, int64_t *launches,
                                     int32_t reset) {
  if (!h || !h->opt.profile) return MCG_EINVAL;
  if (ms) *ms = h->prof_ms;
  if (launches) *launches = h->prof_launches;
  if (reset) {
    h->prof_ms = 0.0;
    h->prof_launches = 0;
  }
  return MCG_OK;
}

// ---------------------------------------------------------------------------
// host-only queries
// ---------------------------------------------------------------------------
extern "C" int minres_cg_workspace_vectors(int32_t k, int32_t precision, int32_t pc_kind,
                                           int32_t *paper, int32_t *total) {
  if (k < 0 || k > MCG_KMAX) return MCG_EINVAL;
  // paper (storage table): MINRES 7 + CG 4 + Vhat k
  if (paper) *paper = 11 + k;
  // this implementation: r1 r2 y v w w1 w2 (7) + rt xbest (2) + z r p q t (5)
  // + Vhat (k); mixed adds the FP32 Vhat shadow (k) and a Jacobi FP32 diagonal
  int t = 7 + 2 + 5 + k;
  const int base = pc_kind & 0xff;
  if (base == MCG_PC_NONE || base == MCG_PC_JACOBI) t += 1;  // inverse diagonal
  if (precision == MCG_PREC_MIXED) t += k + ((base == MCG_PC_NONE || base == MCG_PC_JACOBI) ? 1 : 0);
  if (total) *total = t;
  return MCG_OK;
}

extern "C" const char *minres_cg_strerror(int code) {
  switch (code) {
    case MCG_OK: return "converged";
    case MCG_MAXIT: return "iteration cap reached";
    case MCG_STAGNATION: return "true residual stagnated";
    case MCG_BREAKDOWN: return "breakdown: a recurrence scalar vanished or became invalid";
    case MCG_NOT_SPD: return "M_mr not positive definite (deflation subspace incomplete)";
    case MCG_EINVAL: return "invalid argument";
    case MCG_EHIP: return "HIP runtime error";
    case MCG_ENOMEM: return "out of memory";
    default: return "unknown status";
  }
}

extern "C" const char *minres_cg_version(void) { return "minres_cg 1.0 gfx950"; }

// explicit instantiations used by other translation units
template void mcg_launch_spmv<double>(const mcg_solver *, const double *, double *, hipStream_t);
template void mcg_launch_spmv<float>(const mcg_solver *, const float *, float *, hipStream_t);
template void mcg_launch_spmv_csr<double>(const mcg_solver *, const double *, double *,
                                          hipStream_t);
template void mcg_launch_spmv_csr<float>(const mcg_solver *, const float *, float *, hipStream_t);
