// Internal structures shared by the translation units of libminrescg.so.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <vector>

#include "../../include/minres_cg.h"
#include "mcg_kernels.h"

// The part of DevState the host polls between chunks of inner iterations.
struct DevPoll {
  int32_t done;
  int32_t status;
  int64_t its;
  int64_t maxit;
  int32_t outer_flag;
  int32_t pad0;
};
static_assert(sizeof(DevPoll) <= sizeof(DevState), "poll prefix");

// Sliced ELL copy of an n x n sparse matrix (layout at k_sell_spmv): bits =
// column width (16: int16 offsets from the row, 32: absolute int32), 0 when
// there is no copy.  FP64 values, and FP32 ones for mixed precision.
struct mcg_sell {
  int bits = 0;
  int n = 0, nslices = 0;
  int maxw = 0;  // widest slice (slots)
  int64_t *off = nullptr;
  void *col = nullptr;
  double *v = nullptr;
  float *v32 = nullptr;
  _Float16 *v16 = nullptr;  // FP16 values for the FP32 products, when requested and in range
};
// Builds the copy from a host CSR (sorted columns, host values).  No copy
// (bits = 0, MCG_OK) when padding would add more than max_pad * nnz entries
// (max_pad < 0: any padding); 16-bit columns when narrow_ok and every offset
// fits.  fp16: also FP16 values, used by the FP32 products instead of the
// FP32 ones, when no value overflows FP16 and every diagonal value is a
// normal FP16 number (for a lower triangular factor with a positive
// diagonal, the rounded factor keeps it).
int mcg_sell_build(mcg_sell *S, int n, const std::vector<int32_t> &rp,
                   const std::vector<int32_t> &ci, const double *v, bool narrow_ok,
                   double max_pad, bool fp32, hipStream_t s, bool fp16 = false);
void mcg_sell_free(mcg_sell *S);
template <typename T>
inline const T *mcg_sell_vals(const mcg_sell &S) {
  if constexpr (sizeof(T) == 8)
    return S.v;
  else
    return S.v32;
}
// y = A x (St != nullptr: return at once after the inner stop)
template <typename T>
void mcg_sell_spmv(const mcg_sell &A, const T *x, T *y, const DevState *St, hipStream_t s);

// Sliced block ELL copy of a matrix of dense bs x bs blocks (layout at
// k_bsell_spmv); bs = 0 when there is no copy.
struct mcg_bsell {
  int bs = 0;
  int nbr = 0, nslices = 0;
  int64_t *off = nullptr;
  int32_t *col = nullptr;
  double *v = nullptr;
  float *v32 = nullptr;
  _Float16 *v16 = nullptr;  // as mcg_sell::v16
  // XCD-aware slice order (k_bsell_spmv): xmap[e], xmap[e + 1] bound the
  // slices of XCD e (e < 8), listed from xmap[9]; nullptr: the launch's own
  // round-robin order.  xmap_sections: the chosen candidate (-1 none).
  int32_t *xmap = nullptr;
  int xmap_sections = -1;
};
// From a host block CSR (brp, bci; values block-major, row-major inside a
// block).  No copy (bs = 0, MCG_OK) when padding would add more than
// max_pad * (number of blocks).
int mcg_bsell_build(mcg_bsell *S, int bs, int nbr, const std::vector<int32_t> &brp,
                    const std::vector<int32_t> &bci, const std::vector<double> &bv,
                    double max_pad, bool fp32, hipStream_t s, bool fp16 = false,
                    int xcd_order = 0);
void mcg_bsell_free(mcg_bsell *S);
// y = A x; DOT: partials of r^T y, y^T y into part (rows of 2) and r^T y into
// compact; part_in != nullptr: also finish the Vhat^T p reduction (see the
// kernel).  Returns the grid size.
template <typename T>
inline const T *mcg_bsell_vals(const mcg_bsell &S) {
  if constexpr (sizeof(T) == 8)
    return S.v;
  else
    return S.v32;
}
template <typename T>
int mcg_bsell_spmv(const mcg_bsell &A, const T *x, T *y, DevState *St, hipStream_t s,
                   bool dot = false, const T *r = nullptr, double *part = nullptr,
                   double *compact = nullptr, const double *part_in = nullptr, int nb_in = 0,
                   int k = 0, int max_grid = 2048);

struct mcg_solver {
  int n = 0;
  int64_t nnz = 0;
  int k = 0, kb = 0, lanes = 8;
  int mmr_split = 0;  // 1: M_mr apply of the Jacobi iteration as SpMV + streaming rank-k pass
  // block CSR copy of A (opt.block_size > 1 and every block dense), used by
  // the inner SpMVs; 0 = none
  int bsr_bs = 0;
  int nbr = 0;
  int64_t nnzb = 0;
  int32_t *b_rp = nullptr, *b_ci = nullptr;
  double *b_v = nullptr;
  float *b_v32 = nullptr;
  mcg_bsell bsa;  // sliced copy of the block CSR copy (preferred when present)
  // sliced ELL copy of A (slices of 64 rows, slot-major; see k_sell_spmv)
  mcg_sell sa;
  mcg_options_t opt{};
  // A (owned copies)
  int32_t *rp = nullptr, *ci = nullptr;
  double *va = nullptr;
  float *va32 = nullptr;
  // deflation data
  double *V = nullptr;
  float *V32 = nullptr;
  // outer FP64 workspace
  double *r1 = nullptr, *r2 = nullptr, *y = nullptr, *v = nullptr, *w = nullptr, *w1 = nullptr,
         *w2 = nullptr, *rt = nullptr, *xbest = nullptr;
  // inner workspace (element type = inner precision)
  void *z = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *t = nullptr;
  // device scalars and reduction scratch
  DevState *S = nullptr, *Saux = nullptr;
  double *part = nullptr;
  double *part2 = nullptr;  // second partials buffer (the Jacobi update's r^T r, r^T t, t^T t)
  unsigned *ticket = nullptr;
  int64_t *hist = nullptr;
  unsigned *badcount = nullptr;
  // host mirrors
  DevPoll *poll = nullptr;     // pinned, 2 slots
  DevState *hstate = nullptr;  // pinned
  hipEvent_t ev[2] = {nullptr, nullptr};
  int grid_tile_max = 2048, grid_stream_max = 1024;
  int hist_cap = 0;
  int64_t last_inner_its = 96;
  // opt-in timing of the M_mr-apply launches (events recorded per launch)
  static constexpr int kProfSlots = 256;      // event pairs per poll slot
  hipEvent_t prof_ev[4 * kProfSlots] = {};    // 2 slots x kProfSlots pairs x 2
  int prof_used[2] = {0, 0};         // event pairs used by the chunk in each poll slot
  int64_t prof_first_iter[2] = {0, 0};  // inner iteration index of the first pair
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  // host copy of the pattern (setup only)
  std::vector<int32_t> h_rp, h_ci;
};

struct mcg_pc {
  mcg_solver *h = nullptr;
  int base = 0;
  bool smw = false;
  bool diag_path = false;
  bool has64 = true;
  double *dinv64 = nullptr;
  float *dinv32 = nullptr;
  void *ildl = nullptr;  // struct ildl_data (mcg_precond.hip)
  void *cct = nullptr;   // struct cct_data
  void *ildlp = nullptr; // struct ildlp_data
  int apply_launches = 0;  // kernel launches of one M_cg apply (ILDL sweeps)
  // 32 inner CG iterations of this (handle, preconditioner) pair captured as a
  // HIP graph on first use ([0] FP64, [1] FP32 inner precision)
  hipGraphExec_t graph32[2] = {nullptr, nullptr};
  bool graph_failed[2] = {false, false};
};

// last HIP error seen by any entry point (written from several host threads
// by the stream-parallel batched solve)
extern std::atomic<hipError_t> mcg_last_hip_error;

int mcg_kb_bucket(int k);
int mcg_grid_tile(const mcg_solver *h);
int mcg_grid_stream(const mcg_solver *h);

template <typename T>
void mcg_launch_spmv(const mcg_solver *h, const T *x, T *y, hipStream_t s);
// the CSR kernels only (lanes per row = h->lanes), also when a block copy exists
template <typename T>
void mcg_launch_spmv_csr(const mcg_solver *h, const T *x, T *y, hipStream_t s);

// second-level preconditioners other than the diagonal ones (mcg_precond.hip)
int mcg_ildl0_create(mcg_pc *p, double pivtol, hipStream_t s);
int mcg_cct_create(mcg_pc *p, const mcg_csr_t *C, hipStream_t s);
int mcg_ildlp_create(mcg_pc *p, double fill, double drop, int sweeps, hipStream_t s);
void mcg_pc_release_extra(mcg_pc *p);
// device arrays of C and C^T (values in the solver's inner precision) and a
// scratch vector, for the fused C C^T iteration
struct mcg_cct_view {
  int lanes;
  const int32_t *c_rp, *c_ci, *ct_rp, *ct_ci;
  const void *c_v, *ct_v;
  void *tmp;
  // block CSR copies of C and C^T (block size = the solver's bsr_bs), or bsr = 0
  int bsr, nbr;
  const int32_t *cb_rp, *cb_ci, *ctb_rp, *ctb_ci;
  const void *cb_v, *ctb_v;
  // sliced ELL copies of C and C^T (when A has one), or nullptr
  const mcg_sell *c_sell, *ct_sell;
  // sliced block copies of C and C^T (when A has one), or nullptr
  const mcg_bsell *c_bsell, *ct_bsell;
};
bool mcg_cct_view_get(const mcg_pc *p, bool fp32, mcg_cct_view *v);
template <typename T>
void mcg_csr_apply(int lanes, int n, const int32_t *rp, const int32_t *ci, const T *va, const T *x,
                   T *y, DevState *S, int check_done, hipStream_t s);
template <typename T>
void mcg_ildl0_apply(const mcg_pc *p, const T *g, T *t, DevState *S, int check_done, hipStream_t s);
template <typename T>
void mcg_cct_apply(const mcg_pc *p, const T *g, T *t, DevState *S, int check_done, hipStream_t s);
template <typename T>
void mcg_ildlp_apply(const mcg_pc *p, const T *g, T *t, DevState *S, int check_done, hipStream_t s);

// SpMV lanes-per-row autotuner (mcg_tune.hip)
int mcg_autotune_lanes(mcg_solver *h, hipStream_t s);

// the iteration's M_mr apply for a diagonal M_cg (fused or split form),
// partials for FIN_MMR; defined in mcg_api.hip
template <typename T>
int mcg_launch_mmr_diag(const mcg_solver *h, const T *p, T *q, const T *dinv, DevState *S,
                         hipStream_t s, double *pi_compact = nullptr);
