// The M_mr apply without a handle and without any allocation, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
//   q = A u + 2 Vhat (|lam| o (Vhat^T u))      (Section 2: the product every
//                                              inner CG iteration applies)
//
// The only device memory beyond the caller's inputs and outputs is the
// file-scope array `scratch` below: per-block partials of Vhat^T u and the k
// coefficients 2 |lam_j| (Vhat^T u)_j.  Every call overwrites what it reads,
// so nothing has to be cleared between calls.  Each GPU holds its own copy
// of the array for the life of the process; host code reaches it only
// through the per-device address from hipGetSymbolAddress (the array's name
// is a host-side stand-in there, not a device address).  Calls that overlap
// on one GPU (several streams or threads) share the array and race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "mcg_internal.h"

namespace {

constexpr int kMaxBlocks = 1024;  // blocks of the Vhat^T u pass (grid-stride)
constexpr int kMaxDevices = 64;
// partials [kMaxBlocks x MCG_KMAX], then the MCG_KMAX coefficients
constexpr size_t kScratchDoubles = (size_t)kMaxBlocks * MCG_KMAX + MCG_KMAX;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mutex;
double *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_ptr(double **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MCG_EHIP;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      mcg_last_hip_error = e;
      return MCG_EHIP;
    }
    g_scratch[dev] = (double *)p;
  }
  *out = g_scratch[dev];
  return MCG_OK;
}

// Per-block partials of Vhat^T u (Vhat n x k column-major): part[b k + j].
template <int KB>
__global__ __launch_bounds__(MCG_BLOCK) void k_na_vtu(int n, const double *__restrict__ u,
                                                      const double *__restrict__ V, int k,
                                                      double *__restrict__ part) {
  double acc[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) acc[j] = 0.0;
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    const double ui = u[i];
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (j < k) acc[j] += V[(size_t)j * n + i] * ui;
  }
  block_partials<KB>(acc, k, part);
}

// coef[j] = 2 |lam_j| sum_b part[b k + j], blocks summed in order (one block).
__global__ void k_na_coef(int nb, int k, const double *__restrict__ part,
                          const double *__restrict__ lam, double *__restrict__ coef) {
  const int j = threadIdx.x;
  if (j >= k) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * k + j];
  coef[j] = 2.0 * fabs(lam[j]) * s;
}

// q += Vhat coef
__global__ __launch_bounds__(MCG_BLOCK) void k_na_rankk(int n, const double *__restrict__ V,
                                                        int k, const double *__restrict__ coef,
                                                        double *__restrict__ q) {
  for (int i = blockIdx.x * MCG_BLOCK + threadIdx.x; i < n; i += gridDim.x * MCG_BLOCK) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += V[(size_t)j * n + i] * coef[j];
    q[i] += acc;
  }
}

template <int KB>
void launch_vtu(int nb, int n, const double *u, const double *V, int k, double *part,
                hipStream_t s) {
  k_na_vtu<KB><<<nb, MCG_BLOCK, 0, s>>>(n, u, V, k, part);
}

}  // namespace

extern "C" int mcg_mmr_apply_noalloc(const mcg_csr_t *A, int32_t k, const double *Vhat,
                                     const double *lam, const double *u, double *q,
                                     void *stream) {
  if (!A || !u || !q || A->n <= 0 || A->nnz < 0 || A->nnz >= ((int64_t)1 << 31) ||
      !A->row_ptr || (A->nnz > 0 && (!A->col || !A->val)))
    return MCG_EINVAL;
  if (k < 0 || k > MCG_KMAX || (k > 0 && (!Vhat || !lam))) return MCG_EINVAL;
  if ((int64_t)A->n * k >= ((int64_t)1 << 31)) return MCG_EINVAL;
  double *sc = nullptr;
  int rc = scratch_ptr(&sc);
  if (rc != MCG_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int n = A->n;
  // q = A u: the library's CSR kernel, lanes per row from the mean row length
  const double mean = (double)A->nnz / n;
  const int gt = std::max(1, std::min((n + MCG_BLOCK - 1) / MCG_BLOCK, 2048));
  if (mean <= 2.0)
    k_spmv<2, double><<<gt, MCG_BLOCK, 0, s>>>(n, A->row_ptr, A->col, A->val, u, q);
  else if (mean <= 4.0)
    k_spmv<4, double><<<gt, MCG_BLOCK, 0, s>>>(n, A->row_ptr, A->col, A->val, u, q);
  else if (mean <= 8.0)
    k_spmv<8, double><<<gt, MCG_BLOCK, 0, s>>>(n, A->row_ptr, A->col, A->val, u, q);
  else if (mean <= 16.0)
    k_spmv<16, double><<<gt, MCG_BLOCK, 0, s>>>(n, A->row_ptr, A->col, A->val, u, q);
  else
    k_spmv<32, double><<<gt, MCG_BLOCK, 0, s>>>(n, A->row_ptr, A->col, A->val, u, q);
  if (k > 0) {
    double *part = sc, *coef = sc + (size_t)kMaxBlocks * MCG_KMAX;
    const int nb = std::max(1, std::min((n + MCG_BLOCK - 1) / MCG_BLOCK, kMaxBlocks));
    if (k <= 8)
      launch_vtu<8>(nb, n, u, Vhat, k, part, s);
    else if (k <= 16)
      launch_vtu<16>(nb, n, u, Vhat, k, part, s);
    else if (k <= 32)
      launch_vtu<32>(nb, n, u, Vhat, k, part, s);
    else
      launch_vtu<64>(nb, n, u, Vhat, k, part, s);
    k_na_coef<<<1, MCG_KMAX, 0, s>>>(nb, k, part, lam, coef);
    const int gs = std::max(1, std::min((n + MCG_BLOCK - 1) / MCG_BLOCK, 1024));
    k_na_rankk<<<gs, MCG_BLOCK, 0, s>>>(n, Vhat, k, coef, q);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    mcg_last_hip_error = e;
    return MCG_EHIP;
  }
  return MCG_OK;
}
