// Setup stage: the k smallest eigenpairs of a sparse symmetric A on the
// device (the deflation data V-hat, Lambda-hat of the method), by
// Chebyshev-filtered subspace iteration with Rayleigh-Ritz.
//
// Blocks of p vectors (p = 16, 32, 48 or 64) are stored row-major (n x p) so
// that a sparse row gathers whole rows of the block.  Device kernels: the
// block product fused with one step of the Chebyshev three-term recurrence,
// the tall-skinny Gram product X^T Y (rows staged in LDS, one p x p partial
// per workgroup, summed in fixed order), the rotation X Q by a small matrix
// and the Ritz residual norms.  The p x p work (Cholesky, triangular inverse,
// symmetric eigensolver) runs on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mcg_deflation.h"
#include "mcg_internal.h"

namespace {

constexpr int EB = 256;  // threads per workgroup; 16 lanes per block row

// Counter-based uniform numbers in [-1, 1): the splitmix64 output function
// (Steele, Lea and Flood, 2014) applied to seed + golden-ratio increments.
__device__ inline double urand(uint64_t seed, uint64_t i) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void k_rand_block(int64_t cnt, uint64_t seed, double *__restrict__ X) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x)
    X[i] = urand(seed, (uint64_t)i);
}

// Y = alpha (A X - c X) + beta Z (Z may be null when beta = 0).  16 lanes per
// row; lane t owns columns t, t + 16, ...: a gathered row of X is read as PC
// coalesced 128-byte pieces, and the row's nonzeros are read once per lane
// group (the same address for all 16 lanes).
template <int PC>
__global__ __launch_bounds__(EB) void k_spmm_cheb(int n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const double *__restrict__ va,
                                                  const double *__restrict__ X,
                                                  double *__restrict__ Y,
                                                  const double *__restrict__ Z, double alpha,
                                                  double c, double beta) {
  constexpr int P = 16 * PC;
  constexpr int RB = EB / 16;
  const int t = threadIdx.x & 15;
  for (int i = blockIdx.x * RB + threadIdx.x / 16; i < n; i += gridDim.x * RB) {
    double acc[PC];
#pragma unroll
    for (int q = 0; q < PC; ++q) acc[q] = 0.0;
    const int s = rp[i], e = rp[i + 1];
    int p = s;
    for (; p + 3 < e; p += 4) {
      int cc[4];
      double a[4], xv[4][PC];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        cc[u] = ci[p + u];
        a[u] = va[p + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < PC; ++q) xv[u][q] = X[(size_t)cc[u] * P + t + 16 * q];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < PC; ++q) acc[q] += a[u] * xv[u][q];
    }
    for (; p < e; ++p) {
      const int cc = ci[p];
      const double a = va[p];
#pragma unroll
      for (int q = 0; q < PC; ++q) acc[q] += a * X[(size_t)cc * P + t + 16 * q];
    }
#pragma unroll
    for (int q = 0; q < PC; ++q) {
      const size_t o = (size_t)i * P + t + 16 * q;
      double y = alpha * (c != 0.0 ? acc[q] - c * X[o] : acc[q]);
      if (Z) y += beta * Z[o];
      Y[o] = y;
    }
  }
}

// One p x p partial of X^T Y per workgroup: 32 rows of X and Y at a time in
// LDS; thread e accumulates entries e, e + 256, ... of the partial.
template <int PC>
__global__ __launch_bounds__(EB) void k_gram(int n, const double *__restrict__ X,
                                             const double *__restrict__ Y,
                                             double *__restrict__ part) {
  constexpr int P = 16 * PC, R = 32, NE = (P * P + EB - 1) / EB;
  __shared__ double xs[R * P], ys[R * P];
  double acc[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) acc[q] = 0.0;
  for (int r0 = blockIdx.x * R; r0 < n; r0 += gridDim.x * R) {
    const int rows = min(R, n - r0);
    __syncthreads();
    for (int e = threadIdx.x; e < R * P; e += EB) {
      const bool in = e / P < rows;
      xs[e] = in ? X[(size_t)r0 * P + e] : 0.0;
      ys[e] = in ? Y[(size_t)r0 * P + e] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = threadIdx.x + q * EB;
      if (e < P * P) {
        const int a = e / P, b = e - a * P;
        double s = 0.0;
#pragma unroll 8
        for (int r = 0; r < R; ++r) s += xs[r * P + a] * ys[r * P + b];
        acc[q] += s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = threadIdx.x + q * EB;
    if (e < P * P) part[(size_t)blockIdx.x * P * P + e] = acc[q];
  }
}

// out[j] = sum over blocks b < nb of part[b * cnt + j], in block order
__global__ void k_sum_blocks(int nb, int cnt, const double *__restrict__ part,
                             double *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * cnt + j];
  out[j] = s;
}

// Xo = X Q (Q: p x p row-major), 16 rows of X per workgroup pass in LDS
template <int PC>
__global__ __launch_bounds__(EB) void k_rotate(int n, const double *__restrict__ X,
                                               const double *__restrict__ Q,
                                               double *__restrict__ Xo) {
  constexpr int P = 16 * PC, RB = EB / 16;
  __shared__ double qs[P * P];
  __shared__ double xs[RB * P];
  for (int e = threadIdx.x; e < P * P; e += EB) qs[e] = Q[e];
  const int t = threadIdx.x & 15, rl = threadIdx.x / 16;
  for (int r0 = blockIdx.x * RB; r0 < n; r0 += gridDim.x * RB) {
    __syncthreads();
    for (int e = threadIdx.x; e < RB * P; e += EB)
      xs[e] = (r0 + e / P < n) ? X[(size_t)r0 * P + e] : 0.0;
    __syncthreads();
    double acc[PC];
#pragma unroll
    for (int q = 0; q < PC; ++q) acc[q] = 0.0;
    for (int i = 0; i < P; ++i) {
      const double xv = xs[rl * P + i];
#pragma unroll
      for (int q = 0; q < PC; ++q) acc[q] += xv * qs[i * P + t + 16 * q];
    }
    const int r = r0 + rl;
    if (r < n) {
#pragma unroll
      for (int q = 0; q < PC; ++q) Xo[(size_t)r * P + t + 16 * q] = acc[q];
    }
  }
}

// Per-workgroup partials of ||W_j - theta_j X_j||^2 for every column j < p
template <int PC>
__global__ __launch_bounds__(EB) void k_colres(int n, const double *__restrict__ X,
                                               const double *__restrict__ W,
                                               const double *__restrict__ theta,
                                               double *__restrict__ part) {
  constexpr int P = 16 * PC, RB = EB / 16;
  __shared__ double red[4 * P];
  const int t = threadIdx.x & 15;
  double th[PC], acc[PC];
#pragma unroll
  for (int q = 0; q < PC; ++q) {
    th[q] = theta[t + 16 * q];
    acc[q] = 0.0;
  }
  for (int r = blockIdx.x * RB + threadIdx.x / 16; r < n; r += gridDim.x * RB) {
#pragma unroll
    for (int q = 0; q < PC; ++q) {
      const size_t o = (size_t)r * P + t + 16 * q;
      const double d = W[o] - th[q] * X[o];
      acc[q] += d * d;
    }
  }
  // lanes t, t + 16, t + 32, t + 48 of a wavefront hold the same columns
#pragma unroll
  for (int q = 0; q < PC; ++q) {
    acc[q] += __shfl_xor(acc[q], 16, 64);
    acc[q] += __shfl_xor(acc[q], 32, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane < 16) {
#pragma unroll
    for (int q = 0; q < PC; ++q) red[wave * P + t + 16 * q] = acc[q];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < P; j += EB)
    part[(size_t)blockIdx.x * P + j] = red[j] + red[P + j] + red[2 * P + j] + red[3 * P + j];
}

// Vhat (n x k, column-major) = the first k columns of the block
__global__ void k_extract(int n, int k, int P, const double *__restrict__ X,
                          double *__restrict__ V) {
  const int64_t cnt = (int64_t)n * k;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < cnt;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / n), r = (int)(idx - (int64_t)j * n);
    V[idx] = X[(size_t)r * P + j];
  }
}

// ---------------------------------------------------------------------------
// host: p x p dense linear algebra (p <= 64)
// ---------------------------------------------------------------------------

// G = R^T R with R upper triangular (row-major p x p); false if a pivot is
// not positive
bool cholesky_upper(const std::vector<double> &G, int p, std::vector<double> &R) {
  R.assign((size_t)p * p, 0.0);
  for (int j = 0; j < p; ++j) {
    double d = G[(size_t)j * p + j];
    for (int i = 0; i < j; ++i) d -= R[(size_t)i * p + j] * R[(size_t)i * p + j];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    const double rjj = std::sqrt(d);
    R[(size_t)j * p + j] = rjj;
    for (int c = j + 1; c < p; ++c) {
      double s = G[(size_t)j * p + c];
      for (int i = 0; i < j; ++i) s -= R[(size_t)i * p + j] * R[(size_t)i * p + c];
      R[(size_t)j * p + c] = s / rjj;
    }
  }
  return true;
}

// inverse of an upper triangular matrix (row-major), by columns
std::vector<double> inv_upper(const std::vector<double> &R, int p) {
  std::vector<double> Ri((size_t)p * p, 0.0);
  for (int c = 0; c < p; ++c) {
    Ri[(size_t)c * p + c] = 1.0 / R[(size_t)c * p + c];
    for (int r = c - 1; r >= 0; --r) {
      double s = 0.0;
      for (int i = r + 1; i <= c; ++i) s += R[(size_t)r * p + i] * Ri[(size_t)i * p + c];
      Ri[(size_t)r * p + c] = -s / R[(size_t)r * p + r];
    }
  }
  return Ri;
}

// Symmetric eigendecomposition H = Q diag(w) Q^T by cyclic Jacobi rotations
// (row-major; columns of Q are the eigenvectors), sorted ascending.
void sym_eig(std::vector<double> H, int p, std::vector<double> &w, std::vector<double> &Q) {
  Q.assign((size_t)p * p, 0.0);
  for (int i = 0; i < p; ++i) Q[(size_t)i * p + i] = 1.0;
  auto at = [&](int i, int j) -> double & { return H[(size_t)i * p + j]; };
  double fro = 0.0;
  for (double v : H) fro += v * v;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < p; ++i)
      for (int j = i + 1; j < p; ++j) off += at(i, j) * at(i, j);
    if (off <= 1e-32 * fro || off == 0.0) break;
    for (int a = 0; a < p; ++a)
      for (int b = a + 1; b < p; ++b) {
        const double hab = at(a, b);
        if (std::fabs(hab) <= 1e-300) continue;
        // rotation angle that zeroes H(a, b)
        const double th = (at(b, b) - at(a, a)) / (2.0 * hab);
        const double tt = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(tt * tt + 1.0), sn = tt * cs;
        for (int k = 0; k < p; ++k) {  // H <- H J (columns a, b)
          const double hka = at(k, a), hkb = at(k, b);
          at(k, a) = cs * hka - sn * hkb;
          at(k, b) = sn * hka + cs * hkb;
        }
        for (int k = 0; k < p; ++k) {  // H <- J^T H (rows a, b)
          const double hak = at(a, k), hbk = at(b, k);
          at(a, k) = cs * hak - sn * hbk;
          at(b, k) = sn * hak + cs * hbk;
        }
        for (int k = 0; k < p; ++k) {  // Q <- Q J
          const double qka = Q[(size_t)k * p + a], qkb = Q[(size_t)k * p + b];
          Q[(size_t)k * p + a] = cs * qka - sn * qkb;
          Q[(size_t)k * p + b] = sn * qka + cs * qkb;
        }
      }
  }
  std::vector<int> order(p);
  for (int i = 0; i < p; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return at(x, x) < at(y, y); });
  w.resize(p);
  std::vector<double> Qs((size_t)p * p);
  for (int c = 0; c < p; ++c) {
    w[c] = at(order[c], order[c]);
    for (int r = 0; r < p; ++r) Qs[(size_t)r * p + c] = Q[(size_t)r * p + order[c]];
  }
  Q.swap(Qs);
}

struct EigWork {
  int n = 0, P = 0, nbg = 0, nbr = 0;
  const int32_t *rp = nullptr, *ci = nullptr;
  const double *va = nullptr;
  double *buf[4] = {nullptr, nullptr, nullptr, nullptr};
  double *W = nullptr, *part = nullptr, *small = nullptr, *small2 = nullptr;
  hipStream_t s = nullptr;
  int spmm_calls = 0;

  ~EigWork() {
    for (double *b : buf)
      if (b) (void)hipFree(b);
    double *o[] = {W, part, small, small2};
    for (double *b : o)
      if (b) (void)hipFree(b);
  }
};

#define MCG_SWITCH_PC(PCv, ...)                         \
  switch (PCv) {                                        \
    case 1: { constexpr int PC = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int PC = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int PC = 3; __VA_ARGS__; } break; \
    default: { constexpr int PC = 4; __VA_ARGS__; } break; \
  }

int spmm(EigWork &w, const double *X, double *Y, const double *Z, double alpha, double c,
         double beta) {
  const int g = std::max(1, std::min((w.n + 15) / 16, 16384));
  MCG_SWITCH_PC(w.P / 16, (k_spmm_cheb<PC><<<g, EB, 0, w.s>>>(w.n, w.rp, w.ci, w.va, X, Y, Z,
                                                              alpha, c, beta)));
  ++w.spmm_calls;
  return hipGetLastError() == hipSuccess ? MCG_OK : MCG_EHIP;
}

// host copy of X^T Y (P x P)
int gram(EigWork &w, const double *X, const double *Y, std::vector<double> &G) {
  const int P = w.P;
  MCG_SWITCH_PC(P / 16, (k_gram<PC><<<w.nbg, EB, 0, w.s>>>(w.n, X, Y, w.part)));
  k_sum_blocks<<<(P * P + 255) / 256, 256, 0, w.s>>>(w.nbg, P * P, w.part, w.small);
  G.resize((size_t)P * P);
  if (hipMemcpyAsync(G.data(), w.small, sizeof(double) * P * P, hipMemcpyDeviceToHost, w.s) !=
          hipSuccess ||
      hipStreamSynchronize(w.s) != hipSuccess)
    return MCG_EHIP;
  return MCG_OK;
}

int rotate(EigWork &w, const double *X, const std::vector<double> &Q, double *Xo) {
  const int P = w.P;
  if (hipMemcpyAsync(w.small2, Q.data(), sizeof(double) * P * P, hipMemcpyHostToDevice, w.s) !=
      hipSuccess)
    return MCG_EHIP;
  const int g = std::max(1, std::min((w.n + 15) / 16, 4096));
  MCG_SWITCH_PC(P / 16, (k_rotate<PC><<<g, EB, 0, w.s>>>(w.n, X, w.small2, Xo)));
  // the next upload of Q must not overwrite small2 before this kernel read it
  return hipStreamSynchronize(w.s) == hipSuccess ? MCG_OK : MCG_EHIP;
}

int free_buffer(const EigWork &w, std::initializer_list<const double *> busy) {
  for (int i = 0; i < 4; ++i) {
    bool used = false;
    for (const double *b : busy) used |= (b == w.buf[i]);
    if (!used) return i;
  }
  return -1;
}

// X <- an orthonormal basis of span(Y) by Cholesky QR, twice (a diagonal
// shift makes the first pass succeed when Y is nearly rank deficient)
int orthonormalise(EigWork &w, double *Y, double **Xout) {
  const int P = w.P;
  double *cur = Y;
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<double> G, R;
    int rc = gram(w, cur, cur, G);
    if (rc) return rc;
    if (!cholesky_upper(G, P, R)) {
      double tr = 0.0;
      for (int i = 0; i < P; ++i) tr += G[(size_t)i * P + i];
      for (int i = 0; i < P; ++i) G[(size_t)i * P + i] += 1e-13 * tr;
      if (!cholesky_upper(G, P, R)) return MCG_BREAKDOWN;
    }
    const int o = free_buffer(w, {cur});
    if ((rc = rotate(w, cur, inv_upper(R, P), w.buf[o]))) return rc;
    cur = w.buf[o];
  }
  *Xout = cur;
  return MCG_OK;
}

// Rayleigh-Ritz on span(X): W = A X, H = X^T W, X <- X Q, W <- W Q; theta
// ascending; res[j] = ||W_j - theta_j X_j||
int rayleigh_ritz(EigWork &w, double **X, std::vector<double> &theta, std::vector<double> &res) {
  const int P = w.P;
  int rc = spmm(w, *X, w.W, nullptr, 1.0, 0.0, 0.0);
  if (rc) return rc;
  std::vector<double> H, Q;
  if ((rc = gram(w, *X, w.W, H))) return rc;
  for (int i = 0; i < P; ++i)
    for (int j = i + 1; j < P; ++j) {
      const double m = 0.5 * (H[(size_t)i * P + j] + H[(size_t)j * P + i]);
      H[(size_t)i * P + j] = H[(size_t)j * P + i] = m;
    }
  sym_eig(H, P, theta, Q);
  const int o1 = free_buffer(w, {*X});
  if ((rc = rotate(w, *X, Q, w.buf[o1]))) return rc;
  const int o2 = free_buffer(w, {*X, w.buf[o1]});
  if ((rc = rotate(w, w.W, Q, w.buf[o2]))) return rc;
  // W <- the rotated block (copy back into W's buffer)
  if (hipMemcpyAsync(w.W, w.buf[o2], sizeof(double) * (size_t)w.n * P, hipMemcpyDeviceToDevice,
                     w.s) != hipSuccess)
    return MCG_EHIP;
  *X = w.buf[o1];
  if (hipMemcpyAsync(w.small2, theta.data(), sizeof(double) * P, hipMemcpyHostToDevice, w.s) !=
      hipSuccess)
    return MCG_EHIP;
  MCG_SWITCH_PC(P / 16, (k_colres<PC><<<w.nbr, EB, 0, w.s>>>(w.n, *X, w.W, w.small2, w.part)));
  k_sum_blocks<<<1, 64, 0, w.s>>>(w.nbr, P, w.part, w.small);
  res.resize(P);
  if (hipMemcpyAsync(res.data(), w.small, sizeof(double) * P, hipMemcpyDeviceToHost, w.s) !=
          hipSuccess ||
      hipStreamSynchronize(w.s) != hipSuccess)
    return MCG_EHIP;
  for (double &r : res) r = std::sqrt(std::max(r, 0.0));
  return MCG_OK;
}

}  // namespace

extern "C" void minres_cg_eig_default_options(mcg_eig_options_t *opt) {
  if (opt) std::memset(opt, 0, sizeof(*opt));
}

extern "C" int minres_cg_lowest_eigs(const mcg_csr_t *A, int32_t k, const mcg_eig_options_t *opt_in,
                                     double *Vhat, double *lam, mcg_eig_stats_t *st,
                                     void *stream) {
  if (!A || !Vhat || !lam || k < 1 || A->n <= 0 || A->nnz <= 0 || !A->row_ptr || !A->col ||
      !A->val || A->nnz >= ((int64_t)1 << 31))
    return MCG_EINVAL;
  mcg_eig_options_t opt;
  minres_cg_eig_default_options(&opt);
  if (opt_in) opt = *opt_in;
  const int n = A->n;
  int P = opt.block > 0 ? opt.block : k + std::max(8, k / 2);
  P = (P + 15) / 16 * 16;
  if (P > 64 || P < k || P > n || opt.degree < 0 || opt.max_outer < 0 || opt.tol < 0.0)
    return MCG_EINVAL;
  const int degree = opt.degree > 0 ? opt.degree : 64;
  const int max_outer = opt.max_outer > 0 ? opt.max_outer : 400;
  const double tol = opt.tol > 0.0 ? opt.tol : 1e-10;
  hipStream_t s = (hipStream_t)stream;

  // structure check and the Gershgorin bound on the host
  std::vector<int32_t> rp(n + 1), ci(A->nnz);
  std::vector<double> va(A->nnz);
  if (hipMemcpy(rp.data(), A->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(ci.data(), A->col, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(va.data(), A->val, sizeof(double) * A->nnz, hipMemcpyDeviceToHost) != hipSuccess)
    return MCG_EHIP;
  if (rp[0] != 0 || rp[n] != A->nnz) return MCG_EINVAL;
  double bound = 0.0;
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return MCG_EINVAL;
    double row = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      if (ci[p] < 0 || ci[p] >= n || (p > rp[i] && ci[p] <= ci[p - 1]) || !std::isfinite(va[p]))
        return MCG_EINVAL;
      row += std::fabs(va[p]);
    }
    bound = std::max(bound, row);
  }

  EigWork w;
  w.n = n;
  w.P = P;
  w.rp = A->row_ptr;
  w.ci = A->col;
  w.va = A->val;
  w.s = s;
  w.nbg = std::max(1, std::min((n + 31) / 32, 1024));
  w.nbr = std::max(1, std::min((n + 15) / 16, 1024));
  const size_t blk = (size_t)n * P;
  for (double *&b : w.buf)
    if (hipMalloc((void **)&b, sizeof(double) * blk) != hipSuccess) return MCG_ENOMEM;
  if (hipMalloc((void **)&w.W, sizeof(double) * blk) != hipSuccess ||
      hipMalloc((void **)&w.part, sizeof(double) * (size_t)std::max(w.nbg * P * P, w.nbr * P)) !=
          hipSuccess ||
      hipMalloc((void **)&w.small, sizeof(double) * P * P) != hipSuccess ||
      hipMalloc((void **)&w.small2, sizeof(double) * P * P) != hipSuccess)
    return MCG_ENOMEM;

  k_rand_block<<<2048, 256, 0, s>>>((int64_t)blk, opt.seed, w.buf[0]);
  double *X = nullptr;
  int rc = orthonormalise(w, w.buf[0], &X);
  std::vector<double> theta, res;
  if (!rc) rc = rayleigh_ritz(w, &X, theta, res);
  int outer = 0;
  bool conv = false;
  double maxres = 0.0;
  while (!rc) {
    maxres = 0.0;
    for (int j = 0; j < k; ++j) maxres = std::max(maxres, res[j]);
    if (maxres <= tol * bound) {
      conv = true;
      break;
    }
    if (outer >= max_outer) break;
    ++outer;
    // filter: damp [a, bound], a = largest Ritz value of the block; scaled
    // three-term recurrence normalised at the smallest Ritz value a0
    const double a = theta[P - 1], a0 = theta[0];
    const double e = 0.5 * (bound - a), c = 0.5 * (bound + a);
    if (!(e > 0.0) || !(a0 < a)) break;
    double sg = e / (a0 - c);
    const double tau = 2.0 / sg;
    double *Y0 = X;
    double *Y1 = w.buf[free_buffer(w, {Y0})];
    if ((rc = spmm(w, Y0, Y1, nullptr, sg / e, c, 0.0))) break;
    for (int d = 2; d <= degree; ++d) {
      const double sn = 1.0 / (tau - sg);
      double *Y2 = w.buf[free_buffer(w, {Y0, Y1})];
      if ((rc = spmm(w, Y1, Y2, Y0, 2.0 * sn / e, c, -sg * sn))) break;
      Y0 = Y1;
      Y1 = Y2;
      sg = sn;
    }
    if (rc) break;
    if ((rc = orthonormalise(w, Y1, &X))) break;
    if ((rc = rayleigh_ritz(w, &X, theta, res))) break;
  }
  if (rc) return rc;
  k_extract<<<2048, 256, 0, s>>>(n, k, P, X, Vhat);
  if (hipStreamSynchronize(s) != hipSuccess) return MCG_EHIP;
  int neg = 0;
  for (int j = 0; j < k; ++j) {
    lam[j] = theta[j];
    neg += theta[j] < 0.0;
  }
  if (st) {
    st->outer_its = outer;
    st->spmm_calls = w.spmm_calls;
    st->negative = neg;
    st->converged = conv ? 1 : 0;
    st->max_residual = maxres;
    st->bound = bound;
    st->next_ritz = k < P ? theta[k] : NAN;
  }
  return MCG_OK;
}
