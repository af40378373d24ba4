// Second-level preconditioners beyond the diagonal ones.
//
// ILDL0: incomplete L D L^T with zero fill on the strictly lower pattern of
// A and signed pivots -- the symmetric form of the ILU(0) of A that the paper
// uses as the inner preconditioner (Section 4).  The factor is computed once
// at create on the host (IKJ order: row i is reduced by the already final
// rows k < i of its lower pattern); t = (L D L^T)^{-1} g is applied on the GPU
// by level-scheduled sweeps.  Rows are grouped in node blocks of `block_size`
// unknowns; a block's level is one more than the highest level of the blocks
// its rows depend on, so each level is one kernel launch over independent
// blocks (8 levels for the 8-colour ordered 27-point matrices).  Dependencies
// inside a block are resolved in registers by the block's lane group.
//
// CCT: t = C (C^T g) with C lower triangular (the learned factor), as two
// CSR products (C^T is stored explicitly).
#include <algorithm>
#include <cmath>
#include <vector>

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

struct ildl_data {
  int n = 0, bs = 1, nlevels = 0;
  // L (strictly lower) and U = L^T (strictly upper), CSR, FP64 + FP32
  int32_t *l_rp = nullptr, *l_ci = nullptr, *u_rp = nullptr, *u_ci = nullptr;
  double *l_v = nullptr, *u_v = nullptr, *dinv = nullptr;
  float *l_v32 = nullptr, *u_v32 = nullptr, *dinv32 = nullptr;
  int32_t *level_nodes = nullptr;       // node ids ordered by level
  std::vector<int32_t> level_ptr;       // host: nodes of level l at [ptr[l], ptr[l+1])
  int64_t modified_pivots = 0;
};

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
// false (no copy) when that fill would exceed half the nonzeros.
bool csr_to_bsr(int n, int bs, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                const std::vector<double> &v, std::vector<int32_t> &brp,
                std::vector<int32_t> &bci, std::vector<double> &bv) {
  const int N = n / bs;
  brp.assign(N + 1, 0);
  bci.clear();
  std::vector<int32_t> mark(N, -1), cols;
  for (int I = 0; I < N; ++I) {
    cols.clear();
    for (int a = 0; a < bs; ++a)
      for (int p = rp[I * bs + a]; p < rp[I * bs + a + 1]; ++p) {
        const int J = ci[p] / bs;
        if (mark[J] != I) {
          mark[J] = I;
          cols.push_back(J);
        }
      }
    std::sort(cols.begin(), cols.end());
    bci.insert(bci.end(), cols.begin(), cols.end());
    brp[I + 1] = (int32_t)bci.size();
  }
  const size_t nvals = bci.size() * (size_t)bs * bs;
  if ((double)nvals > 1.5 * (double)v.size()) return false;
  bv.assign(nvals, 0.0);
  for (int I = 0; I < N; ++I)
    for (int a = 0; a < bs; ++a)
      for (int p = rp[I * bs + a]; p < rp[I * bs + a + 1]; ++p) {
        const int J = ci[p] / bs, b = ci[p] % bs;
        const auto it = std::lower_bound(bci.begin() + brp[I], bci.begin() + brp[I + 1], J);
        const size_t blk = (size_t)(it - bci.begin());
        bv[(blk * bs + a) * bs + b] = v[p];
      }
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
  return std::vector<TO>(v.begin(), v.end());
}

void csr_transpose(int n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                   const std::vector<double> &v, std::vector<int32_t> &trp,
                   std::vector<int32_t> &tci, std::vector<double> &tv) {
  trp.assign(n + 1, 0);
  for (int32_t c : ci) trp[c + 1]++;
  for (int i = 0; i < n; ++i) trp[i + 1] += trp[i];
  tci.resize(ci.size());
  tv.resize(ci.size());
  std::vector<int32_t> fill(trp.begin(), trp.end() - 1);
  for (int i = 0; i < n; ++i)  // rows in increasing order -> sorted columns in the transpose
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
      const int32_t q = fill[ci[p]]++;
      tci[q] = i;
      tv[q] = v[p];
    }
}

// ---------------------------------------------------------------------------
// sweep kernels: G lanes per node block; levels launched in order
// ---------------------------------------------------------------------------
template <int G, int BS, typename T>
__global__ __launch_bounds__(256) void k_ildl_forward(
    int nnodes_level, const int32_t *__restrict__ nodes, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ ci, const T *__restrict__ lv, const T *__restrict__ g,
    T *__restrict__ u, const DevState *__restrict__ S, int check_done) {
  if (check_done && S->done) return;
  const int lane = threadIdx.x & (G - 1);
  const int slot = (blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (slot >= nnodes_level) return;  // whole lane group leaves together
  const int node = nodes[slot];
  const int r0 = node * BS;
  T ub[BS];
#pragma unroll
  for (int d = 0; d < BS; ++d) {
    const int i = r0 + d;
    const int s = rp[i], e = rp[i + 1];
    const int eext = e - d;  // the last d entries are the block's own columns r0..i-1
    T acc = 0;
    for (int p = s + lane; p < eext; p += G) acc += lv[p] * u[ci[p]];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
    T ui = g[i] - acc;
#pragma unroll
    for (int q = 0; q < d; ++q) ui -= lv[eext + q] * ub[q];
    ub[d] = ui;
    if (lane == 0) u[i] = ui;
  }
}

template <int G, int BS, typename T>
__global__ __launch_bounds__(256) void k_ildl_backward(
    int nnodes_level, const int32_t *__restrict__ nodes, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ ci, const T *__restrict__ uv, const T *__restrict__ dinv,
    T *__restrict__ t, const DevState *__restrict__ S, int check_done) {
  if (check_done && S->done) return;
  const int lane = threadIdx.x & (G - 1);
  const int slot = (blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (slot >= nnodes_level) return;
  const int node = nodes[slot];
  const int r0 = node * BS;
  T tb[BS];
#pragma unroll
  for (int d = BS - 1; d >= 0; --d) {
    const int i = r0 + d;
    const int s = rp[i], e = rp[i + 1];
    const int nint = BS - 1 - d;  // the first entries are the block's own columns i+1..r0+bs-1
    T acc = 0;
    for (int p = s + nint + lane; p < e; p += G) acc += uv[p] * t[ci[p]];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
    T ti = t[i] * dinv[i] - acc;
#pragma unroll
    for (int q = 0; q < nint; ++q) ti -= uv[s + q] * tb[d + 1 + q];
    tb[d] = ti;
    if (lane == 0) t[i] = ti;
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
  // IKJ: w holds row i (lower part + diagonal) in dense form
  std::vector<double> w(n, 0.0);
  std::vector<int32_t> mark(n, -1);
  int64_t modified = 0;
  for (int i = 0; i < n; ++i) {
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
      ++modified;
    }
    // an exactly zero (pivtol = 0) or non-finite pivot has no inverse
    if (!(wi != 0.0) || !std::isfinite(wi)) return MCG_EINVAL;
    d[i] = wi;
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
  D->n = n;
  D->bs = bs;
  D->modified_pivots = modified;
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
  D->level_ptr.assign(D->nlevels + 1, 0);
  for (int I = 0; I < nn; ++I) D->level_ptr[lev[I] + 1]++;
  for (int l = 0; l < D->nlevels; ++l) D->level_ptr[l + 1] += D->level_ptr[l];
  std::vector<int32_t> order(nn);
  {
    std::vector<int32_t> fill(D->level_ptr.begin(), D->level_ptr.end() - 1);
    for (int I = 0; I < nn; ++I) order[fill[lev[I]]++] = I;
  }
  // U = L^T (rows hold entries of the columns of L)
  std::vector<int32_t> urp, uci;
  std::vector<double> uv;
  csr_transpose(n, lrp, lci, lv, urp, uci, uv);
  std::vector<double> dinv(n);
  for (int i = 0; i < n; ++i) dinv[i] = 1.0 / d[i];
  int rc;
  if ((rc = upload(&D->l_rp, lrp.data(), lrp.size())) || (rc = upload(&D->l_ci, lci.data(), lci.size())) ||
      (rc = upload(&D->l_v, lv.data(), lv.size())) || (rc = upload(&D->u_rp, urp.data(), urp.size())) ||
      (rc = upload(&D->u_ci, uci.data(), uci.size())) || (rc = upload(&D->u_v, uv.data(), uv.size())) ||
      (rc = upload(&D->dinv, dinv.data(), dinv.size())) ||
      (rc = upload(&D->level_nodes, order.data(), order.size())))
    return rc;
  if (h->opt.precision == MCG_PREC_MIXED) {
    auto lv32 = convert<float>(lv), uv32 = convert<float>(uv), di32 = convert<float>(dinv);
    if ((rc = upload(&D->l_v32, lv32.data(), lv32.size())) ||
        (rc = upload(&D->u_v32, uv32.data(), uv32.size())) ||
        (rc = upload(&D->dinv32, di32.data(), di32.size())))
      return rc;
  }
  return MCG_OK;
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
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return MCG_EINVAL;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
      if (ci[q] < 0 || ci[q] > i) return MCG_EINVAL;  // lower triangular
      if (q > rp[i] && ci[q] <= ci[q - 1]) return MCG_EINVAL;
      if (!std::isfinite(v[q])) return MCG_EINVAL;
    }
  }
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
        if ((rc = mcg_bsell_build(&D->c_bsell, bs, n / bs, brp, bci, bv, 0.5, mixed, s, mixed)) ||
            (rc = mcg_bsell_build(&D->ct_bsell, bs, n / bs, tbrp, tbci, tbv, 0.5, mixed, s,
                                  mixed)))
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

void mcg_pc_release_extra(mcg_pc *p) {
  if (p->ildl) {
    ildl_data *D = (ildl_data *)p->ildl;
    void *b[] = {D->l_rp, D->l_ci, D->u_rp, D->u_ci, D->l_v, D->u_v, D->dinv, D->l_v32, D->u_v32,
                 D->dinv32, D->level_nodes};
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

template <typename T>
void mcg_ildl0_apply(const mcg_pc *p, const T *g, T *t, DevState *S, int check_done,
                     hipStream_t s) {
  const ildl_data *D = (const ildl_data *)p->ildl;
  constexpr int G = 16;
  const T *lv = pick<T>(D->l_v, D->l_v32), *uv = pick<T>(D->u_v, D->u_v32);
  const T *dinv = pick<T>(D->dinv, D->dinv32);
  switch (D->bs) {
#define MCG_ILDL_SWEEPS(BSV)                                                                    \
  case BSV:                                                                                     \
    for (int l = 0; l < D->nlevels; ++l) {                                                      \
      const int cnt = D->level_ptr[l + 1] - D->level_ptr[l];                                    \
      k_ildl_forward<G, BSV, T><<<(cnt * G + 255) / 256, 256, 0, s>>>(                          \
          cnt, D->level_nodes + D->level_ptr[l], D->l_rp, D->l_ci, lv, g, t, S, check_done);    \
    }                                                                                           \
    for (int l = D->nlevels - 1; l >= 0; --l) {                                                 \
      const int cnt = D->level_ptr[l + 1] - D->level_ptr[l];                                    \
      k_ildl_backward<G, BSV, T><<<(cnt * G + 255) / 256, 256, 0, s>>>(                         \
          cnt, D->level_nodes + D->level_ptr[l], D->u_rp, D->u_ci, uv, dinv, t, S, check_done); \
    }                                                                                           \
    break;
    MCG_ILDL_SWEEPS(1)
    MCG_ILDL_SWEEPS(2)
    MCG_ILDL_SWEEPS(3)
    MCG_ILDL_SWEEPS(4)
#undef MCG_ILDL_SWEEPS
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

int mcg_ildl0_levels(const mcg_pc *p) {
  return p && p->ildl ? ((const ildl_data *)p->ildl)->nlevels : 0;
}

int64_t mcg_ildl0_modified_pivots(const mcg_pc *p) {
  return p && p->ildl ? ((const ildl_data *)p->ildl)->modified_pivots : 0;
}

template void mcg_ildl0_apply<double>(const mcg_pc *, const double *, double *, DevState *, int,
                                      hipStream_t);
template void mcg_ildl0_apply<float>(const mcg_pc *, const float *, float *, DevState *, int,
                                     hipStream_t);
template void mcg_cct_apply<double>(const mcg_pc *, const double *, double *, DevState *, int,
                                    hipStream_t);
template void mcg_cct_apply<float>(const mcg_pc *, const float *, float *, DevState *, int,
                                   hipStream_t);
