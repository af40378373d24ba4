// Learned second-level preconditioner M_cg^{-1} = C C^T (network defined in
// include/mcg_learned.h).
//
// Data layout in HBM (all FP32 unless noted):
//   node graph   node_ptr[N+1], src[E], dst[E], rev[E] (int32): directed edges
//                I != J sorted by (I, J); rev[e] is the edge (J, I)
//   features     xn[N][dn], fe[E][de]
//   activations  h[l][N][32] (l = 0..4), e[l][E][32] (l = 0..4),
//                m[l][E][32], agg[l][N][32], rl[l][N][32] (l = 0..3)
//   heads        ct[E*de + N*dn] (C block values before row scaling),
//                o[N][dn] (pre-softplus node outputs)
//   C            c_rp/c_ci (int32), c_val (FP64) on lower(A); c_map[p] = the
//                ct slot of nonzero p; transpose ct_rp/ct_ci/ct_perm
// Every per-node and per-edge row is 32 floats = 128 B, so a row is one
// aligned cache line and an MFMA operand fragment (8 consecutive features)
// is two 16-byte loads.
//
// Kernels.  The four hidden edge and node MLPs (96 -> 32 and 64 -> 32) and
// their backward products run on v_mfma_f32_16x16x32_bf16: one wavefront
// owns 16 edges (or 16 nodes), loads [h_src; h_dst; e] as three K = 32
// slices straight from HBM, and keeps the BF16 weight fragments in
// registers.  Weight gradients (sum over all edges of dV^T X) are MFMA
// products with K running over edges, accumulated per wavefront and reduced
// deterministically.  The input embeddings and output heads (K or N <= 16)
// and the loss SpMMs are plain vector kernels.  Aggregation over neighbours
// is a segmented sum over the CSR of the node graph (no atomics); the
// backward's scatter to destination nodes is a gather through rev[].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/mcg_learned.h"
#include "mcg_internal.h"

namespace {

constexpr int HID = 32;
constexpr int NLAYER = 4;
constexpr float kEpsOff = 0.1f;
constexpr float kDiagFloor = 1e-3f;
constexpr int kMaxBS = 4;
constexpr int kMaxDeg = 64;
constexpr int kMaxNB = 32;
constexpr int kWgradWaves = 1024;   // wavefronts of the weight-gradient reductions
constexpr int kOuterBlocks = 512;   // blocks of the small outer-product reductions

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void ld8(const float *p, float v[8]) {
  const float4 a = *reinterpret_cast<const float4 *>(p);
  const float4 b = *reinterpret_cast<const float4 *>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

__device__ __forceinline__ void st8(float *p, const float v[8]) {
  *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
  *reinterpret_cast<float4 *>(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
}

__device__ __forceinline__ bf16x8 cvt8(const float v[8]) {
  bf16x8 r;
#pragma unroll
  for (int q = 0; q < 8; ++q) r[q] = (__bf16)v[q];
  return r;
}

__device__ __forceinline__ bf16x8 ldw8(const __bf16 *p) {
  return *reinterpret_cast<const bf16x8 *>(p);
}

// ---------------------------------------------------------------------------
// parameters

struct Layout {
  int bs, dn, de;
  int64_t win_n, win_e, layer0, layer_stride, w_oe, w_od, b_od, total;
  int64_t w1(int l) const { return layer0 + l * layer_stride; }
  int64_t b1(int l) const { return w1(l) + HID * 3 * HID; }
  int64_t w2(int l) const { return b1(l) + HID; }
  int64_t b2(int l) const { return w2(l) + HID * 2 * HID; }
};

Layout make_layout(int bs) {
  Layout L{};
  L.bs = bs;
  L.dn = bs * (bs + 1) / 2;
  L.de = bs * bs;
  L.win_n = 0;
  L.win_e = HID * L.dn;
  L.layer0 = L.win_e + HID * L.de;
  L.layer_stride = HID * 3 * HID + HID + HID * 2 * HID + HID;
  L.w_oe = L.layer0 + NLAYER * L.layer_stride;
  L.w_od = L.w_oe + L.de * HID;
  L.b_od = L.w_od + L.dn * HID;
  L.total = L.b_od + L.dn;
  return L;
}

// theta_r = bf16(theta) as float; wbf = the hidden-layer weights as bf16,
// per layer W1 (32 x 96) then W2 (32 x 64)
__global__ void k_round_params(int64_t P, const float *theta, float *theta_r, __bf16 *wbf,
                               int64_t layer0, int64_t layer_stride) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const __bf16 b = (__bf16)theta[i];
  theta_r[i] = (float)b;
  const int64_t rel = i - layer0;
  if (rel >= 0 && rel < NLAYER * layer_stride) {
    const int l = (int)(rel / layer_stride);
    const int64_t o = rel - l * layer_stride;
    const int64_t w1n = HID * 3 * HID, w2o = w1n + HID;
    if (o < w1n)
      wbf[(int64_t)l * (HID * 5 * HID) + o] = b;
    else if (o >= w2o && o < w2o + HID * 2 * HID)
      wbf[(int64_t)l * (HID * 5 * HID) + w1n + (o - w2o)] = b;
  }
}

// ---------------------------------------------------------------------------
// forward

// y[r][j] = sum_k W[j][k] x[r][k], W (32 x K) row-major, K <= 16
__global__ void k_embed(int64_t R, int K, const float *x, const float *W, float *y) {
  __shared__ float w[HID * 16];
  for (int t = threadIdx.x; t < HID * K; t += blockDim.x) w[t] = W[t];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * HID) return;
  const int64_t r = i / HID;
  const int j = (int)(i % HID);
  float acc = 0.f;
  for (int k = 0; k < K; ++k) acc += w[j * K + k] * x[r * K + k];
  y[i] = acc;
}

// edge MLP of one layer: m = relu(W1 [h_src; h_dst; e_in] + b1),
// e_out = e_in + m; one wavefront per 16 edges
__global__ __launch_bounds__(256) void k_edge_fwd(int64_t E, const int32_t *__restrict__ src,
                                                  const int32_t *__restrict__ dst,
                                                  const float *__restrict__ h,
                                                  const float *__restrict__ e_in,
                                                  const __bf16 *__restrict__ W1,
                                                  const float *__restrict__ b1,
                                                  float *__restrict__ m_out,
                                                  float *__restrict__ e_out) {
  const int lane = threadIdx.x & 63;
  const int64_t e0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 16;
  if (e0 >= E) return;
  const int i = lane & 15, kq = lane >> 4;
  bf16x8 wb[2][3];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) wb[nt][kk] = ldw8(W1 + (16 * nt + i) * 96 + 32 * kk + 8 * kq);
  const int64_t e = min(e0 + i, E - 1);
  float v[8];
  ld8(h + (int64_t)src[e] * HID + 8 * kq, v);
  const bf16x8 a0 = cvt8(v);
  ld8(h + (int64_t)dst[e] * HID + 8 * kq, v);
  const bf16x8 a1 = cvt8(v);
  ld8(e_in + e * HID + 8 * kq, v);
  const bf16x8 a2 = cvt8(v);
  f32x4 acc[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    acc[nt] = mfma16(a0, wb[nt][0], acc[nt]);
    acc[nt] = mfma16(a1, wb[nt][1], acc[nt]);
    acc[nt] = mfma16(a2, wb[nt][2], acc[nt]);
  }
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const int j = 16 * nt + i;
    const float bj = b1[j];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t er = e0 + 4 * kq + r;
      if (er < E) {
        const float mv = fmaxf(acc[nt][r] + bj, 0.f);
        m_out[er * HID + j] = mv;
        e_out[er * HID + j] = e_in[er * HID + j] + mv;
      }
    }
  }
}

// node MLP of one layer: a = sum over the node's edges of m,
// h_out = h_in + relu(W2 [h_in; a] + b2); one wavefront per 16 nodes
__global__ __launch_bounds__(256) void k_node_fwd(int N, const int32_t *__restrict__ node_ptr,
                                                  const float *__restrict__ h_in,
                                                  const float *__restrict__ m,
                                                  const __bf16 *__restrict__ W2,
                                                  const float *__restrict__ b2,
                                                  float *__restrict__ agg,
                                                  float *__restrict__ rl,
                                                  float *__restrict__ h_out) {
  const int lane = threadIdx.x & 63;
  const int64_t n0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 16;
  if (n0 >= N) return;
  const int i = lane & 15, kq = lane >> 4;
  bf16x8 wb[2][2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) wb[nt][kk] = ldw8(W2 + (16 * nt + i) * 64 + 32 * kk + 8 * kq);
  const int64_t I = min(n0 + i, (int64_t)N - 1);
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, v[8];
  for (int p = node_ptr[I]; p < node_ptr[I + 1]; ++p) {
    ld8(m + (int64_t)p * HID + 8 * kq, v);
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] += v[q];
  }
  if (n0 + i < N) st8(agg + I * HID + 8 * kq, s);
  ld8(h_in + I * HID + 8 * kq, v);
  const bf16x8 a0 = cvt8(v), a1 = cvt8(s);
  f32x4 acc[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    acc[nt] = mfma16(a0, wb[nt][0], acc[nt]);
    acc[nt] = mfma16(a1, wb[nt][1], acc[nt]);
  }
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const int j = 16 * nt + i;
    const float bj = b2[j];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t nr = n0 + 4 * kq + r;
      if (nr < N) {
        const float rv = fmaxf(acc[nt][r] + bj, 0.f);
        rl[nr * HID + j] = rv;
        h_out[nr * HID + j] = h_in[nr * HID + j] + rv;
      }
    }
  }
}

__device__ __forceinline__ float softplus(float x) {
  return x > 20.f ? x : log1pf(expf(x));
}
__device__ __forceinline__ float sigmoid(float x) { return 1.f / (1.f + expf(-x)); }

// is slot q of the packed lower triangle (row-major) a diagonal entry
__device__ __forceinline__ bool tri_diag(int q, int bs) {
  for (int a = 0; a < bs; ++a)
    if (q == a * (a + 3) / 2) return true;
  return false;
}

// off-diagonal blocks (J < I): ct[e][q] = 0.1 * sum_k W_oe[q][k] e[e][k]
__global__ void k_heads_edges(int64_t E, int de, const int32_t *src, const int32_t *dst,
                              const float *e_fin, const float *W_oe, float *ct) {
  __shared__ float w[kMaxBS * kMaxBS * HID];
  for (int t = threadIdx.x; t < de * HID; t += blockDim.x) w[t] = W_oe[t];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E || dst[e] >= src[e]) return;
  float x[HID];
  for (int k = 0; k < HID; k += 8) ld8(e_fin + e * HID + k, x + k);
  for (int q = 0; q < de; ++q) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < HID; ++k) acc += w[q * HID + k] * x[k];
    ct[e * de + q] = kEpsOff * acc;
  }
}

// diagonal blocks: o = W_od h + b_od; softplus(o) + floor on the diagonal,
// 0.1 * o strictly below
__global__ void k_heads_nodes(int N, int bs, int dn, int64_t ct_off, const float *h_fin,
                              const float *W_od, const float *b_od, float *o_save, float *ct) {
  __shared__ float w[(kMaxBS * (kMaxBS + 1) / 2) * (HID + 1)];
  for (int t = threadIdx.x; t < dn * HID; t += blockDim.x) w[t] = W_od[t];
  for (int t = threadIdx.x; t < dn; t += blockDim.x) w[dn * HID + t] = b_od[t];
  __syncthreads();
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= N) return;
  float x[HID];
  for (int k = 0; k < HID; k += 8) ld8(h_fin + I * HID + k, x + k);
  for (int q = 0; q < dn; ++q) {
    float acc = w[dn * HID + q];
#pragma unroll
    for (int k = 0; k < HID; ++k) acc += w[q * HID + k] * x[k];
    o_save[I * dn + q] = acc;
    ct[ct_off + I * dn + q] = tri_diag(q, bs) ? softplus(acc) + kDiagFloor : kEpsOff * acc;
  }
}

// C values: c_val[p] = ct[map[p]] / s[row]; FP64 for the preconditioner,
// FP32 copies of C and C^T for the training products
__global__ void k_c_values(int n, const int32_t *c_rp, const int32_t *c_map, const double *s,
                           const float *ct, double *c_val, float *c_f) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double inv = 1.0 / s[r];
  for (int p = c_rp[r]; p < c_rp[r + 1]; ++p) {
    const double v = (double)ct[c_map[p]] * inv;
    c_val[p] = v;
    c_f[p] = (float)v;
  }
}

__global__ void k_gather_f(int64_t cnt, const int32_t *perm, const float *in, float *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) out[i] = in[perm[i]];
}

// ---------------------------------------------------------------------------
// loss

// Y = A X for nb interleaved columns (element (i, b) at i*nb + b)
__global__ void k_spmm(int n, int nb, const int32_t *rp, const int32_t *ci, const float *val,
                       const float *X, float *Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * nb) return;
  const int r = (int)(t / nb), b = (int)(t % nb);
  float acc = 0.f;
  for (int p = rp[r]; p < rp[r + 1]; ++p) acc += val[p] * X[(int64_t)ci[p] * nb + b];
  Y[t] = acc;
}

// R = Zh - Z (in place in Zh) and per-block column sums of R^2 and Z^2;
// block of 256 threads = 256 / nb rows x nb columns
__global__ __launch_bounds__(256) void k_loss_partials(int n, int nb, float *Zh, const float *Z,
                                                       double *part) {
  __shared__ double sr[256], sz[256];
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double r2 = 0.0, z2 = 0.0;
  if (t < (int64_t)n * nb) {
    const float r = Zh[t] - Z[t];
    Zh[t] = r;
    r2 = (double)r * r;
    z2 = (double)Z[t] * Z[t];
  }
  sr[threadIdx.x] = r2;
  sz[threadIdx.x] = z2;
  __syncthreads();
  for (int w = 128; w >= nb; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sr[threadIdx.x] += sr[threadIdx.x + w];
      sz[threadIdx.x] += sz[threadIdx.x + w];
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < nb) {
    part[(int64_t)blockIdx.x * 2 * nb + threadIdx.x] = sr[threadIdx.x];
    part[(int64_t)blockIdx.x * 2 * nb + nb + threadIdx.x] = sz[threadIdx.x];
  }
}

// loss = mean_b R2_b / Z2_b; coef_b = 2 / (nb Z2_b).  One block of 1024
// threads: 2 nb columns x (1024 / 2nb) groups, group g summing the block
// partials b = g, g + groups, ... then the groups in order (deterministic).
__global__ __launch_bounds__(1024) void k_loss_final(int nblk_, int nb, const double *part,
                                                     double *loss, float *coef) {
  __shared__ double red[1024];
  __shared__ double acc[2 * kMaxNB];
  const int w = 2 * nb, groups = 1024 / w;
  const int c = threadIdx.x % w, g = threadIdx.x / w;
  double s = 0.0;
  if (g < groups)
    for (int b = g; b < nblk_; b += groups) s += part[(int64_t)b * w + c];
  red[threadIdx.x] = s;
  __syncthreads();
  if ((int)threadIdx.x < w) {
    double tot = 0.0;
    for (int q = 0; q < groups; ++q) tot += red[q * w + threadIdx.x];
    acc[threadIdx.x] = tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double L = 0.0;
    for (int b = 0; b < nb; ++b) {
      const double z2 = acc[nb + b] > 0.0 ? acc[nb + b] : 1.0;
      L += acc[b] / z2;
      coef[b] = (float)(2.0 / (nb * z2));
    }
    *loss = L / nb;
  }
}

__global__ void k_scale_cols(int64_t cnt, int nb, const float *coef, float *G) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) G[t] *= coef[t % nb];
}

// dL/dC on C's pattern: sum_b G[r,b] U[c,b] + Y[r,b] W[c,b], then into the
// ct slot with the row scaling undone
__global__ void k_sddmm(int n, int nb, const int32_t *c_rp, const int32_t *c_ci,
                        const int32_t *c_map, const double *s, const float *Y, const float *U,
                        const float *G, const float *W, float *dct) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  float g[kMaxNB], y[kMaxNB];
  for (int b = 0; b < nb; ++b) {
    g[b] = G[(int64_t)r * nb + b];
    y[b] = Y[(int64_t)r * nb + b];
  }
  const float inv = (float)(1.0 / s[r]);
  for (int p = c_rp[r]; p < c_rp[r + 1]; ++p) {
    const int64_t c = c_ci[p];
    float acc = 0.f;
    for (int b = 0; b < nb; ++b) acc += g[b] * U[c * nb + b] + y[b] * W[c * nb + b];
    dct[c_map[p]] = acc * inv;
  }
}

// ---------------------------------------------------------------------------
// backward

__global__ void k_heads_edges_bwd(int64_t E, int de, const int32_t *src, const int32_t *dst,
                                  const float *dct, const float *W_oe, float *dE) {
  __shared__ float w[kMaxBS * kMaxBS * HID];
  for (int t = threadIdx.x; t < de * HID; t += blockDim.x) w[t] = W_oe[t];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  float out[HID];
#pragma unroll
  for (int k = 0; k < HID; ++k) out[k] = 0.f;
  if (dst[e] < src[e]) {
    for (int q = 0; q < de; ++q) {
      const float d = kEpsOff * dct[e * de + q];
#pragma unroll
      for (int k = 0; k < HID; ++k) out[k] += d * w[q * HID + k];
    }
  }
  for (int k = 0; k < HID; k += 8) st8(dE + e * HID + k, out + k);
}

__global__ void k_heads_nodes_bwd(int N, int bs, int dn, int64_t ct_off, const float *o_save,
                                  const float *dct, const float *W_od, float *dO, float *dH) {
  __shared__ float w[(kMaxBS * (kMaxBS + 1) / 2) * HID];
  for (int t = threadIdx.x; t < dn * HID; t += blockDim.x) w[t] = W_od[t];
  __syncthreads();
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= N) return;
  float out[HID];
#pragma unroll
  for (int k = 0; k < HID; ++k) out[k] = 0.f;
  for (int q = 0; q < dn; ++q) {
    const float g = dct[ct_off + I * dn + q];
    const float d = tri_diag(q, bs) ? g * sigmoid(o_save[I * dn + q]) : kEpsOff * g;
    dO[I * dn + q] = d;
#pragma unroll
    for (int k = 0; k < HID; ++k) out[k] += d * w[q * HID + k];
  }
  for (int k = 0; k < HID; k += 8) st8(dH + I * HID + k, out + k);
}

// node MLP backward: dU = dH * [rl > 0]; [dh | da] = dU W2;
// dHl = dH + dh (the residual path), da kept for the edges
__global__ __launch_bounds__(256) void k_node_bwd(int N, const float *__restrict__ dH,
                                                  const float *__restrict__ rl,
                                                  const __bf16 *__restrict__ W2,
                                                  float *__restrict__ dU,
                                                  float *__restrict__ dHl,
                                                  float *__restrict__ da) {
  const int lane = threadIdx.x & 63;
  const int64_t n0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 16;
  if (n0 >= N) return;
  const int i = lane & 15, kq = lane >> 4;
  // B[k = j][c] = W2[j][c]: lane holds j = 8 kq + q, c = 16 nt + i
  bf16x8 wb[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int q = 0; q < 8; ++q) wb[nt][q] = W2[(8 * kq + q) * 64 + 16 * nt + i];
  const int64_t I = min(n0 + i, (int64_t)N - 1);
  float g[8], r8[8];
  ld8(dH + I * HID + 8 * kq, g);
  ld8(rl + I * HID + 8 * kq, r8);
  const bool valid = n0 + i < N;
#pragma unroll
  for (int q = 0; q < 8; ++q) g[q] = (valid && r8[q] > 0.f) ? g[q] : 0.f;
  if (valid) st8(dU + I * HID + 8 * kq, g);
  const bf16x8 a = cvt8(g);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    f32x4 acc = mfma16(a, wb[nt], f32x4{0.f, 0.f, 0.f, 0.f});
    const int c = 16 * (nt & 1) + i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t nr = n0 + 4 * kq + r;
      if (nr < N) {
        if (nt < 2)
          dHl[nr * HID + c] = dH[nr * HID + c] + acc[r];
        else
          da[nr * HID + c] = acc[r];
      }
    }
  }
}

// edge MLP backward: dV = (dE + da[src]) * [m > 0]; dX = dV W1 split into
// the source part dXs, the destination part dXd and the residual edge
// path dE += dX_e (in place)
__global__ __launch_bounds__(256) void k_edge_bwd(int64_t E, const int32_t *__restrict__ src,
                                                  const float *__restrict__ m,
                                                  const float *__restrict__ da,
                                                  const __bf16 *__restrict__ W1,
                                                  float *dE, float *__restrict__ dV,
                                                  float *__restrict__ dXs,
                                                  float *__restrict__ dXd) {
  const int lane = threadIdx.x & 63;
  const int64_t e0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 16;
  if (e0 >= E) return;
  const int i = lane & 15, kq = lane >> 4;
  bf16x8 wb[6];
#pragma unroll
  for (int nt = 0; nt < 6; ++nt)
#pragma unroll
    for (int q = 0; q < 8; ++q) wb[nt][q] = W1[(8 * kq + q) * 96 + 16 * nt + i];
  const int64_t e = min(e0 + i, E - 1);
  const bool valid = e0 + i < E;
  float g[8], a8[8], m8[8];
  ld8(dE + e * HID + 8 * kq, g);
  ld8(da + (int64_t)src[e] * HID + 8 * kq, a8);
  ld8(m + e * HID + 8 * kq, m8);
#pragma unroll
  for (int q = 0; q < 8; ++q) g[q] = (valid && m8[q] > 0.f) ? g[q] + a8[q] : 0.f;
  if (valid) st8(dV + e * HID + 8 * kq, g);
  const bf16x8 a = cvt8(g);
  f32x4 acc[6];
#pragma unroll
  for (int nt = 0; nt < 6; ++nt) acc[nt] = mfma16(a, wb[nt], f32x4{0.f, 0.f, 0.f, 0.f});
  // every lane's loads of dE are complete (their values fed the MFMAs)
  // before any store below
#pragma unroll
  for (int nt = 0; nt < 6; ++nt) {
    const int c = 16 * (nt & 1) + i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t er = e0 + 4 * kq + r;
      if (er < E) {
        if (nt < 2)
          dXs[er * HID + c] = acc[nt][r];
        else if (nt < 4)
          dXd[er * HID + c] = acc[nt][r];
        else
          dE[er * HID + c] += acc[nt][r];
      }
    }
  }
}

// dHl[I] += sum over the node's edges of dXs[e] + dXd[rev[e]]
__global__ void k_node_gather(int N, const int32_t *node_ptr, const int32_t *rev,
                              const float *dXs, const float *dXd, float *dHl) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * HID) return;
  const int64_t I = t / HID;
  const int j = (int)(t % HID);
  float acc = dHl[t];
  for (int p = node_ptr[I]; p < node_ptr[I + 1]; ++p)
    acc += dXs[(int64_t)p * HID + j] + dXd[(int64_t)rev[p] * HID + j];
  dHl[t] = acc;
}

// Weight gradient of a hidden layer, dW (32 x 32NP) = sum_r dY[r]^T X[r] and
// db = sum_r dY[r], X[r] = [x0[idx0[r]]; x1[idx1[r]]; x2[r]] (NP parts, an
// index array may be NULL = identity).  MFMA with K over rows: A[j][k] =
// dY[k][j], B[k][c] = X[k][c].  One partial (32*32NP + 32 floats) per
// wavefront, summed by k_reduce_partials.
template <int NP>
__global__ __launch_bounds__(256) void k_wgrad(int64_t R, const float *__restrict__ dY,
                                               const int32_t *__restrict__ idx0,
                                               const float *__restrict__ x0,
                                               const int32_t *__restrict__ idx1,
                                               const float *__restrict__ x1,
                                               const float *__restrict__ x2,
                                               float *__restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int i = lane & 15, kq = lane >> 4;
  f32x4 acc[2][2 * NP];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2 * NP; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum[2] = {0.f, 0.f};
  const float *xs[3] = {x0, x1, x2};
  const int32_t *ix[3] = {idx0, idx1, nullptr};
  for (int64_t r0 = w * 32; r0 < R; r0 += nw * 32) {
    int64_t row[8];
    bool ok[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t rk = r0 + 8 * kq + q;
      ok[q] = rk < R;
      row[q] = ok[q] ? rk : R - 1;
    }
    bf16x8 a[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float v = ok[q] ? dY[row[q] * HID + 16 * mt + i] : 0.f;
        bsum[mt] += v;
        a[mt][q] = (__bf16)v;
      }
#pragma unroll
    for (int part_ = 0; part_ < NP; ++part_) {
      int64_t base[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        base[q] = (ix[part_] ? (int64_t)ix[part_][row[q]] : row[q]) * HID;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        bf16x8 b;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          b[q] = (__bf16)(ok[q] ? xs[part_][base[q] + 16 * half + i] : 0.f);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
          acc[mt][2 * part_ + half] = mfma16(a[mt], b, acc[mt][2 * part_ + half]);
      }
    }
  }
  const int ncol = 32 * NP;
  float *out = part + w * (32 * ncol + 32);
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2 * NP; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(16 * mt + 4 * kq + r) * ncol + 16 * nt + i] = acc[mt][nt][r];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    float s = bsum[mt];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (kq == 0) out[32 * ncol + 16 * mt + i] = s;
  }
}

// out[p][q] = sum_r a[r][p] b[r][q] (p < P, q < Q, P*Q <= 1024), plus
// (with_bias) out[P*Q + p] = sum_r a[r][p]; one partial per block
__global__ __launch_bounds__(256) void k_outer(int64_t R, int P, int Q, const float *a,
                                               const float *b, int with_bias, float *part) {
  constexpr int CH = 64;
  __shared__ float sa[CH * 32], sb[CH * 32];
  const int cnt = P * Q;
  float acc[4] = {0.f, 0.f, 0.f, 0.f}, bacc = 0.f;
  const int64_t per = (R + gridDim.x - 1) / gridDim.x;
  const int64_t r_lo = blockIdx.x * per, r_hi = min(R, r_lo + per);
  for (int64_t c0 = r_lo; c0 < r_hi; c0 += CH) {
    const int rows = (int)min((int64_t)CH, r_hi - c0);
    __syncthreads();
    for (int t = threadIdx.x; t < rows * P; t += blockDim.x) sa[t] = a[c0 * P + t];
    for (int t = threadIdx.x; t < rows * Q; t += blockDim.x) sb[t] = b[c0 * Q + t];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = threadIdx.x + 256 * u;
      if (t < cnt) {
        const int p = t / Q, q = t % Q;
        float s = 0.f;
        for (int r = 0; r < rows; ++r) s += sa[r * P + p] * sb[r * Q + q];
        acc[u] += s;
      }
    }
    if (with_bias && (int)threadIdx.x < P)
      for (int r = 0; r < rows; ++r) bacc += sa[r * P + threadIdx.x];
  }
  const int stride = cnt + (with_bias ? P : 0);
  float *out = part + (int64_t)blockIdx.x * stride;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int t = threadIdx.x + 256 * u;
    if (t < cnt) out[t] = acc[u];
  }
  if (with_bias && (int)threadIdx.x < P) out[cnt + threadIdx.x] = bacc;
}

// grad[t] = scale * sum_w part[w][t]: a block of 256 threads covers 32
// outputs with 8 groups, group g summing the partials w = g, g + 8, ... (FP64,
// fixed order, so the result is deterministic); blocks = ceil(cnt / 32)
__global__ __launch_bounds__(256) void k_reduce_partials(int nparts, int cnt, const float *part,
                                                         float scale, float *grad) {
  __shared__ double acc[8][32];
  const int j = threadIdx.x & 31, g = threadIdx.x >> 5;
  const int t = blockIdx.x * 32 + j;
  double s = 0.0;
  if (t < cnt)
    for (int w = g; w < nparts; w += 8) s += part[(int64_t)w * cnt + t];
  acc[g][j] = s;
  __syncthreads();
  if (g == 0 && t < cnt) {
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) tot += acc[q][j];
    grad[t] = (float)(scale * tot);
  }
}

__global__ void k_adam(int64_t P, const float *g, float *theta, float *m1, float *m2, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float m = b1 * m1[i] + (1.f - b1) * gi;
  const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = m;
  m2[i] = v;
  theta[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

inline unsigned nblk(int64_t work, int bsz) { return (unsigned)((work + bsz - 1) / bsz); }

}  // namespace

// ---------------------------------------------------------------------------
// handle

struct mcg_learned {
  int n = 0, N = 0, bs = 1;
  int64_t E = 0, nnzC = 0;
  Layout L{};
  // graph
  int32_t *node_ptr = nullptr, *src = nullptr, *dst = nullptr, *rev = nullptr;
  float *xn = nullptr, *fe = nullptr;
  double *s = nullptr;
  // C
  int32_t *c_rp = nullptr, *c_ci = nullptr, *c_map = nullptr;
  int32_t *t_rp = nullptr, *t_ci = nullptr, *t_perm = nullptr;
  double *c_val = nullptr;
  float *c_f = nullptr, *t_f = nullptr;
  // parameters
  float *theta = nullptr, *theta_r = nullptr, *grad = nullptr;
  __bf16 *wbf = nullptr;
  // activations
  float *h[NLAYER + 1] = {}, *e[NLAYER + 1] = {}, *m[NLAYER] = {}, *agg[NLAYER] = {},
        *rl[NLAYER] = {};
  float *ct = nullptr, *o_save = nullptr;
  // backward
  float *dct = nullptr, *dO = nullptr, *dH = nullptr, *dHl = nullptr, *dE = nullptr,
        *da = nullptr, *dU = nullptr, *dV = nullptr, *dXs = nullptr, *dXd = nullptr;
  float *part = nullptr;
  int64_t part_floats = 0;
  // loss
  float *U = nullptr, *Zh = nullptr, *G = nullptr, *W = nullptr, *coef = nullptr;
  double *lpart = nullptr, *dloss = nullptr, *hloss = nullptr;
  int nb_cap = 0;
  // timing
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  std::vector<void *> allocs;
};

namespace {

template <typename T>
int dalloc(mcg_learned *h, T **p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  if (hipMalloc((void **)p, sizeof(T) * (size_t)count) != hipSuccess) {
    (void)hipGetLastError();
    return MCG_ENOMEM;
  }
  h->allocs.push_back(*p);
  return MCG_OK;
}

#define MCG_TRY(x)                \
  do {                            \
    const int rc_ = (x);          \
    if (rc_ != MCG_OK) return rc_; \
  } while (0)

int upload(const void *host, void *dev, size_t bytes, hipStream_t s) {
  if (bytes == 0) return MCG_OK;
  if (hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return MCG_EHIP;
  return MCG_OK;
}

// Host build of the node graph, the features, C's pattern and its map.
int build_graph(mcg_learned *h, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                const std::vector<double> &va, hipStream_t st) {
  const int n = h->n, bs = h->bs, N = h->N, dn = h->L.dn, de = h->L.de;
  std::vector<double> diag(n, 0.0);
  for (int r = 0; r < n; ++r)
    for (int p = rp[r]; p < rp[r + 1]; ++p)
      if (ci[p] == r) diag[r] += va[p];
  std::vector<double> s(n);
  for (int r = 0; r < n; ++r) {
    if (!(std::fabs(diag[r]) > 0.0) || !std::isfinite(diag[r])) return MCG_EINVAL;
    s[r] = std::sqrt(std::fabs(diag[r]));
  }
  // neighbour sets
  std::vector<int32_t> node_ptr(N + 1, 0), mark(N, -1);
  std::vector<int32_t> nbr;
  nbr.reserve((size_t)rp[n] / std::max(1, bs * bs) + N);
  std::vector<int32_t> tmp;
  for (int I = 0; I < N; ++I) {
    tmp.clear();
    for (int a = 0; a < bs; ++a) {
      const int r = I * bs + a;
      for (int p = rp[r]; p < rp[r + 1]; ++p) {
        const int c = ci[p];
        if (c < 0 || c >= n) return MCG_EINVAL;
        const int J = c / bs;
        if (J != I && mark[J] != I) {
          mark[J] = I;
          tmp.push_back(J);
        }
      }
    }
    if ((int)tmp.size() > kMaxDeg) return MCG_EINVAL;
    std::sort(tmp.begin(), tmp.end());
    nbr.insert(nbr.end(), tmp.begin(), tmp.end());
    node_ptr[I + 1] = (int32_t)nbr.size();
  }
  const int64_t E = (int64_t)nbr.size();
  if (E >= ((int64_t)1 << 31) / HID) return MCG_EINVAL;
  h->E = E;
  auto find_edge = [&](int I, int J) -> int64_t {
    const auto b = nbr.begin() + node_ptr[I], en = nbr.begin() + node_ptr[I + 1];
    const auto it = std::lower_bound(b, en, J);
    return (it != en && *it == J) ? (int64_t)(it - nbr.begin()) : -1;
  };
  std::vector<int32_t> srcv(E), rev(E);
  for (int I = 0; I < N; ++I)
    for (int p = node_ptr[I]; p < node_ptr[I + 1]; ++p) {
      srcv[p] = I;
      const int64_t q = find_edge(nbr[p], I);
      if (q < 0) return MCG_EINVAL;  // pattern not symmetric
      rev[p] = (int32_t)q;
    }
  // features and C's pattern
  std::vector<float> xn((size_t)N * dn, 0.f), fe((size_t)E * de, 0.f);
  std::vector<int32_t> crp(n + 1, 0), cci, cmap;
  cci.reserve((size_t)rp[n] / 2 + n);
  cmap.reserve((size_t)rp[n] / 2 + n);
  for (int r = 0; r < n; ++r) {
    const int I = r / bs, a = r % bs;
    for (int p = rp[r]; p < rp[r + 1]; ++p) {
      const int c = ci[p], J = c / bs, b = c % bs;
      const double at = va[p] / (s[r] * s[c]);
      int64_t slot = -1;
      if (J == I) {
        if (b <= a) {
          xn[(size_t)I * dn + a * (a + 1) / 2 + b] += (float)at;
          slot = E * de + (int64_t)I * dn + a * (a + 1) / 2 + b;
        }
      } else {
        const int64_t eidx = find_edge(I, J);
        fe[(size_t)eidx * de + a * bs + b] += (float)at;
        if (J < I) slot = eidx * de + a * bs + b;
      }
      if (slot >= 0) {
        cci.push_back(c);
        cmap.push_back((int32_t)slot);
      }
    }
    crp[r + 1] = (int32_t)cci.size();
  }
  h->nnzC = (int64_t)cci.size();
  // C^T
  const int64_t nc = h->nnzC;
  std::vector<int32_t> trp(n + 1, 0), tci(nc), tperm(nc);
  for (int64_t p = 0; p < nc; ++p) ++trp[cci[p] + 1];
  for (int r = 0; r < n; ++r) trp[r + 1] += trp[r];
  {
    std::vector<int32_t> fill(trp.begin(), trp.end() - 1);
    for (int r = 0; r < n; ++r)
      for (int p = crp[r]; p < crp[r + 1]; ++p) {
        const int32_t q = fill[cci[p]]++;
        tci[q] = r;
        tperm[q] = p;
      }
  }
  MCG_TRY(dalloc(h, &h->node_ptr, N + 1));
  MCG_TRY(dalloc(h, &h->src, E));
  MCG_TRY(dalloc(h, &h->dst, E));
  MCG_TRY(dalloc(h, &h->rev, E));
  MCG_TRY(dalloc(h, &h->xn, (int64_t)N * dn));
  MCG_TRY(dalloc(h, &h->fe, E * de));
  MCG_TRY(dalloc(h, &h->s, n));
  MCG_TRY(dalloc(h, &h->c_rp, n + 1));
  MCG_TRY(dalloc(h, &h->c_ci, nc));
  MCG_TRY(dalloc(h, &h->c_map, nc));
  MCG_TRY(dalloc(h, &h->t_rp, n + 1));
  MCG_TRY(dalloc(h, &h->t_ci, nc));
  MCG_TRY(dalloc(h, &h->t_perm, nc));
  MCG_TRY(upload(node_ptr.data(), h->node_ptr, sizeof(int32_t) * (N + 1), st));
  MCG_TRY(upload(srcv.data(), h->src, sizeof(int32_t) * E, st));
  MCG_TRY(upload(nbr.data(), h->dst, sizeof(int32_t) * E, st));
  MCG_TRY(upload(rev.data(), h->rev, sizeof(int32_t) * E, st));
  MCG_TRY(upload(xn.data(), h->xn, sizeof(float) * xn.size(), st));
  MCG_TRY(upload(fe.data(), h->fe, sizeof(float) * fe.size(), st));
  MCG_TRY(upload(s.data(), h->s, sizeof(double) * n, st));
  MCG_TRY(upload(crp.data(), h->c_rp, sizeof(int32_t) * (n + 1), st));
  MCG_TRY(upload(cci.data(), h->c_ci, sizeof(int32_t) * nc, st));
  MCG_TRY(upload(cmap.data(), h->c_map, sizeof(int32_t) * nc, st));
  MCG_TRY(upload(trp.data(), h->t_rp, sizeof(int32_t) * (n + 1), st));
  MCG_TRY(upload(tci.data(), h->t_ci, sizeof(int32_t) * nc, st));
  MCG_TRY(upload(tperm.data(), h->t_perm, sizeof(int32_t) * nc, st));
  // the host vectors are freed on return: wait for the copies
  return hipStreamSynchronize(st) == hipSuccess ? MCG_OK : MCG_EHIP;
}

int alloc_network(mcg_learned *h) {
  const int64_t N = h->N, E = h->E, P = h->L.total;
  MCG_TRY(dalloc(h, &h->theta, P));
  MCG_TRY(dalloc(h, &h->theta_r, P));
  MCG_TRY(dalloc(h, &h->grad, P));
  MCG_TRY(dalloc(h, &h->wbf, (int64_t)NLAYER * HID * 5 * HID));
  for (int l = 0; l <= NLAYER; ++l) {
    MCG_TRY(dalloc(h, &h->h[l], N * HID));
    MCG_TRY(dalloc(h, &h->e[l], E * HID));
  }
  for (int l = 0; l < NLAYER; ++l) {
    MCG_TRY(dalloc(h, &h->m[l], E * HID));
    MCG_TRY(dalloc(h, &h->agg[l], N * HID));
    MCG_TRY(dalloc(h, &h->rl[l], N * HID));
  }
  const int64_t nct = E * h->L.de + N * h->L.dn;
  MCG_TRY(dalloc(h, &h->ct, nct));
  MCG_TRY(dalloc(h, &h->o_save, N * h->L.dn));
  MCG_TRY(dalloc(h, &h->c_val, h->nnzC));
  MCG_TRY(dalloc(h, &h->c_f, h->nnzC));
  MCG_TRY(dalloc(h, &h->t_f, h->nnzC));
  return MCG_OK;
}

int alloc_backward(mcg_learned *h, int nb) {
  const int64_t N = h->N, E = h->E, n = h->n;
  if (!h->dct) {
    const int64_t nct = E * h->L.de + N * h->L.dn;
    MCG_TRY(dalloc(h, &h->dct, nct));
    MCG_TRY(dalloc(h, &h->dO, N * h->L.dn));
    MCG_TRY(dalloc(h, &h->dH, N * HID));
    MCG_TRY(dalloc(h, &h->dHl, N * HID));
    MCG_TRY(dalloc(h, &h->da, N * HID));
    MCG_TRY(dalloc(h, &h->dU, N * HID));
    MCG_TRY(dalloc(h, &h->dE, E * HID));
    MCG_TRY(dalloc(h, &h->dV, E * HID));
    MCG_TRY(dalloc(h, &h->dXs, E * HID));
    MCG_TRY(dalloc(h, &h->dXd, E * HID));
    h->part_floats = std::max<int64_t>((int64_t)kWgradWaves * (32 * 96 + 32),
                                       (int64_t)kOuterBlocks * (HID * 16 + 16));
    MCG_TRY(dalloc(h, &h->part, h->part_floats));
    MCG_TRY(dalloc(h, &h->dloss, 1));
    MCG_TRY(dalloc(h, &h->coef, kMaxNB));
    if (hipHostMalloc((void **)&h->hloss, sizeof(double)) != hipSuccess) return MCG_ENOMEM;
  }
  if (nb > h->nb_cap) {
    // loss buffers are replaced, not freed, when nb grows (they stay owned
    // by the handle until mcg_learned_free)
    MCG_TRY(dalloc(h, &h->U, n * nb));
    MCG_TRY(dalloc(h, &h->Zh, n * nb));
    MCG_TRY(dalloc(h, &h->G, n * nb));
    MCG_TRY(dalloc(h, &h->W, n * nb));
    MCG_TRY(dalloc(h, &h->lpart, (int64_t)nblk(n * nb, 256) * 2 * nb));
    h->nb_cap = nb;
  }
  return MCG_OK;
}

int forward_impl(mcg_learned *h, hipStream_t st) {
  const Layout &L = h->L;
  const int64_t N = h->N, E = h->E, P = L.total;
  k_round_params<<<nblk(P, 256), 256, 0, st>>>(P, h->theta, h->theta_r, h->wbf, L.layer0,
                                               L.layer_stride);
  const float *tr = h->theta_r;
  if (hipEventRecord(h->ev0, st) != hipSuccess) return MCG_EHIP;
  k_embed<<<nblk(N * HID, 256), 256, 0, st>>>(N, L.dn, h->xn, tr + L.win_n, h->h[0]);
  if (E > 0) k_embed<<<nblk(E * HID, 256), 256, 0, st>>>(E, L.de, h->fe, tr + L.win_e, h->e[0]);
  for (int l = 0; l < NLAYER; ++l) {
    const __bf16 *w1 = h->wbf + (int64_t)l * HID * 5 * HID;
    const __bf16 *w2 = w1 + HID * 3 * HID;
    if (E > 0)
      k_edge_fwd<<<nblk(E, 64), 256, 0, st>>>(E, h->src, h->dst, h->h[l], h->e[l], w1,
                                              tr + L.b1(l), h->m[l], h->e[l + 1]);
    k_node_fwd<<<nblk(N, 64), 256, 0, st>>>((int)N, h->node_ptr, h->h[l], h->m[l], w2,
                                            tr + L.b2(l), h->agg[l], h->rl[l], h->h[l + 1]);
  }
  if (hipEventRecord(h->ev1, st) != hipSuccess) return MCG_EHIP;
  h->timed = true;
  if (E > 0)
    k_heads_edges<<<nblk(E, 256), 256, 0, st>>>(E, L.de, h->src, h->dst, h->e[NLAYER],
                                                tr + L.w_oe, h->ct);
  k_heads_nodes<<<nblk(N, 256), 256, 0, st>>>((int)N, h->bs, L.dn, E * L.de, h->h[NLAYER],
                                              tr + L.w_od, tr + L.b_od, h->o_save, h->ct);
  k_c_values<<<nblk(h->n, 256), 256, 0, st>>>(h->n, h->c_rp, h->c_map, h->s, h->ct, h->c_val,
                                              h->c_f);
  k_gather_f<<<nblk(h->nnzC, 256), 256, 0, st>>>(h->nnzC, h->t_perm, h->c_f, h->t_f);
  return hipGetLastError() == hipSuccess ? MCG_OK : MCG_EHIP;
}

// grad[off .. off + cnt) from the partials of k_outer
void outer_grad(mcg_learned *h, int64_t R, int P, int Q, const float *a, const float *b,
                int with_bias, float scale, int64_t off, hipStream_t st) {
  const int cnt = P * Q + (with_bias ? P : 0);
  if (R <= 0) {
    k_reduce_partials<<<nblk(cnt, 32), 256, 0, st>>>(0, cnt, h->part, scale, h->grad + off);
    return;
  }
  k_outer<<<kOuterBlocks, 256, 0, st>>>(R, P, Q, a, b, with_bias, h->part);
  k_reduce_partials<<<nblk(cnt, 32), 256, 0, st>>>(kOuterBlocks, cnt, h->part, scale,
                                                   h->grad + off);
}

template <int NP>
void wgrad(mcg_learned *h, int64_t R, const float *dY, const int32_t *i0, const float *x0,
           const int32_t *i1, const float *x1, const float *x2, int64_t off, hipStream_t st) {
  const int cnt = 32 * 32 * NP + 32;
  if (R > 0) {
    k_wgrad<NP><<<kWgradWaves / 4, 256, 0, st>>>(R, dY, i0, x0, i1, x1, x2, h->part);
    k_reduce_partials<<<nblk(cnt, 32), 256, 0, st>>>(kWgradWaves, cnt, h->part, 1.f,
                                                     h->grad + off);
  } else {
    k_reduce_partials<<<nblk(cnt, 32), 256, 0, st>>>(0, cnt, h->part, 1.f, h->grad + off);
  }
}

int backward_impl(mcg_learned *h, const float *Y, const float *Z, int nb, hipStream_t st) {
  const Layout &L = h->L;
  const int n = h->n;
  const int64_t N = h->N, E = h->E, nnb = (int64_t)n * nb;
  const float *tr = h->theta_r;
  // loss: U = C^T Y, Zh = C U, R = Zh - Z, G = coef R, W = C^T G
  k_spmm<<<nblk(nnb, 256), 256, 0, st>>>(n, nb, h->t_rp, h->t_ci, h->t_f, Y, h->U);
  k_spmm<<<nblk(nnb, 256), 256, 0, st>>>(n, nb, h->c_rp, h->c_ci, h->c_f, h->U, h->Zh);
  const unsigned lb = nblk(nnb, 256);
  k_loss_partials<<<lb, 256, 0, st>>>(n, nb, h->Zh, Z, h->lpart);
  k_loss_final<<<1, 1024, 0, st>>>((int)lb, nb, h->lpart, h->dloss, h->coef);
  k_scale_cols<<<nblk(nnb, 256), 256, 0, st>>>(nnb, nb, h->coef, h->Zh);
  float *G = h->Zh;
  k_spmm<<<nblk(nnb, 256), 256, 0, st>>>(n, nb, h->t_rp, h->t_ci, h->t_f, G, h->W);
  const int64_t nct = E * L.de + N * L.dn;
  k_fill<float><<<nblk(nct, 256), 256, 0, st>>>(nct, 0.f, h->dct);
  k_sddmm<<<nblk(n, 256), 256, 0, st>>>(n, nb, h->c_rp, h->c_ci, h->c_map, h->s, Y, h->U, G,
                                        h->W, h->dct);
  // heads
  if (E > 0)
    k_heads_edges_bwd<<<nblk(E, 256), 256, 0, st>>>(E, L.de, h->src, h->dst, h->dct,
                                                    tr + L.w_oe, h->dE);
  k_heads_nodes_bwd<<<nblk(N, 256), 256, 0, st>>>((int)N, h->bs, L.dn, E * L.de, h->o_save,
                                                  h->dct, tr + L.w_od, h->dO, h->dH);
  outer_grad(h, E, L.de, HID, h->dct, h->e[NLAYER], 0, kEpsOff, L.w_oe, st);
  outer_grad(h, N, L.dn, HID, h->dO, h->h[NLAYER], 1, 1.f, L.w_od, st);
  // layers, last to first; dH holds dL/dh_{l+1}, dE holds dL/de_{l+1}
  for (int l = NLAYER - 1; l >= 0; --l) {
    const __bf16 *w1 = h->wbf + (int64_t)l * HID * 5 * HID;
    const __bf16 *w2 = w1 + HID * 3 * HID;
    k_node_bwd<<<nblk(N, 64), 256, 0, st>>>((int)N, h->dH, h->rl[l], w2, h->dU, h->dHl, h->da);
    if (E > 0) {
      k_edge_bwd<<<nblk(E, 64), 256, 0, st>>>(E, h->src, h->m[l], h->da, w1, h->dE, h->dV,
                                              h->dXs, h->dXd);
      k_node_gather<<<nblk(N * HID, 256), 256, 0, st>>>((int)N, h->node_ptr, h->rev, h->dXs,
                                                        h->dXd, h->dHl);
    }
    wgrad<3>(h, E, h->dV, h->src, h->h[l], h->dst, h->h[l], h->e[l], L.w1(l), st);
    wgrad<2>(h, N, h->dU, nullptr, h->h[l], nullptr, h->agg[l], nullptr, L.w2(l), st);
    std::swap(h->dH, h->dHl);
  }
  // input embeddings: dW_in_n = dh0^T xn, dW_in_e = de0^T fe
  outer_grad(h, N, HID, L.dn, h->dH, h->xn, 0, 1.f, L.win_n, st);
  outer_grad(h, E, HID, L.de, h->dE, h->fe, 0, 1.f, L.win_e, st);
  return hipGetLastError() == hipSuccess ? MCG_OK : MCG_EHIP;
}

}  // namespace

extern "C" {

int mcg_learned_create(mcg_learned_t *out, const mcg_csr_t *A, int32_t block_size, void *stream) {
  if (!out) return MCG_EINVAL;
  *out = nullptr;
  if (!A || !A->row_ptr || !A->col || !A->val || A->n <= 0 || A->nnz <= 0) return MCG_EINVAL;
  if (block_size < 1 || block_size > kMaxBS || A->n % block_size != 0) return MCG_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int n = A->n;
  std::vector<int32_t> rp(n + 1), ci(A->nnz);
  std::vector<double> va(A->nnz);
  if (hipMemcpyAsync(rp.data(), A->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost,
                     st) != hipSuccess ||
      hipMemcpyAsync(ci.data(), A->col, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipMemcpyAsync(va.data(), A->val, sizeof(double) * A->nnz, hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return MCG_EHIP;
  if (rp[0] != 0 || rp[n] != A->nnz) return MCG_EINVAL;
  for (int r = 0; r < n; ++r)
    if (rp[r + 1] < rp[r]) return MCG_EINVAL;
  auto *h = new mcg_learned();
  h->n = n;
  h->bs = block_size;
  h->N = n / block_size;
  h->L = make_layout(block_size);
  int rc = build_graph(h, rp, ci, va, st);
  if (rc == MCG_OK) rc = alloc_network(h);
  if (rc == MCG_OK && (hipEventCreate(&h->ev0) != hipSuccess ||
                       hipEventCreate(&h->ev1) != hipSuccess))
    rc = MCG_EHIP;
  if (rc == MCG_OK) {
    k_fill<float><<<nblk(h->L.total, 256), 256, 0, st>>>(h->L.total, 0.f, h->theta);
    if (hipGetLastError() != hipSuccess) rc = MCG_EHIP;
  }
  if (rc != MCG_OK) {
    mcg_learned_free(h);
    return rc;
  }
  *out = h;
  return MCG_OK;
}

void mcg_learned_free(mcg_learned_t h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  for (void *p : h->allocs) (void)hipFree(p);
  if (h->hloss) (void)hipHostFree(h->hloss);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  delete h;
}

int64_t mcg_learned_num_params(mcg_learned_t h) { return h ? h->L.total : -1; }

int mcg_learned_sizes(mcg_learned_t h, int64_t *nodes, int64_t *edges, int64_t *nnz_c) {
  if (!h) return MCG_EINVAL;
  if (nodes) *nodes = h->N;
  if (edges) *edges = h->E;
  if (nnz_c) *nnz_c = h->nnzC;
  return MCG_OK;
}

int mcg_learned_set_params(mcg_learned_t h, const float *theta, void *stream) {
  if (!h || !theta) return MCG_EINVAL;
  return hipMemcpyAsync(h->theta, theta, sizeof(float) * h->L.total, hipMemcpyDeviceToDevice,
                        (hipStream_t)stream) == hipSuccess
             ? MCG_OK
             : MCG_EHIP;
}

int mcg_learned_get_params(mcg_learned_t h, float *theta, void *stream) {
  if (!h || !theta) return MCG_EINVAL;
  return hipMemcpyAsync(theta, h->theta, sizeof(float) * h->L.total, hipMemcpyDeviceToDevice,
                        (hipStream_t)stream) == hipSuccess
             ? MCG_OK
             : MCG_EHIP;
}

int mcg_learned_forward(mcg_learned_t h, void *stream) {
  if (!h) return MCG_EINVAL;
  return forward_impl(h, (hipStream_t)stream);
}

int mcg_learned_factor(mcg_learned_t h, mcg_csr_t *C) {
  if (!h || !C) return MCG_EINVAL;
  C->n = h->n;
  C->nnz = h->nnzC;
  C->row_ptr = h->c_rp;
  C->col = h->c_ci;
  C->val = h->c_val;
  return MCG_OK;
}

int mcg_learned_factor_copy(mcg_learned_t h, int32_t *row_ptr, int32_t *col, double *val,
                            void *stream) {
  if (!h || !row_ptr || !col || !val) return MCG_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(row_ptr, h->c_rp, sizeof(int32_t) * (h->n + 1), hipMemcpyDeviceToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(col, h->c_ci, sizeof(int32_t) * h->nnzC, hipMemcpyDeviceToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(val, h->c_val, sizeof(double) * h->nnzC, hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
    return MCG_EHIP;
  return MCG_OK;
}

int mcg_learned_loss_grad(mcg_learned_t h, const float *Y, const float *Z, int32_t nb,
                          double *loss, float *grad, void *stream) {
  if (!h || !Y || !Z || nb < 1 || nb > kMaxNB || (nb & (nb - 1))) return MCG_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  MCG_TRY(alloc_backward(h, nb));
  MCG_TRY(forward_impl(h, st));
  MCG_TRY(backward_impl(h, Y, Z, nb, st));
  if (grad && hipMemcpyAsync(grad, h->grad, sizeof(float) * h->L.total, hipMemcpyDeviceToDevice,
                             st) != hipSuccess)
    return MCG_EHIP;
  if (loss) {
    if (hipMemcpyAsync(h->hloss, h->dloss, sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return MCG_EHIP;
    *loss = *h->hloss;
  }
  return MCG_OK;
}

int mcg_learned_adam(int64_t P, float *theta, const float *grad, float *m1, float *m2, float lr,
                     float beta1, float beta2, float eps, int32_t step, void *stream) {
  if (P <= 0 || !theta || !grad || !m1 || !m2 || step < 1 || !(lr > 0.f) ||
      !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return MCG_EINVAL;
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  k_adam<<<nblk(P, 256), 256, 0, (hipStream_t)stream>>>(P, grad, theta, m1, m2, lr, beta1, beta2,
                                                        eps, c1, c2);
  return hipGetLastError() == hipSuccess ? MCG_OK : MCG_EHIP;
}

double mcg_learned_forward_ms(mcg_learned_t h) {
  if (!h || !h->timed) return -1.0;
  float ms = 0.f;
  if (hipEventSynchronize(h->ev1) != hipSuccess ||
      hipEventElapsedTime(&ms, h->ev0, h->ev1) != hipSuccess)
    return -1.0;
  return ms;
}

}  // extern "C"
