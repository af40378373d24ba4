/*
 * Plain FP64 CPU oracle of the two-level nested MINRES-CG scheme
 * (Manguoglu & Mehrmann, "A robust iterative scheme for symmetric indefinite
 * systems", Section 2, Algorithm "minres_cg").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the
 * HIP implementation: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code with the GPU library.
 *
 * Everything is written for readability: one loop per mathematical step, in
 * the order the method states them, FP64 throughout.  OpenMP only splits the
 * row loops (SpMV, dot products, axpy) across host cores.
 *
 * Notation (Section 2):
 *   A        sparse symmetric indefinite, CSR (row_ptr, col, val), full pattern
 *   Vhat     n x k, column-major, approximate invariant subspace of the k
 *            negative eigenvalues; lam[k] < 0 the eigenvalues (Lambda_hat)
 *   M_mr     = A + 2 Vhat |Lambda_hat| Vhat^T            (first level)
 *   M_cg     approximation of A used inside CG           (second level)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* status codes (mirrored by the tests) */
#define ORC_OK 0
#define ORC_MAXIT 1
#define ORC_STAGNATION 2
#define ORC_BREAKDOWN 3
#define ORC_NOT_SPD 4
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-3)

/* inner (CG) preconditioner kinds */
#define ORC_PC_NONE 0    /* t = g                                   */
#define ORC_PC_JACOBI 1  /* t = g ./ diag(A)                        */
#define ORC_PC_ILDL0 2   /* t = (L D L^T)^{-1} g, incomplete LDL^T(0) */
#define ORC_PC_DENSE 3   /* t = Minv g, dense (tiny pin tests only)  */
#define ORC_PC_CCT 4     /* t = C (C^T g), C lower triangular CSR    */
#define ORC_PC_ILDLP 5   /* t = (P^T L D L^T P)^{-1} g, pivoted ILDL^T(fill, drop) */

/* outer (MINRES) preconditioner kinds */
#define ORC_OUT_PCG 0    /* y = approximate M_mr^{-1} r by inner PCG (the method) */
#define ORC_OUT_DENSE 1  /* y = Minv r, dense (tiny pin tests only)               */
#define ORC_OUT_NONE 2   /* y = r (plain MINRES)                                  */

/* ------------------------------------------------------------------------ */
/* BLAS-1 / SpMV building blocks                                             */
/* ------------------------------------------------------------------------ */

static double dot(int64_t n, const double *x, const double *y) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
  return s;
}

static double nrm2(int64_t n, const double *x) { return sqrt(dot(n, x, x)); }

/* y = A x */
void orc_spmv(int32_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
              const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) s += val[p] * x[col[p]];
    y[i] = s;
  }
}

/* q = M_mr u = A u + 2 Vhat (|Lambda_hat| (Vhat^T u))   (Section 2, the
 * matrix-vector procedure following Algorithm "minres_cg": one SpMV, one
 * tall-skinny Vhat^T u, one rank-k update).  |lam_j| = -lam_j since lam < 0. */
void orc_mmr_apply(int32_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                   int32_t k, const double *Vhat, const double *lam, const double *u,
                   double *q) {
  orc_spmv(n, row_ptr, col, val, u, q);
  if (k <= 0) return;
  double *s = (double *)malloc(sizeof(double) * (size_t)k);
  for (int32_t j = 0; j < k; ++j) s[j] = dot(n, Vhat + (int64_t)j * n, u); /* Vhat^T u */
  for (int32_t j = 0; j < k; ++j) s[j] *= 2.0 * fabs(lam[j]);              /* 2|Lambda| */
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int32_t j = 0; j < k; ++j) acc += Vhat[(int64_t)j * n + i] * s[j];
    q[i] += acc;
  }
  free(s);
}

/* ------------------------------------------------------------------------ */
/* Incomplete LDL^T(0): the symmetric form of the ILU(0) of A used as M_cg   */
/* (Section 4: ILU(0) of the coefficient matrix as the inner preconditioner).*/
/* L is unit lower triangular on the strictly-lower pattern of A, D diagonal */
/* and may be indefinite.  Row (up-looking) form:                            */
/*   l_ij d_j = a_ij - sum_{m<j, m in pat(i) and pat(j)} l_im d_m l_jm       */
/*   d_i      = a_ii - sum_{m<i, m in pat(i)} l_im^2 d_m                     */
/* A pivot with |d_i| < pivtol*max_j|a_ij| is replaced by sign(d_i) times   */
/* that floor (a zero pivot made the paper switch to MILU for one matrix;    */
/* this keeps L D L^T regular instead).                                      */
/* Output: lower CSR (l_ptr, l_col, l_val) of the strictly lower part, d[n]. */
/* l_ptr/l_col/l_val must hold n+1 / nnz_lower / nnz_lower entries.          */
/* Returns the number of modified pivots, or ORC_EINVAL.                     */
/* ------------------------------------------------------------------------ */
int64_t orc_ildl0_nnz_lower(int32_t n, const int32_t *row_ptr, const int32_t *col) {
  int64_t c = 0;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
      if (col[p] < i) ++c;
  return c;
}

int32_t orc_ildl0_factor(int32_t n, const int32_t *row_ptr, const int32_t *col,
                         const double *val, double pivtol, int32_t *l_ptr, int32_t *l_col,
                         double *l_val, double *d) {
  /* pattern of L = strictly lower part of A */
  int64_t c = 0;
  l_ptr[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
      if (col[p] < i) { l_col[c] = col[p]; l_val[c] = val[p]; ++c; }
    l_ptr[i + 1] = (int32_t)c;
  }
  /* position of column m inside the current row i (or -1) */
  int64_t *where = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!where) return ORC_ENOMEM;
  for (int32_t i = 0; i < n; ++i) where[i] = -1;
  int32_t modified = 0;
  for (int32_t i = 0; i < n; ++i) {
    double aii = 0.0, rowmax = 0.0;
    int found = 0;
    for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      if (col[p] == i) { aii = val[p]; found = 1; }
      if (fabs(val[p]) > rowmax) rowmax = fabs(val[p]);
    }
    if (!found) { free(where); return ORC_EINVAL; }
    for (int32_t p = l_ptr[i]; p < l_ptr[i + 1]; ++p) where[l_col[p]] = p;
    /* l_ij for j in pat(i), increasing j (columns are sorted) */
    for (int32_t p = l_ptr[i]; p < l_ptr[i + 1]; ++p) {
      int32_t j = l_col[p];
      double s = l_val[p]; /* a_ij */
      for (int32_t q = l_ptr[j]; q < l_ptr[j + 1]; ++q) {
        int32_t m = l_col[q];          /* m < j, m in pat(j) */
        int64_t pim = where[m];
        if (pim >= 0) s -= l_val[pim] * d[m] * l_val[q]; /* m in pat(i) too */
      }
      l_val[p] = s / d[j];
    }
    double di = aii;
    for (int32_t p = l_ptr[i]; p < l_ptr[i + 1]; ++p) di -= l_val[p] * l_val[p] * d[l_col[p]];
    double floor_ = pivtol * rowmax;
    if (fabs(di) < floor_) { di = (di < 0.0 ? -floor_ : floor_); ++modified; }
    d[i] = di;
    for (int32_t p = l_ptr[i]; p < l_ptr[i + 1]; ++p) where[l_col[p]] = -1;
  }
  free(where);
  return modified;
}

/* t = (L D L^T)^{-1} g by forward substitution, diagonal scaling and
 * backward substitution in natural order. */
void orc_ildl0_solve(int32_t n, const int32_t *l_ptr, const int32_t *l_col, const double *l_val,
                     const double *d, const double *g, double *t) {
  for (int32_t i = 0; i < n; ++i) { /* L u = g */
    double s = g[i];
    for (int32_t p = l_ptr[i]; p < l_ptr[i + 1]; ++p) s -= l_val[p] * t[l_col[p]];
    t[i] = s;
  }
  for (int32_t i = 0; i < n; ++i) t[i] /= d[i]; /* D w = u */
  for (int32_t i = n - 1; i >= 0; --i) {       /* L^T t = w (column sweep) */
    double ti = t[i];
    for (int32_t p = l_ptr[i]; p < l_ptr[i + 1]; ++p) t[l_col[p]] -= l_val[p] * ti;
  }
}

/* ------------------------------------------------------------------------ */
/* Incomplete LDL^T with symmetric pivoting, fill factor and drop tolerance  */
/* (the robust second-level preconditioner of Section 4, "ILDL^T(fill,       */
/* drop)": an incomplete Bunch-Parlett-type factorization P A P^T ~ L D L^T  */
/* with 1x1 and 2x2 pivots).  Column by column (left-looking), k = 0..n-1:   */
/*  1. w = column c = perm[k] of the current Schur complement: A's column c  */
/*     restricted to the not yet pivoted rows, minus the contributions of    */
/*     the finished columns j with L(c, j) != 0 (2x2 blocks as blocks);      */
/*  2. Bunch-Kaufman choice (alpha = (1 + sqrt 17)/8) between a 1x1 pivot at */
/*     c, a 1x1 pivot at the row r of the largest off-diagonal |w_r|, or a   */
/*     2x2 pivot (c, r) -- the latter two need column r of the Schur         */
/*     complement, built the same way; r moves to position k (1x1) or k+1;  */
/*  3. the new column(s) of L = w / d (w D^-1 for a 2x2 pivot);              */
/*  4. dropping, per column: entries with |l| < drop * ||l||_2 go; of the    */
/*     rest only the fill * m largest stay (m = A's off-diagonal entries in  */
/*     column c in rows not yet pivoted; fill <= 0: no limit), ties broken  */
/*     by the smaller original row index.                                    */
/* L's rows are kept by ORIGINAL index while the factorization runs, so a    */
/* symmetric interchange only swaps two entries of perm.  A 1x1 pivot with   */
/* |d| < 1e-8 max|A| becomes sign(d) times that floor.  With fill >= n and   */
/* drop = 0 nothing is dropped and the factorization is exact.               */
/* Result: perm (logical -> original), L strictly lower in logical CSR,      */
/* D as dd[k] (diagonal) and doff[k] = D(k, k+1) where k starts a 2x2 block, */
/* bsize[k] = 1, 2 (first of a 2x2 block) or 0 (its second row).           */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t n;
  int32_t *perm, *bsize;
  double *dd, *doff;
  int32_t *l_ptr, *l_col;
  double *l_val;
  int64_t nnz_l;
} orc_ildlp;

typedef struct { int32_t idx; double val; } orc_ent;        /* (index, value) */
typedef struct { orc_ent *e; int64_t n, cap; } orc_vec;

static int vec_push(orc_vec *v, int32_t idx, double val) {
  if (v->n == v->cap) {
    int64_t nc = v->cap ? 2 * v->cap : 8;
    orc_ent *ne = (orc_ent *)realloc(v->e, sizeof(orc_ent) * (size_t)nc);
    if (!ne) return -1;
    v->e = ne; v->cap = nc;
  }
  v->e[v->n].idx = idx; v->e[v->n].val = val; v->n++;
  return 0;
}

/* sort key of the fill rule: |value| descending, then original index ascending */
static int cmp_keep(const void *a, const void *b) {
  const orc_ent *x = (const orc_ent *)a, *y = (const orc_ent *)b;
  double ax = fabs(x->val), ay = fabs(y->val);
  if (ax > ay) return -1;
  if (ax < ay) return 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

typedef struct {
  int32_t n;
  const int32_t *rp, *ci;
  const double *va;
  int32_t *pivoted, *iperm;
  orc_vec *col;      /* L column j: (original row, value)  */
  orc_vec *row;      /* row by original index: (column j, value) */
  int32_t *bsize;
  double *dd, *doff;
} ildlp_state;

/* w (dense, by original index, zero outside `touched`) = Schur column of the
 * original index c over the rows not yet pivoted; returns the touched count. */
static int32_t schur_column(const ildlp_state *S, int32_t c, double *w, int32_t *touched,
                            char *mark) {
  int32_t nt = 0;
  for (int32_t p = S->rp[c]; p < S->rp[c + 1]; ++p) {
    int32_t o = S->ci[p];
    if (S->pivoted[o]) continue;
    if (!mark[o]) { mark[o] = 1; touched[nt++] = o; w[o] = 0.0; }
    w[o] += S->va[p];
  }
  const orc_vec *rw = &S->row[c];
  for (int64_t q = 0; q < rw->n; ++q) {
    int32_t j = rw->e[q].idx;
    if (S->bsize[j] == 1) {
      double coef = S->dd[j] * rw->e[q].val;
      const orc_vec *cj = &S->col[j];
      for (int64_t t = 0; t < cj->n; ++t) {
        int32_t o = cj->e[t].idx;
        if (S->pivoted[o]) continue;
        if (!mark[o]) { mark[o] = 1; touched[nt++] = o; w[o] = 0.0; }
        w[o] -= cj->e[t].val * coef;
      }
    } else {
      /* 2x2 block (s, s + 1): handled once, at its first entry in the row */
      int32_t s = S->bsize[j] == 2 ? j : j - 1;
      if (j == s + 1 && q > 0 && rw->e[q - 1].idx == s) continue;
      double a = 0.0, b = 0.0;
      if (j == s) {
        a = rw->e[q].val;
        if (q + 1 < rw->n && rw->e[q + 1].idx == s + 1) b = rw->e[q + 1].val;
      } else {
        b = rw->e[q].val;
      }
      double u1 = S->dd[s] * a + S->doff[s] * b;
      double u2 = S->doff[s] * a + S->dd[s + 1] * b;
      for (int32_t h = 0; h < 2; ++h) {
        const orc_vec *cj = &S->col[s + h];
        double coef = h == 0 ? u1 : u2;
        for (int64_t t = 0; t < cj->n; ++t) {
          int32_t o = cj->e[t].idx;
          if (S->pivoted[o]) continue;
          if (!mark[o]) { mark[o] = 1; touched[nt++] = o; w[o] = 0.0; }
          w[o] -= cj->e[t].val * coef;
        }
      }
    }
  }
  return nt;
}

/* number of off-diagonal entries of A's column c in rows not yet pivoted */
static int32_t unpivoted_count(const ildlp_state *S, int32_t c) {
  int32_t m = 0;
  for (int32_t p = S->rp[c]; p < S->rp[c + 1]; ++p)
    if (S->ci[p] != c && !S->pivoted[S->ci[p]]) ++m;
  return m;
}

/* drop + fill rule on the candidate entries of one new column k of L; the
 * kept ones are stored in col[k] and appended to the rows */
static int store_column(ildlp_state *S, int32_t k, orc_ent *cand, int32_t nc, double fill,
                        double drop, int32_t m_a) {
  double nrm = 0.0;
  for (int32_t i = 0; i < nc; ++i) nrm += cand[i].val * cand[i].val;
  nrm = sqrt(nrm);
  int32_t nk = 0;
  for (int32_t i = 0; i < nc; ++i)
    if (cand[i].val != 0.0 && fabs(cand[i].val) >= drop * nrm) cand[nk++] = cand[i];
  if (fill > 0.0) {
    int32_t lim = (int32_t)ceil(fill * (double)m_a);
    if (lim < 1) lim = 1;
    if (nk > lim) {
      qsort(cand, (size_t)nk, sizeof(orc_ent), cmp_keep);
      nk = lim;
    }
  }
  for (int32_t i = 0; i < nk; ++i) {
    if (vec_push(&S->col[k], cand[i].idx, cand[i].val)) return -1;
    if (vec_push(&S->row[cand[i].idx], k, cand[i].val)) return -1;
  }
  return 0;
}

static void swap_pos(ildlp_state *S, int32_t *perm, int32_t p, int32_t q) {
  if (p == q) return;
  int32_t a = perm[p], b = perm[q];
  perm[p] = b; perm[q] = a;
  S->iperm[b] = p; S->iperm[a] = q;
}

void orc_ildlp_free(orc_ildlp *F) {
  if (!F) return;
  free(F->perm); free(F->bsize); free(F->dd); free(F->doff);
  free(F->l_ptr); free(F->l_col); free(F->l_val);
  free(F);
}

orc_ildlp *orc_ildlp_factor(int32_t n, const int32_t *rp, const int32_t *ci, const double *va,
                            double fill, double drop) {
  const double alpha = (1.0 + sqrt(17.0)) / 8.0;
  orc_ildlp *F = (orc_ildlp *)calloc(1, sizeof(orc_ildlp));
  ildlp_state S;
  memset(&S, 0, sizeof(S));
  S.n = n; S.rp = rp; S.ci = ci; S.va = va;
  F->n = n;
  F->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  F->bsize = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  F->dd = (double *)calloc((size_t)n, sizeof(double));
  F->doff = (double *)calloc((size_t)n, sizeof(double));
  S.pivoted = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  S.iperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  S.col = (orc_vec *)calloc((size_t)n, sizeof(orc_vec));
  S.row = (orc_vec *)calloc((size_t)n, sizeof(orc_vec));
  S.bsize = F->bsize; S.dd = F->dd; S.doff = F->doff;
  double *w1 = (double *)calloc((size_t)n, sizeof(double));
  double *w2 = (double *)calloc((size_t)n, sizeof(double));
  int32_t *t1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *t2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  char *m1 = (char *)calloc((size_t)n, 1), *m2 = (char *)calloc((size_t)n, 1);
  orc_ent *cand = (orc_ent *)malloc(sizeof(orc_ent) * (size_t)(2 * n + 2));
  int failed = 0;
  double amax = 0.0;
  for (int64_t p = 0; p < (n > 0 ? rp[n] : 0); ++p) if (fabs(va[p]) > amax) amax = fabs(va[p]);
  const double floor_ = 1e-8 * amax;
  for (int32_t i = 0; i < n; ++i) { F->perm[i] = i; S.iperm[i] = i; }
  int32_t k = 0;
  while (k < n && !failed) {
    int32_t c = F->perm[k];
    int32_t nt1 = schur_column(&S, c, w1, t1, m1);
    double absakk = m1[c] ? fabs(w1[c]) : 0.0;
    double colmax = 0.0;
    int32_t r = -1;
    for (int32_t i = 0; i < nt1; ++i) {
      int32_t o = t1[i];
      if (o == c) continue;
      double v = fabs(w1[o]);
      if (v > colmax || (v == colmax && v > 0.0 && S.iperm[o] < S.iperm[r])) { colmax = v; r = o; }
    }
    int two = 0, piv = c; /* pivot original index (1x1) */
    int32_t nt2 = 0;
    if (colmax > 0.0 && !(absakk >= alpha * colmax)) {
      nt2 = schur_column(&S, r, w2, t2, m2);
      double rowmax = 0.0;
      for (int32_t i = 0; i < nt2; ++i) {
        int32_t o = t2[i];
        if (o == r) continue;
        if (fabs(w2[o]) > rowmax) rowmax = fabs(w2[o]);
      }
      double arr = m2[r] ? fabs(w2[r]) : 0.0;
      if (absakk * rowmax >= alpha * colmax * colmax) {
        piv = c;
      } else if (arr >= alpha * rowmax) {
        piv = r;
      } else {
        two = 1;
      }
    }
    if (!two) {
      const double *w = (piv == c) ? w1 : w2;
      const int32_t *tt = (piv == c) ? t1 : t2;
      int32_t nt = (piv == c) ? nt1 : nt2;
      swap_pos(&S, F->perm, k, S.iperm[piv]);
      double d = w[piv];
      if ((piv == c ? m1[piv] : m2[piv]) == 0) d = 0.0;
      if (fabs(d) < floor_) d = (d < 0.0 ? -floor_ : floor_);
      int32_t m_a = unpivoted_count(&S, piv);
      S.pivoted[piv] = 1;
      int32_t nc = 0;
      for (int32_t i = 0; i < nt; ++i) {
        int32_t o = tt[i];
        if (o == piv) continue;
        cand[nc].idx = o; cand[nc].val = w[o] / d; ++nc;
      }
      F->bsize[k] = 1; F->dd[k] = d;
      if (store_column(&S, k, cand, nc, fill, drop, m_a)) failed = 1;
      k += 1;
    } else {
      /* 2x2 pivot: c at k, r at k + 1 */
      swap_pos(&S, F->perm, k + 1, S.iperm[r]);
      double a = m1[c] ? w1[c] : 0.0, b = m1[r] ? w1[r] : 0.0, e = m2[r] ? w2[r] : 0.0;
      double det = a * e - b * b;
      int32_t ma1 = unpivoted_count(&S, c), ma2 = unpivoted_count(&S, r);
      S.pivoted[c] = 1; S.pivoted[r] = 1;
      F->bsize[k] = 2; F->bsize[k + 1] = 0;
      F->dd[k] = a; F->dd[k + 1] = e; F->doff[k] = b;
      /* rows touched by either column: union of t1 and t2 */
      int32_t nc = 0;
      for (int32_t h = 0; h < 2 && !failed; ++h) {
        nc = 0;
        for (int32_t src = 0; src < 2; ++src) {
          const int32_t *tt = src == 0 ? t1 : t2;
          int32_t nt = src == 0 ? nt1 : nt2;
          for (int32_t i = 0; i < nt; ++i) {
            int32_t o = tt[i];
            if (o == c || o == r) continue;
            if (src == 1 && m1[o]) continue;         /* already taken from t1 */
            double x1 = m1[o] ? w1[o] : 0.0, x2 = m2[o] ? w2[o] : 0.0;
            /* [l1 l2] = [x1 x2] D^{-1}, D^{-1} = [[e, -b], [-b, a]] / det */
            double l = h == 0 ? (x1 * e - x2 * b) / det : (x2 * a - x1 * b) / det;
            cand[nc].idx = o; cand[nc].val = l; ++nc;
          }
        }
        if (store_column(&S, k + h, cand, nc, fill, drop, h == 0 ? ma1 : ma2)) failed = 1;
      }
      k += 2;
    }
    for (int32_t i = 0; i < nt1; ++i) m1[t1[i]] = 0;
    for (int32_t i = 0; i < nt2; ++i) m2[t2[i]] = 0;
  }
  /* L in logical CSR */
  int64_t nnz = 0;
  for (int32_t j = 0; j < n; ++j) nnz += S.col[j].n;
  F->nnz_l = nnz;
  F->l_ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  F->l_col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
  F->l_val = (double *)malloc(sizeof(double) * (size_t)(nnz + 1));
  if (!failed) {
    for (int32_t j = 0; j < n; ++j)
      for (int64_t t = 0; t < S.col[j].n; ++t) F->l_ptr[S.iperm[S.col[j].e[t].idx] + 1]++;
    for (int32_t i = 0; i < n; ++i) F->l_ptr[i + 1] += F->l_ptr[i];
    int32_t *fillp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) fillp[i] = F->l_ptr[i];
    for (int32_t j = 0; j < n; ++j)   /* columns in increasing order: rows come out sorted */
      for (int64_t t = 0; t < S.col[j].n; ++t) {
        int32_t i = S.iperm[S.col[j].e[t].idx];
        F->l_col[fillp[i]] = j; F->l_val[fillp[i]] = S.col[j].e[t].val; fillp[i]++;
      }
    free(fillp);
  }
  for (int32_t j = 0; j < n; ++j) { free(S.col[j].e); free(S.row[j].e); }
  free(S.col); free(S.row); free(S.pivoted); free(S.iperm);
  free(w1); free(w2); free(t1); free(t2); free(m1); free(m2); free(cand);
  if (failed) { orc_ildlp_free(F); return NULL; }
  return F;
}

/* t = A^{-1} g through the factor: y = P g, L u = y, D w = u (1x1 and 2x2
 * blocks), L^T v = w, t = P^T v. */
void orc_ildlp_solve(const orc_ildlp *F, const double *g, double *t) {
  int32_t n = F->n;
  double *u = (double *)malloc(sizeof(double) * (size_t)n);
  for (int32_t i = 0; i < n; ++i) u[i] = g[F->perm[i]];
  for (int32_t i = 0; i < n; ++i)          /* L u = y */
    for (int32_t p = F->l_ptr[i]; p < F->l_ptr[i + 1]; ++p) u[i] -= F->l_val[p] * u[F->l_col[p]];
  for (int32_t i = 0; i < n; ++i) {        /* D w = u */
    if (F->bsize[i] == 1) {
      u[i] /= F->dd[i];
    } else if (F->bsize[i] == 2) {
      double a = F->dd[i], b = F->doff[i], e = F->dd[i + 1];
      double det = a * e - b * b, x = u[i], y = u[i + 1];
      u[i] = (e * x - b * y) / det;
      u[i + 1] = (a * y - b * x) / det;
    }
  }
  for (int32_t i = n - 1; i >= 0; --i)     /* L^T v = w (column sweep) */
    for (int32_t p = F->l_ptr[i]; p < F->l_ptr[i + 1]; ++p) u[F->l_col[p]] -= F->l_val[p] * u[i];
  for (int32_t i = 0; i < n; ++i) t[F->perm[i]] = u[i];
  free(u);
}

/* The same operator with each triangular solve replaced by `sweeps` (>= 1)
 * Jacobi sweeps, a reading of this library (the paper applies the factor
 * exactly): with L = I + L_s (L_s strictly lower),
 *   u_0 = y,  u_j = y - L_s u_{j-1}        (u_s = sum_{i<=s} (-L_s)^i y),
 *   v_0 = w,  v_j = w - L_s^T v_{j-1}      (v_s = sum_{i<=s} (-L_s^T)^i w),
 * with y = P g, w = D^{-1} u_s, t = P^T v_s: t = P^T S^T D^{-1} S P g with
 * S = sum_{i<=s} (-L_s)^i, a symmetric operator.  L_s is nilpotent, so the
 * result is the exact solve once s reaches the depth of L's dependencies. */
void orc_ildlp_solve_sweeps(const orc_ildlp *F, int32_t sweeps, const double *g, double *t) {
  int32_t n = F->n;
  double *y = (double *)malloc(sizeof(double) * (size_t)n);
  double *a = (double *)malloc(sizeof(double) * (size_t)n);
  double *b = (double *)malloc(sizeof(double) * (size_t)n);
  for (int32_t i = 0; i < n; ++i) y[i] = g[F->perm[i]];
  memcpy(a, y, sizeof(double) * (size_t)n);                  /* u_0 = y */
  for (int32_t j = 0; j < sweeps; ++j) {                       /* b = y - L_s a */
    for (int32_t i = 0; i < n; ++i) {
      double s = y[i];
      for (int32_t p = F->l_ptr[i]; p < F->l_ptr[i + 1]; ++p) s -= F->l_val[p] * a[F->l_col[p]];
      b[i] = s;
    }
    double *x = a; a = b; b = x;
  }
  for (int32_t i = 0; i < n; ++i) {                            /* y = w = D^{-1} u_s */
    if (F->bsize[i] == 1) {
      y[i] = a[i] / F->dd[i];
    } else if (F->bsize[i] == 2) {
      double p = F->dd[i], q = F->doff[i], e = F->dd[i + 1];
      double det = p * e - q * q;
      y[i] = (e * a[i] - q * a[i + 1]) / det;
      y[i + 1] = (p * a[i + 1] - q * a[i]) / det;
    }
  }
  memcpy(a, y, sizeof(double) * (size_t)n);                  /* v_0 = w */
  for (int32_t j = 0; j < sweeps; ++j) {                       /* b = w - L_s^T a */
    memcpy(b, y, sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < n; ++i)
      for (int32_t p = F->l_ptr[i]; p < F->l_ptr[i + 1]; ++p) b[F->l_col[p]] -= F->l_val[p] * a[i];
    double *x = a; a = b; b = x;
  }
  for (int32_t i = 0; i < n; ++i) t[F->perm[i]] = a[i];
  free(y); free(a); free(b);
}

/* ------------------------------------------------------------------------ */
/* Problem + preconditioner description                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t n;
  const int32_t *row_ptr, *col;
  const double *val;
  int32_t k;
  const double *Vhat; /* n x k column-major */
  const double *lam;  /* k, negative */
} orc_problem;

typedef struct {
  int32_t kind;                         /* ORC_PC_* */
  const double *diag;                   /* JACOBI: diag(A)            */
  const int32_t *l_ptr, *l_col;         /* ILDL0: strictly lower L    */
  const double *l_val, *d;              /* ILDL0: values, D           */
  const double *dense;                  /* DENSE: n x n row-major     */
  const int32_t *c_ptr, *c_col;         /* CCT: C lower CSR           */
  const double *c_val;
  int32_t smw;                          /* 1: MINRES-CG* (Section 2.1) */
  const orc_ildlp *ildlp;               /* ILDLP: the factor            */
  int32_t ildlp_sweeps;                 /* ILDLP: 0 exact, s > 0 sweeps */
} orc_inner_pc;

/* t = M_cg^{-1} g.  With smw = 1 the Sherman-Morrison-Woodbury form of
 * Section 2.1 is used: M_cg^{-1} = Atilde^{-1} - 2 Vhat Lambda_hat^{-1} Vhat^T. */
static void inner_pc_apply(const orc_problem *P, const orc_inner_pc *pc, const double *g,
                           double *t) {
  int32_t n = P->n;
  switch (pc->kind) {
    case ORC_PC_NONE:
      memcpy(t, g, sizeof(double) * (size_t)n);
      break;
    case ORC_PC_JACOBI:
#pragma omp parallel for schedule(static)
      for (int32_t i = 0; i < n; ++i) t[i] = g[i] / pc->diag[i];
      break;
    case ORC_PC_ILDL0:
      orc_ildl0_solve(n, pc->l_ptr, pc->l_col, pc->l_val, pc->d, g, t);
      break;
    case ORC_PC_DENSE:
#pragma omp parallel for schedule(static)
      for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t j = 0; j < n; ++j) s += pc->dense[(int64_t)i * n + j] * g[j];
        t[i] = s;
      }
      break;
    case ORC_PC_ILDLP:
      if (pc->ildlp_sweeps > 0)
        orc_ildlp_solve_sweeps(pc->ildlp, pc->ildlp_sweeps, g, t);
      else
        orc_ildlp_solve(pc->ildlp, g, t);
      break;
    case ORC_PC_CCT: {
      /* u = C^T g (scatter over rows of C), then t = C u */
      double *u = (double *)calloc((size_t)n, sizeof(double));
      for (int32_t i = 0; i < n; ++i)
        for (int32_t p = pc->c_ptr[i]; p < pc->c_ptr[i + 1]; ++p)
          u[pc->c_col[p]] += pc->c_val[p] * g[i];
      orc_spmv(n, pc->c_ptr, pc->c_col, pc->c_val, u, t);
      free(u);
      break;
    }
  }
  if (pc->smw && P->k > 0) {
    for (int32_t j = 0; j < P->k; ++j) {
      const double *vj = P->Vhat + (int64_t)j * n;
      double c = -2.0 * dot(n, vj, g) / P->lam[j];
#pragma omp parallel for schedule(static)
      for (int32_t i = 0; i < n; ++i) t[i] += c * vj[i];
    }
  }
}

/* t = M_cg^{-1} g on its own (the second-level apply, for the pin tests). */
void orc_precond_apply(const orc_problem *P, const orc_inner_pc *pc, const double *g, double *t) {
  inner_pc_apply(P, pc, g, t);
}

/* ------------------------------------------------------------------------ */
/* Inner solve: preconditioned CG on M_mr z = y with z0 = 0 (Section 2: CG   */
/* with a symmetric, possibly indefinite preconditioner M_cg; Galerkin       */
/* condition, energy-norm optimality in the M_mr norm).                      */
/* Stops when ||r||_2 <= rtol ||y||_2 or after maxit iterations.             */
/* Guards: p^T M_mr p <= 0 -> ORC_NOT_SPD;  rho = r^T M_cg^{-1} r with       */
/* |rho| <= eps*||r||*||t|| -> ORC_BREAKDOWN.  *its gets the iteration count. */
/* ------------------------------------------------------------------------ */
int32_t orc_pcg(const orc_problem *P, const orc_inner_pc *pc, const double *y, double *z,
                double rtol, int64_t maxit, int64_t *its, double *relres) {
  int32_t n = P->n;
  size_t bytes = sizeof(double) * (size_t)n;
  double *r = (double *)malloc(bytes), *t = (double *)malloc(bytes);
  double *p = (double *)malloc(bytes), *q = (double *)malloc(bytes);
  int32_t status = ORC_MAXIT;
  *its = 0;
  memset(z, 0, bytes);
  double ynorm = nrm2(n, y);
  if (relres) *relres = 0.0;
  if (ynorm == 0.0) { status = ORC_OK; goto done; }
  memcpy(r, y, bytes);
  inner_pc_apply(P, pc, r, t);
  double rho = dot(n, r, t);
  if (!(fabs(rho) > 2.220446049250313e-16 * ynorm * nrm2(n, t))) { status = ORC_BREAKDOWN; goto done; }
  memcpy(p, t, bytes);
  for (int64_t j = 1; j <= maxit; ++j) {
    orc_mmr_apply(n, P->row_ptr, P->col, P->val, P->k, P->Vhat, P->lam, p, q);
    double pi = dot(n, p, q);
    if (!(pi > 0.0)) { status = ORC_NOT_SPD; break; }
    double alpha = rho / pi;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) { z[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
    *its = j;
    double rn = nrm2(n, r);
    if (relres) *relres = rn / ynorm;
    if (rn <= rtol * ynorm) { status = ORC_OK; break; }
    if (j == maxit) break;
    inner_pc_apply(P, pc, r, t);
    double rho_new = dot(n, r, t);
    if (!(fabs(rho_new) > 2.220446049250313e-16 * rn * nrm2(n, t))) { status = ORC_BREAKDOWN; break; }
    double beta = rho_new / rho;
    rho = rho_new;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) p[i] = t[i] + beta * p[i];
  }
done:
  free(r); free(t); free(p); free(q);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Outer solve: preconditioned MINRES (Paige & Saunders 1975) on A x = b.    */
/* The preconditioner is applied as y = M^{-1} r, with M = M_mr applied by   */
/* the inner PCG above (the method), or a fixed dense M^{-1} / identity for  */
/* the pin tests.  Lanczos in the M^{-1} inner product, QR of the tridiagonal */
/* by Givens rotations, short-recurrence update of x.  Convergence is judged */
/* on the true relative residual ||b - A x||_2 / ||b||_2, recomputed every   */
/* outer iteration.                                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t outer_kind;     /* ORC_OUT_* */
  const double *dense;    /* ORC_OUT_DENSE: n x n row-major M^{-1} */
  double rtol_out, rtol_in;
  int32_t maxit_out;
  int64_t maxit_in;       /* per inner solve */
  int64_t maxit_in_total; /* budget over all inner solves */
  int32_t stag_window;    /* outer iterations without improvement -> stagnation */
  int32_t keep_best;      /* 1: on non-convergence return the iterate with the
                             smallest true residual instead of the last one */
} orc_opts;

typedef struct {
  int32_t status;
  int32_t outer_its;
  int64_t inner_its_total;
  double final_relres;
  int32_t hist_cap;        /* capacity of the arrays below (>= maxit_out + 1) */
  int64_t *inner_its;      /* per inner solve (outer_its + 1 entries) */
  double *relres;          /* true relative residual after each outer its */
  double *phibar;          /* MINRES residual estimate after each outer its */
} orc_stats;

static int32_t outer_precond(const orc_problem *P, const orc_inner_pc *pc, const orc_opts *o,
                             const double *r, double *y, orc_stats *st, int32_t solve_idx,
                             int64_t *budget) {
  int32_t n = P->n;
  if (o->outer_kind == ORC_OUT_NONE) { memcpy(y, r, sizeof(double) * (size_t)n); return ORC_OK; }
  if (o->outer_kind == ORC_OUT_DENSE) {
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int32_t j = 0; j < n; ++j) s += o->dense[(int64_t)i * n + j] * r[j];
      y[i] = s;
    }
    return ORC_OK;
  }
  int64_t cap = o->maxit_in < *budget ? o->maxit_in : *budget;
  int64_t its = 0;
  int32_t s = orc_pcg(P, pc, r, y, o->rtol_in, cap, &its, NULL);
  *budget -= its;
  st->inner_its_total += its;
  if (solve_idx < st->hist_cap) st->inner_its[solve_idx] = its;
  if (s == ORC_MAXIT && *budget > 0) s = ORC_OK; /* per-solve cap: accept the iterate */
  return s;
}

int32_t orc_minres_cg(const orc_problem *P, const orc_inner_pc *pc, const orc_opts *o,
                      const double *b, double *x, orc_stats *st) {
  int32_t n = P->n;
  size_t bytes = sizeof(double) * (size_t)n;
  double *r1 = (double *)malloc(bytes), *r2 = (double *)malloc(bytes);
  double *y = (double *)malloc(bytes), *v = (double *)malloc(bytes);
  double *w = (double *)calloc((size_t)n, sizeof(double));
  double *w1 = (double *)calloc((size_t)n, sizeof(double));
  double *w2 = (double *)calloc((size_t)n, sizeof(double));
  double *rt = (double *)malloc(bytes), *xbest = (double *)malloc(bytes);
  int64_t budget = o->maxit_in_total;
  st->status = ORC_MAXIT; st->outer_its = 0; st->inner_its_total = 0;
  int32_t status = ORC_MAXIT;

  double bnorm = nrm2(n, b);
  /* r1 = b - A x0 */
  orc_spmv(n, P->row_ptr, P->col, P->val, x, r1);
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) r1[i] = b[i] - r1[i];
  double rnorm = nrm2(n, r1);
  double best = rnorm;
  memcpy(xbest, x, bytes);
  st->final_relres = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  if (st->hist_cap > 0) { st->relres[0] = st->final_relres; st->phibar[0] = rnorm; }
  if (bnorm == 0.0 || rnorm <= o->rtol_out * bnorm) {
    status = ORC_OK;
    if (bnorm == 0.0) memset(x, 0, bytes);
    goto done;
  }
  int32_t s = outer_precond(P, pc, o, r1, y, st, 0, &budget);
  if (s != ORC_OK) { status = s; goto done; }
  double beta1 = dot(n, r1, y);
  if (!(beta1 > 0.0)) { status = ORC_BREAKDOWN; goto done; }
  beta1 = sqrt(beta1);
  if (st->hist_cap > 0) st->phibar[0] = beta1;

  double beta = beta1, oldb = 0.0, dbar = 0.0, epsln = 0.0, phibar = beta1;
  double cs = -1.0, sn = 0.0;
  memcpy(r2, r1, bytes);
  int32_t since_best = 0;
  for (int32_t itn = 1; itn <= o->maxit_out; ++itn) {
    /* Lanczos step in the M^{-1} inner product */
    double sc = 1.0 / beta;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) v[i] = sc * y[i];
    orc_spmv(n, P->row_ptr, P->col, P->val, v, y);
    if (itn >= 2) {
      double f = beta / oldb;
#pragma omp parallel for schedule(static)
      for (int32_t i = 0; i < n; ++i) y[i] -= f * r1[i];
    }
    double alfa = dot(n, v, y);
    double f2 = alfa / beta;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) y[i] -= f2 * r2[i];
    memcpy(r1, r2, bytes);
    memcpy(r2, y, bytes);
    s = outer_precond(P, pc, o, r2, y, st, itn, &budget);
    if (s != ORC_OK && s != ORC_MAXIT) { status = s; break; }
    oldb = beta;
    double b2 = dot(n, r2, y);
    if (!(b2 >= 0.0)) { status = ORC_BREAKDOWN; break; }
    beta = sqrt(b2);

    /* apply the previous rotation, build and apply the new one */
    double oldeps = epsln;
    double delta = cs * dbar + sn * alfa;
    double gbar = sn * dbar - cs * alfa;
    epsln = sn * beta;
    dbar = -cs * beta;
    double gamma = hypot(gbar, beta);
    if (gamma < 2.220446049250313e-16) gamma = 2.220446049250313e-16;
    cs = gbar / gamma;
    sn = beta / gamma;
    double phi = cs * phibar;
    phibar = sn * phibar;

    /* w_k = (v_k - eps_k w_{k-2} - delta_k w_{k-1}) / gamma_k ; x += phi w */
    double *tmp = w1; w1 = w2; w2 = w; w = tmp;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
      w[i] = (v[i] - oldeps * w1[i] - delta * w2[i]) / gamma;
      x[i] += phi * w[i];
    }

    /* true residual */
    orc_spmv(n, P->row_ptr, P->col, P->val, x, rt);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) rt[i] = b[i] - rt[i];
    rnorm = nrm2(n, rt);
    st->outer_its = itn;
    if (itn < st->hist_cap) { st->relres[itn] = rnorm / bnorm; st->phibar[itn] = phibar; }
    st->final_relres = rnorm / bnorm;
    if (rnorm < best) {
      if (rnorm < best * (1.0 - 1e-3)) since_best = 0; else ++since_best;
      best = rnorm;
      memcpy(xbest, x, bytes);
    } else {
      ++since_best;
    }
    if (rnorm <= o->rtol_out * bnorm) { status = ORC_OK; break; }
    if (s == ORC_MAXIT || budget <= 0) { status = ORC_MAXIT; break; }
    if (o->stag_window > 0 && since_best >= o->stag_window) { status = ORC_STAGNATION; break; }
    if (beta == 0.0) { status = ORC_BREAKDOWN; break; }
  }
  if (status != ORC_OK && o->keep_best) { /* leave the best iterate in x */
    memcpy(x, xbest, bytes);
    st->final_relres = best / bnorm;
  }
done:
  st->status = status;
  free(r1); free(r2); free(y); free(v); free(w); free(w1); free(w2); free(rt); free(xbest);
  return status;
}

/* number of OpenMP threads the oracle runs with */
int32_t orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* set the number of OpenMP threads of later calls (t >= 1; timing only) */
void orc_set_num_threads(int32_t t) {
#ifdef _OPENMP
  if (t >= 1) omp_set_num_threads(t);
#else
  (void)t;
#endif
}
