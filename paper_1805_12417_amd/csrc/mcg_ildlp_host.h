// Host-side pivoted incomplete L D L^T (Section 4's ILDL^T(fill, drop)), used
// by the MCG_PC_ILDLP preconditioner at create.  Plain C++, no device code.
//
// Column by column in A's order: the column of the current Schur complement
// (A's column over the rows not yet pivoted, minus the kept columns'
// contributions), the Bunch-Kaufman choice of a 1x1 or 2x2 pivot
// (alpha = (1 + sqrt 17) / 8), the new column(s) of L, then dropping
// (|l| < drop ||l||_2) and the fill limit (the ceil(fill m) largest, m = A's
// off-diagonal entries of the pivot column in rows not yet pivoted, ties to
// the smaller original row; fill <= 0: no limit).  Rows of L are kept by
// original index while the factorization runs, so an interchange only
// touches the permutation.  A 1x1 pivot below 1e-8 max|a_ij| in magnitude
// becomes that floor with its sign.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

struct PivotedLDL {
  std::vector<int32_t> perm, bsize;          // logical -> original; 1, 2 (block start), 0
  std::vector<double> dd, doff;              // D: diagonal, D(k, k+1) at block starts
  std::vector<int32_t> lrp, lci;             // L strictly lower, logical CSR
  std::vector<double> lv;
};

class PivotedBuilder {
 public:
  PivotedBuilder(int n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                 const std::vector<double> &va, double fill, double drop)
      : n_(n), rp_(rp), ci_(ci), va_(va), fill_(fill), drop_(drop), cols_(n), rows_(n),
        pivoted_(n, 0), pos_(n), a_(n), b_(n) {
    for (double x : va) amax_ = std::max(amax_, std::fabs(x));
  }

  void run(PivotedLDL &F) {
    const double alpha = (1.0 + std::sqrt(17.0)) / 8.0;
    const double floor_ = 1e-8 * amax_;
    F.perm.resize(n_);
    F.bsize.assign(n_, 0);
    F.dd.assign(n_, 0.0);
    F.doff.assign(n_, 0.0);
    for (int i = 0; i < n_; ++i) F.perm[i] = pos_[i] = i;
    perm_ = &F.perm;
    bsize_ = &F.bsize;
    dd_ = &F.dd;
    doff_ = &F.doff;
    int k = 0;
    while (k < n_) {
      const int c = F.perm[k];
      schur(c, a_);
      const double akk = a_.on[c] ? std::fabs(a_.w[c]) : 0.0;
      double colmax = 0.0;
      int r = -1;
      for (int o : a_.list) {
        if (o == c) continue;
        const double v = std::fabs(a_.w[o]);
        if (v > colmax || (v == colmax && v > 0.0 && pos_[o] < pos_[r])) {
          colmax = v;
          r = o;
        }
      }
      bool twobytwo = false;
      int piv = c;
      bool have_b = false;
      if (colmax > 0.0 && !(akk >= alpha * colmax)) {
        schur(r, b_);
        have_b = true;
        double rowmax = 0.0;
        for (int o : b_.list)
          if (o != r) rowmax = std::max(rowmax, std::fabs(b_.w[o]));
        const double arr = b_.on[r] ? std::fabs(b_.w[r]) : 0.0;
        if (akk * rowmax >= alpha * colmax * colmax)
          piv = c;
        else if (arr >= alpha * rowmax)
          piv = r;
        else
          twobytwo = true;
      }
      if (!twobytwo) {
        const Dense &W = piv == c ? a_ : b_;
        interchange(k, pos_[piv]);
        double d = W.on[piv] ? W.w[piv] : 0.0;
        if (std::fabs(d) < floor_) d = d < 0.0 ? -floor_ : floor_;
        const int m = offdiag_unpivoted(piv);
        pivoted_[piv] = 1;
        cand_.clear();
        for (int o : W.list)
          if (o != piv) cand_.push_back({o, W.w[o] / d});
        F.bsize[k] = 1;
        F.dd[k] = d;
        keep(k, m);
        k += 1;
      } else {
        interchange(k + 1, pos_[r]);
        const double a = a_.on[c] ? a_.w[c] : 0.0, b = a_.on[r] ? a_.w[r] : 0.0;
        const double e = b_.on[r] ? b_.w[r] : 0.0;
        const double det = a * e - b * b;
        const int m1 = offdiag_unpivoted(c), m2 = offdiag_unpivoted(r);
        pivoted_[c] = pivoted_[r] = 1;
        F.bsize[k] = 2;
        F.bsize[k + 1] = 0;
        F.dd[k] = a;
        F.dd[k + 1] = e;
        F.doff[k] = b;
        for (int h = 0; h < 2; ++h) {
          cand_.clear();
          auto add = [&](int o) {
            const double x1 = a_.on[o] ? a_.w[o] : 0.0, x2 = b_.on[o] ? b_.w[o] : 0.0;
            const double l = h == 0 ? (x1 * e - x2 * b) / det : (x2 * a - x1 * b) / det;
            cand_.push_back({o, l});
          };
          for (int o : a_.list)
            if (o != c && o != r) add(o);
          for (int o : b_.list)
            if (o != c && o != r && !a_.on[o]) add(o);
          keep(k + h, h == 0 ? m1 : m2);
        }
        k += 2;
      }
      a_.reset();
      if (have_b) b_.reset();
    }
    // L in logical CSR, rows sorted by column
    F.lrp.assign(n_ + 1, 0);
    for (int j = 0; j < n_; ++j)
      for (const Ent &x : cols_[j]) F.lrp[pos_[x.idx] + 1]++;
    for (int i = 0; i < n_; ++i) F.lrp[i + 1] += F.lrp[i];
    F.lci.resize(F.lrp[n_]);
    F.lv.resize(F.lrp[n_]);
    std::vector<int32_t> at(F.lrp.begin(), F.lrp.end() - 1);
    for (int j = 0; j < n_; ++j)
      for (const Ent &x : cols_[j]) {
        const int i = pos_[x.idx];
        F.lci[at[i]] = j;
        F.lv[at[i]] = x.val;
        ++at[i];
      }
  }

 private:
  struct Ent {
    int32_t idx;
    double val;
  };
  // one Schur complement column, dense by original index, with its support
  struct Dense {
    std::vector<double> w;
    std::vector<char> on;
    std::vector<int32_t> list;
    explicit Dense(int n) : w(n, 0.0), on(n, 0) {}
    void touch(int o) {
      if (!on[o]) {
        on[o] = 1;
        w[o] = 0.0;
        list.push_back(o);
      }
    }
    void reset() {
      for (int o : list) on[o] = 0;
      list.clear();
    }
  };

  // column c of the current Schur complement, rows not yet pivoted
  void schur(int c, Dense &W) {
    for (int32_t q = rp_[c]; q < rp_[c + 1]; ++q) {
      const int o = ci_[q];
      if (pivoted_[o]) continue;
      W.touch(o);
      W.w[o] += va_[q];
    }
    const std::vector<Ent> &row = rows_[c];
    for (size_t q = 0; q < row.size(); ++q) {
      const int j = row[q].idx;
      const int bsj = (*bsize_)[j];
      if (bsj == 1) {
        const double coef = (*dd_)[j] * row[q].val;
        subtract(j, coef, W);
        continue;
      }
      const int s0 = bsj == 2 ? j : j - 1;  // 2x2 block (s0, s0 + 1), taken once
      if (j == s0 + 1 && q > 0 && row[q - 1].idx == s0) continue;
      double xa = 0.0, xb = 0.0;
      if (j == s0) {
        xa = row[q].val;
        if (q + 1 < row.size() && row[q + 1].idx == s0 + 1) xb = row[q + 1].val;
      } else {
        xb = row[q].val;
      }
      const double u1 = (*dd_)[s0] * xa + (*doff_)[s0] * xb;
      const double u2 = (*doff_)[s0] * xa + (*dd_)[s0 + 1] * xb;
      subtract(s0, u1, W);
      subtract(s0 + 1, u2, W);
    }
  }

  void subtract(int j, double coef, Dense &W) {
    for (const Ent &x : cols_[j]) {
      if (pivoted_[x.idx]) continue;
      W.touch(x.idx);
      W.w[x.idx] -= x.val * coef;
    }
  }

  int offdiag_unpivoted(int c) const {
    int m = 0;
    for (int32_t q = rp_[c]; q < rp_[c + 1]; ++q)
      if (ci_[q] != c && !pivoted_[ci_[q]]) ++m;
    return m;
  }

  void interchange(int p, int q) {
    if (p == q) return;
    std::vector<int32_t> &perm = *perm_;
    const int a = perm[p], b = perm[q];
    perm[p] = b;
    perm[q] = a;
    pos_[b] = p;
    pos_[a] = q;
  }

  // dropping and the fill limit on cand_, then store column k
  void keep(int k, int m) {
    double ss = 0.0;
    for (const Ent &x : cand_) ss += x.val * x.val;
    const double nrm = std::sqrt(ss);
    size_t nk = 0;
    for (size_t i = 0; i < cand_.size(); ++i)
      if (cand_[i].val != 0.0 && std::fabs(cand_[i].val) >= drop_ * nrm) cand_[nk++] = cand_[i];
    cand_.resize(nk);
    if (fill_ > 0.0) {
      const size_t lim = (size_t)std::max(1.0, std::ceil(fill_ * (double)m));
      if (cand_.size() > lim) {
        std::sort(cand_.begin(), cand_.end(), [](const Ent &x, const Ent &y) {
          const double ax = std::fabs(x.val), ay = std::fabs(y.val);
          if (ax != ay) return ax > ay;
          return x.idx < y.idx;
        });
        cand_.resize(lim);
      }
    }
    for (const Ent &x : cand_) {
      cols_[k].push_back(x);
      rows_[x.idx].push_back({k, x.val});
    }
  }

  int n_;
  const std::vector<int32_t> &rp_, &ci_;
  const std::vector<double> &va_;
  double fill_, drop_, amax_ = 0.0;
  std::vector<std::vector<Ent>> cols_, rows_;  // L by column (original rows); rows: (column, value)
  std::vector<char> pivoted_;
  std::vector<int32_t> pos_;                   // original -> logical
  Dense a_, b_;
  std::vector<Ent> cand_;
  std::vector<int32_t> *perm_ = nullptr, *bsize_ = nullptr;
  std::vector<double> *dd_ = nullptr, *doff_ = nullptr;
};
