// Host-side integer kernel basis of A (Section 3.1 of the paper):
//  * column-style Hermite normal form A K = (H | 0) with K unimodular
//    (Lemma 3.1); B = last n - rank(A) columns of K spans Ker_Z(A)
//    (Theorem 3.2);
//  * LLL reduction (Appendix A, Algorithm 3) in exact integer arithmetic
//    using the integral Gram-Schmidt quantities d_k (Gram determinants) and
//    lambda_ij = d_j mu_ij (Cohen, "A Course in Computational Algebraic
//    Number Theory", Sec. 2.6);
//  * the coordinate map P = (B^T B)^{-1} B^T (Section 3.1) in binary64.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "bigint.h"
#include "graver_internal.h"

namespace graver {
namespace {

struct Overflow {};

inline int64_t chk_mul(int64_t a, int64_t b) {
  int64_t r;
  if (__builtin_mul_overflow(a, b, &r)) throw Overflow();
  return r;
}
inline int64_t chk_sub(int64_t a, int64_t b) {
  int64_t r;
  if (__builtin_sub_overflow(a, b, &r)) throw Overflow();
  return r;
}
inline int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b, r = a % b;
  if (r != 0 && ((r < 0) != (b < 0))) --q;
  return q;
}

// Columns are stored contiguously: col[c][row].
struct ColMat {
  int rows, cols;
  std::vector<int64_t> v;
  ColMat(int r, int c) : rows(r), cols(c), v((size_t)r * c, 0) {}
  int64_t& at(int r, int c) { return v[(size_t)c * rows + r]; }
  int64_t* col(int c) { return &v[(size_t)c * rows]; }
};

// Hermite normal form by unimodular column operations.  Row i: among the
// columns p..n-1 pick the nonzero entry of smallest magnitude (ties: lowest
// column), move it to column p, reduce every other column k > p by
// floor(w_ik / w_ip) times column p; repeat until column p is the only
// nonzero among p..n-1.  Make the pivot positive, reduce entries left of
// it into [0, pivot), advance p.  Rows without a nonzero in p..n-1 are
// dependent and give no pivot.  Returns the rank; K is n x n.
int hnf(int m, int n, const int64_t* A, ColMat& K) {
  ColMat W(m, n);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) W.at(i, j) = A[(size_t)i * n + j];
  for (int i = 0; i < n; ++i) K.at(i, i) = 1;
  auto axpy = [&](int dst, int src, int64_t q) {  // col dst -= q col src
    int64_t *wd = W.col(dst), *ws = W.col(src), *kd = K.col(dst), *ks = K.col(src);
    for (int r = 0; r < m; ++r) wd[r] = chk_sub(wd[r], chk_mul(q, ws[r]));
    for (int r = 0; r < n; ++r) kd[r] = chk_sub(kd[r], chk_mul(q, ks[r]));
  };
  auto swapc = [&](int a, int b) {
    for (int r = 0; r < m; ++r) std::swap(W.at(r, a), W.at(r, b));
    for (int r = 0; r < n; ++r) std::swap(K.at(r, a), K.at(r, b));
  };
  int p = 0;
  for (int i = 0; i < m && p < n; ++i) {
    bool pivoted = false;
    for (;;) {
      int piv = -1;
      int64_t best = 0;
      for (int k = p; k < n; ++k) {
        int64_t w = W.at(i, k);
        if (w == 0) continue;
        if (w == INT64_MIN) throw Overflow();
        int64_t a = w < 0 ? -w : w;
        if (piv < 0 || a < best) {
          piv = k;
          best = a;
        }
      }
      if (piv < 0) break;
      if (piv != p) swapc(p, piv);
      pivoted = true;
      bool clean = true;
      for (int k = p + 1; k < n; ++k) {
        if (W.at(i, k) != 0) {
          int64_t q = floor_div(W.at(i, k), W.at(i, p));
          axpy(k, p, q);
          if (W.at(i, k) != 0) clean = false;
        }
      }
      if (clean) break;
    }
    if (!pivoted) continue;
    if (W.at(i, p) < 0) {
      for (int r = 0; r < m; ++r) W.at(r, p) = chk_sub(0, W.at(r, p));
      for (int r = 0; r < n; ++r) K.at(r, p) = chk_sub(0, K.at(r, p));
    }
    for (int j = 0; j < p; ++j) {
      int64_t q = floor_div(W.at(i, j), W.at(i, p));
      if (q != 0) axpy(j, p, q);
    }
    ++p;
  }
  return p;
}

// LLL in the paper's order (Appendix A, Algorithm 3): with i from the
// second vector, size-reduce b_i against b_{i-1}, ..., b_1, then exchange
// b_i, b_{i-1} when ||b*_{i-1}||^2 > 2 ||b*_i||^2 (i.e. D[i]^2 > 2 D[i+1]
// D[i-1]) and step back (not below the second vector), else advance.
// b: d vectors of length n (int64, overflow-checked).
void lll(int n, int d, std::vector<std::vector<int64_t>>& b) {
  if (d <= 1) return;
  std::vector<BigInt> D(d + 1);
  std::vector<std::vector<BigInt>> lam(d, std::vector<BigInt>(d));
  D[0] = BigInt(1);
  auto dot = [&](int a, int c) {
    __int128 s = 0;
    for (int r = 0; r < n; ++r) s += (__int128)b[a][r] * b[c][r];
    return BigInt::from_i128(s);
  };
  for (int k = 0; k < d; ++k) {
    for (int j = 0; j <= k; ++j) {
      BigInt u = dot(k, j);
      for (int i = 0; i < j; ++i) u = BigInt::div_exact(D[i + 1] * u - lam[k][i] * lam[j][i], D[i]);
      if (j < k) {
        lam[k][j] = u;
      } else {
        if (u.is_zero()) throw std::logic_error("kernel basis columns are dependent");
        D[k + 1] = u;
      }
    }
  }
  auto size_reduce = [&](int k, int j) {
    BigInt q = BigInt::div_round_half_even(lam[k][j], D[j + 1]);
    if (q.is_zero()) return;
    if (!q.fits_i64()) throw Overflow();
    int64_t qi = q.to_i64();
    for (int r = 0; r < n; ++r) b[k][r] = chk_sub(b[k][r], chk_mul(qi, b[j][r]));
    lam[k][j] = lam[k][j] - q * D[j + 1];
    for (int i = 0; i < j; ++i) lam[k][i] = lam[k][i] - q * lam[j][i];
  };
  auto exchange = [&](int k) {
    std::swap(b[k], b[k - 1]);
    for (int j = 0; j < k - 1; ++j) std::swap(lam[k][j], lam[k - 1][j]);
    BigInt lk = lam[k][k - 1];
    BigInt Bn = BigInt::div_exact(D[k - 1] * D[k + 1] + lk * lk, D[k]);
    for (int i = k + 1; i < d; ++i) {
      BigInt t = lam[i][k];
      lam[i][k] = BigInt::div_exact(D[k + 1] * lam[i][k - 1] - lk * t, D[k]);
      lam[i][k - 1] = BigInt::div_exact(Bn * t + lk * lam[i][k], D[k + 1]);
    }
    D[k] = Bn;
  };
  int i = 1;
  const BigInt two(2);
  while (i < d) {
    for (int j = i - 1; j >= 0; --j) size_reduce(i, j);
    if (D[i] * D[i] > two * D[i + 1] * D[i - 1]) {
      exchange(i);
      i = i - 1 > 1 ? i - 1 : 1;
    } else {
      ++i;
    }
  }
}

// ---- kernel basis with reduction interleaved in the elimination ---------
//
// The unreduced kernel columns of the elimination above have entries of the
// size of A's maximal minors, which leave int64 for dense enough A.  Here
// the rows of A are taken one at a time on a basis of the lattice
// {x in Z^n : A_0 x = ... = A_{i-1} x = 0} (initially the unit vectors):
// the row's values v = a_i . b_c on the basis vectors are brought to a single
// nonzero by unimodular column operations (nearest-integer quotients), the
// vector holding it leaves the basis, and the remaining vectors, a basis of
// the lattice with row i added (they are unimodular combinations of the old
// ones with a_i . b = 0), are LLL-reduced before the next row.  The result
// spans Ker_Z(A) (Theorem 3.2: any basis of that lattice) with short
// vectors throughout.  Reduction: LLL with a binary64 Gram-Schmidt computed
// from the exact integer Gram matrix (Schnorr and Euchner, 1994), Lovasz
// parameter 0.99 and size bound 0.51; every basis operation is exact integer
// arithmetic, so the basis is a basis of the lattice whatever the rounding.

constexpr int64_t kRedMax = (int64_t)1 << 40;  // entry bound of the reduced path
constexpr int64_t kRedTrigger = 1 << 12;        // entries beyond this trigger a reduction

struct FpLattice {
  int n = 0;
  std::vector<std::vector<int64_t>> b;   // basis vectors (length n)
  std::vector<std::vector<__int128>> G;  // exact Gram matrix
  std::vector<std::vector<double>> mu, r;

  static __int128 dot(const std::vector<int64_t>& x, const std::vector<int64_t>& y) {
    __int128 s = 0;
    for (size_t t = 0; t < x.size(); ++t) s += (__int128)x[t] * y[t];
    return s;
  }
  void gram_all() {
    const int k = (int)b.size();
    G.assign(k, std::vector<__int128>(k));
    for (int i = 0; i < k; ++i)
      for (int j = 0; j <= i; ++j) G[i][j] = G[j][i] = dot(b[i], b[j]);
  }
  // b[i] -= q b[j], with the Gram matrix kept exact
  void axpy(int i, int j, int64_t q) {
    if (q == 0) return;
    for (int t = 0; t < n; ++t) {
      const int64_t v = chk_sub(b[i][t], chk_mul(q, b[j][t]));
      if (v > kRedMax || v < -kRedMax) throw Overflow();
      b[i][t] = v;
    }
    const int k = (int)b.size();
    const __int128 gii = G[i][i] - 2 * (__int128)q * G[i][j] + (__int128)q * q * G[j][j];
    for (int l = 0; l < k; ++l)
      if (l != i) G[i][l] = G[l][i] = G[i][l] - (__int128)q * G[j][l];
    G[i][i] = gii;
  }
  void swap_vec(int i, int j) {
    std::swap(b[i], b[j]);
    std::swap(G[i], G[j]);
    for (auto& row : G) std::swap(row[i], row[j]);
  }
  void drop(int i) {  // remove vector i (order of the others kept)
    b.erase(b.begin() + i);
    G.erase(G.begin() + i);
    for (auto& row : G) row.erase(row.begin() + i);
  }
  void gso_row(int i) {
    double* ri = r[i].data();
    for (int j = 0; j <= i; ++j) {
      const double* mj = mu[j].data();
      // four partial sums (the order only moves rounding; exact integer
      // operations keep the basis a basis)
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int l = 0;
      for (; l + 4 <= j; l += 4) {
        s0 += mj[l] * ri[l];
        s1 += mj[l + 1] * ri[l + 1];
        s2 += mj[l + 2] * ri[l + 2];
        s3 += mj[l + 3] * ri[l + 3];
      }
      for (; l < j; ++l) s0 += mj[l] * ri[l];
      const double v = (double)G[i][j] - ((s0 + s1) + (s2 + s3));
      ri[j] = v;
      if (j < i) mu[i][j] = v / r[j][j];
    }
  }
  // LLL from vector `start` on (the vectors before it are assumed reduced)
  void lll(int start) {
    const int k = (int)b.size();
    if (k < 2) return;
    mu.assign(k, std::vector<double>(k, 0.0));
    r.assign(k, std::vector<double>(k, 0.0));
    for (int i = 0; i < std::max(start, 1); ++i) gso_row(i);
    int kap = std::max(start, 1);
    const double delta = 0.99, eta = 0.51;
    int64_t steps = 0;
    const int64_t cap = 200LL * k * k + 100000;
    while (kap < k) {
      if (++steps > cap) break;  // rounding cycles: stop (still a basis)
      // size reduction, repeated from the exact Gram matrix until no
      // coefficient exceeds eta (b*_kap and r[kap][kap] do not change)
      for (int pass = 0; pass < 64; ++pass) {
        gso_row(kap);
        bool any = false;
        for (int j = kap - 1; j >= 0; --j) {
          const double m = mu[kap][j];
          if (!(std::fabs(m) > eta)) continue;
          if (!(std::fabs(m) < 9.0e15)) throw Overflow();
          const int64_t q = (int64_t)std::nearbyint(m);
          axpy(kap, j, q);
          for (int l = 0; l < j; ++l) mu[kap][l] -= (double)q * mu[j][l];
          mu[kap][j] -= (double)q;
          any = true;
        }
        if (!any) break;
      }
      const double m1 = mu[kap][kap - 1];
      if (delta * r[kap - 1][kap - 1] > r[kap][kap] + m1 * m1 * r[kap - 1][kap - 1]) {
        swap_vec(kap, kap - 1);
        kap = std::max(kap - 1, 1);
        if (kap == 1) gso_row(0);
      } else {
        ++kap;
      }
    }
  }
};

// Kernel basis of A (m x n) by rows with interleaved reduction; returns the
// basis vectors.
std::vector<std::vector<int64_t>> kernel_interleaved(int m, int n, const int64_t* A) {
  FpLattice L;
  L.n = n;
  L.b.assign(n, std::vector<int64_t>(n, 0));
  for (int i = 0; i < n; ++i) L.b[i][i] = 1;
  L.gram_all();
  std::vector<int32_t> nzc;
  std::vector<int64_t> nzv;
  for (int i = 0; i < m; ++i) {
    nzc.clear();
    nzv.clear();
    for (int j = 0; j < n; ++j)
      if (A[(size_t)i * n + j] != 0) {
        nzc.push_back(j);
        nzv.push_back(A[(size_t)i * n + j]);
      }
    const int k = (int)L.b.size();
    std::vector<int64_t> v(k);
    for (int c = 0; c < k; ++c) {
      __int128 s = 0;
      for (size_t t = 0; t < nzc.size(); ++t) s += (__int128)nzv[t] * L.b[c][nzc[t]];
      if (s > INT64_MAX / 4 || s < -(INT64_MAX / 4)) throw Overflow();
      v[c] = (int64_t)s;
    }
    // Euclid over the basis vectors: pivot on the smallest |v_c| (ties: the
    // shortest vector, then the lowest index) until one nonzero remains
    int piv = -1;
    for (;;) {
      piv = -1;
      for (int c = 0; c < k; ++c) {
        if (v[c] == 0) continue;
        if (piv < 0) {
          piv = c;
          continue;
        }
        const int64_t a = v[c] < 0 ? -v[c] : v[c], bp = v[piv] < 0 ? -v[piv] : v[piv];
        if (a < bp || (a == bp && L.G[c][c] < L.G[piv][piv])) piv = c;
      }
      if (piv < 0) break;
      bool clean = true;
      for (int c = 0; c < k; ++c) {
        if (c == piv || v[c] == 0) continue;
        const int64_t q = (int64_t)std::llround((long double)v[c] / (long double)v[piv]);
        L.axpy(c, piv, q);
        v[c] -= q * v[piv];
        if (v[c] != 0) clean = false;
      }
      if (clean) break;
    }
    if (piv < 0) continue;  // a_i depends on earlier rows
    L.drop(piv);
    // reduce once the entries have grown (and after the last row)
    int64_t mx = 0;
    for (const auto& vec : L.b)
      for (int64_t x : vec) mx = std::max<int64_t>(mx, x < 0 ? -x : x);
    if (mx > kRedTrigger) L.lll(0);
  }
  L.lll(0);
  return L.b;
}

// P = (B^T B)^{-1} B^T by Cholesky of the exact Gram matrix (binary64) and
// one step of iterative refinement, solving for all n right-hand sides at
// once (row-major d x n panels, so the inner loops run along contiguous
// memory).
void projector(int n, int d, const std::vector<std::vector<int64_t>>& b, double* P) {
  std::vector<double> G((size_t)d * d), L((size_t)d * d, 0.0);
  int64_t bmax = 0;
  for (int i = 0; i < d; ++i)
    for (int r = 0; r < n; ++r) bmax = std::max<int64_t>(bmax, b[i][r] < 0 ? -b[i][r] : b[i][r]);
  const bool small = bmax < ((int64_t)1 << 20) && (__int128)n * bmax * bmax < ((__int128)1 << 62);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j <= i; ++j) {
      double v;
      if (small) {  // exact in int64
        int64_t s = 0;
        const int64_t* bi = b[i].data();
        const int64_t* bj = b[j].data();
        for (int r = 0; r < n; ++r) s += bi[r] * bj[r];
        v = (double)s;
      } else {
        __int128 s = 0;
        for (int r = 0; r < n; ++r) s += (__int128)b[i][r] * b[j][r];
        v = (double)s;
      }
      G[(size_t)i * d + j] = G[(size_t)j * d + i] = v;
    }
  for (int j = 0; j < d; ++j) {
    double s = G[(size_t)j * d + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * d + k] * L[(size_t)j * d + k];
    const double dj = std::sqrt(s);
    L[(size_t)j * d + j] = dj;
    for (int i = j + 1; i < d; ++i) {
      double t = G[(size_t)i * d + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * d + k] * L[(size_t)j * d + k];
      L[(size_t)i * d + j] = t / dj;
    }
  }
  // X (d x n) = G^{-1} R for a d x n panel R, in place
  auto solve = [&](std::vector<double>& X) {
    for (int i = 0; i < d; ++i) {
      double* xi = &X[(size_t)i * n];
      for (int k = 0; k < i; ++k) {
        const double l = L[(size_t)i * d + k];
        const double* xk = &X[(size_t)k * n];
        for (int r = 0; r < n; ++r) xi[r] -= l * xk[r];
      }
      const double inv = 1.0 / L[(size_t)i * d + i];
      for (int r = 0; r < n; ++r) xi[r] *= inv;
    }
    for (int i = d - 1; i >= 0; --i) {
      double* xi = &X[(size_t)i * n];
      for (int k = i + 1; k < d; ++k) {
        const double l = L[(size_t)k * d + i];
        const double* xk = &X[(size_t)k * n];
        for (int r = 0; r < n; ++r) xi[r] -= l * xk[r];
      }
      const double inv = 1.0 / L[(size_t)i * d + i];
      for (int r = 0; r < n; ++r) xi[r] *= inv;
    }
  };
  std::vector<double> X((size_t)d * n), E((size_t)d * n);
  for (int i = 0; i < d; ++i)
    for (int r = 0; r < n; ++r) X[(size_t)i * n + r] = (double)b[i][r];
  solve(X);
  // residual B^T - G X, then the correction
  for (int i = 0; i < d; ++i) {
    double* ei = &E[(size_t)i * n];
    for (int r = 0; r < n; ++r) ei[r] = (double)b[i][r];
    for (int k = 0; k < d; ++k) {
      const double gik = G[(size_t)i * d + k];
      if (gik == 0.0) continue;
      const double* xk = &X[(size_t)k * n];
      for (int r = 0; r < n; ++r) ei[r] -= gik * xk[r];
    }
  }
  solve(E);
  for (size_t t = 0; t < (size_t)d * n; ++t) P[t] = X[t] + E[t];
}

}  // namespace

graver_status kernel_basis_host(int32_t m, int32_t n, const int64_t* A, int32_t do_lll,
                                int64_t* B_out, int32_t* d_out, double* P_out) {
  try {
    std::vector<std::vector<int64_t>> b;
    try {
      // Lemma 3.1 as stated: the Hermite normal form's kernel columns, then
      // (optionally) Algorithm 3 in exact arithmetic
      ColMat K(n, n);
      int r = hnf(m, n, A, K);
      int d = n - r;
      b.assign(d, std::vector<int64_t>(n));
      for (int c = 0; c < d; ++c)
        for (int row = 0; row < n; ++row) b[c][row] = K.at(row, r + c);
      if (do_lll) lll(n, d, b);
    } catch (const Overflow&) {
      // its int64 entries overflow: the same lattice with reduction
      // interleaved (always reduced, whatever do_lll says)
      b = kernel_interleaved(m, n, A);
    }
    const int d = (int)b.size();
    // exact check A B = 0 (Theorem 3.2 relies on it)
    for (int i = 0; i < m; ++i)
      for (int c = 0; c < d; ++c) {
        __int128 s = 0;
        for (int j = 0; j < n; ++j) s += (__int128)A[(size_t)i * n + j] * b[c][j];
        if (s != 0) return set_error(GRAVER_E_NOT_KERNEL, "computed basis is not in Ker(A)");
      }
    for (int row = 0; row < n; ++row)
      for (int c = 0; c < d; ++c) B_out[(size_t)row * d + c] = b[c][row];
    *d_out = d;
    if (P_out && d > 0) projector(n, d, b, P_out);
    return GRAVER_OK;
  } catch (const Overflow&) {
    return set_error(GRAVER_E_OVERFLOW, "int64 overflow in the kernel basis computation");
  } catch (const std::exception& e) {
    return set_error(GRAVER_E_INVALID, std::string("kernel basis: ") + e.what());
  }
}

}  // namespace graver
