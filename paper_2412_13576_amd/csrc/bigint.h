// Minimal signed arbitrary-precision integer for the exact lattice
// reduction on the host (Gram determinants of the kernel basis exceed
// 128 bits for n in the hundreds).  Sign-magnitude, 32-bit limbs, little
// endian; division is Knuth's Algorithm D (TAOCP vol. 2, 4.3.1).
#pragma once

#include <cstdint>
#include <stdexcept>
#include <vector>

namespace graver {

class BigInt {
 public:
  BigInt() = default;
  BigInt(int64_t v) {  // NOLINT(runtime/explicit)
    neg_ = v < 0;
    uint64_t m = neg_ ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
    while (m) {
      mag_.push_back((uint32_t)m);
      m >>= 32;
    }
  }
  static BigInt from_i128(__int128 v) {
    BigInt r;
    r.neg_ = v < 0;
    unsigned __int128 m = r.neg_ ? (unsigned __int128)0 - (unsigned __int128)v : (unsigned __int128)v;
    while (m) {
      r.mag_.push_back((uint32_t)m);
      m >>= 32;
    }
    return r;
  }

  bool is_zero() const { return mag_.empty(); }
  bool is_neg() const { return neg_; }
  int sign() const { return mag_.empty() ? 0 : (neg_ ? -1 : 1); }

  bool fits_i64() const {
    if (mag_.size() > 2) return false;
    uint64_t m = to_u64_mag();
    return neg_ ? m <= (uint64_t)1 << 63 : m < (uint64_t)1 << 63;
  }
  int64_t to_i64() const {
    uint64_t m = to_u64_mag();
    return neg_ ? (int64_t)((uint64_t)0 - m) : (int64_t)m;
  }

  friend BigInt operator-(const BigInt& a) {
    BigInt r = a;
    if (!r.mag_.empty()) r.neg_ = !r.neg_;
    return r;
  }
  friend BigInt operator+(const BigInt& a, const BigInt& b) {
    if (a.neg_ == b.neg_) return make(add_mag(a.mag_, b.mag_), a.neg_);
    int c = cmp_mag(a.mag_, b.mag_);
    if (c == 0) return BigInt();
    if (c > 0) return make(sub_mag(a.mag_, b.mag_), a.neg_);
    return make(sub_mag(b.mag_, a.mag_), b.neg_);
  }
  friend BigInt operator-(const BigInt& a, const BigInt& b) { return a + (-b); }
  friend BigInt operator*(const BigInt& a, const BigInt& b) {
    if (a.mag_.empty() || b.mag_.empty()) return BigInt();
    return make(mul_mag(a.mag_, b.mag_), a.neg_ != b.neg_);
  }
  friend bool operator==(const BigInt& a, const BigInt& b) {
    return a.neg_ == b.neg_ && a.mag_ == b.mag_;
  }
  friend bool operator<(const BigInt& a, const BigInt& b) { return compare(a, b) < 0; }
  friend bool operator>(const BigInt& a, const BigInt& b) { return compare(a, b) > 0; }

  static int compare(const BigInt& a, const BigInt& b) {
    int sa = a.sign(), sb = b.sign();
    if (sa != sb) return sa < sb ? -1 : 1;
    int c = cmp_mag(a.mag_, b.mag_);
    return sa >= 0 ? c : -c;
  }

  // Truncated division of magnitudes; quotient sign = product of signs,
  // remainder sign = sign of the dividend (C semantics).
  static void divmod_trunc(const BigInt& a, const BigInt& b, BigInt& q, BigInt& r) {
    if (b.mag_.empty()) throw std::domain_error("BigInt division by zero");
    std::vector<uint32_t> qm, rm;
    divmod_mag(a.mag_, b.mag_, qm, rm);
    q = make(std::move(qm), a.neg_ != b.neg_);
    r = make(std::move(rm), a.neg_);
  }
  // Exact division (the caller guarantees b divides a).
  static BigInt div_exact(const BigInt& a, const BigInt& b) {
    BigInt q, r;
    divmod_trunc(a, b, q, r);
    if (!r.is_zero()) throw std::logic_error("BigInt inexact division");
    return q;
  }
  // Nearest integer to a / b (b > 0), ties to even.
  static BigInt div_round_half_even(const BigInt& a, const BigInt& b) {
    BigInt q, r;
    divmod_trunc(a, b, q, r);
    if (r.is_neg()) {  // make floor division: r in [0, b)
      q = q - BigInt(1);
      r = r + b;
    }
    BigInt twice = r + r;
    int c = compare(twice, b);
    if (c > 0 || (c == 0 && q.is_odd())) q = q + BigInt(1);
    return q;
  }
  bool is_odd() const { return !mag_.empty() && (mag_[0] & 1u); }

 private:
  bool neg_ = false;
  std::vector<uint32_t> mag_;

  uint64_t to_u64_mag() const {
    uint64_t m = 0;
    if (mag_.size() > 0) m |= mag_[0];
    if (mag_.size() > 1) m |= (uint64_t)mag_[1] << 32;
    return m;
  }
  static void trim(std::vector<uint32_t>& v) {
    while (!v.empty() && v.back() == 0) v.pop_back();
  }
  static BigInt make(std::vector<uint32_t> m, bool neg) {
    BigInt r;
    trim(m);
    r.mag_ = std::move(m);
    r.neg_ = r.mag_.empty() ? false : neg;
    return r;
  }
  static int cmp_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;)
      if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
  }
  static std::vector<uint32_t> add_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    const std::vector<uint32_t>& x = a.size() >= b.size() ? a : b;
    const std::vector<uint32_t>& y = a.size() >= b.size() ? b : a;
    std::vector<uint32_t> r(x.size() + 1);
    uint64_t carry = 0;
    for (size_t i = 0; i < x.size(); ++i) {
      uint64_t s = (uint64_t)x[i] + (i < y.size() ? y[i] : 0) + carry;
      r[i] = (uint32_t)s;
      carry = s >> 32;
    }
    r[x.size()] = (uint32_t)carry;
    return r;
  }
  static std::vector<uint32_t> sub_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    // requires |a| >= |b|
    std::vector<uint32_t> r(a.size());
    int64_t borrow = 0;
    for (size_t i = 0; i < a.size(); ++i) {
      int64_t s = (int64_t)a[i] - (i < b.size() ? (int64_t)b[i] : 0) - borrow;
      borrow = s < 0;
      r[i] = (uint32_t)(s + (borrow << 32));
    }
    return r;
  }
  static std::vector<uint32_t> mul_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    std::vector<uint32_t> r(a.size() + b.size(), 0);
    for (size_t i = 0; i < a.size(); ++i) {
      uint64_t carry = 0;
      for (size_t j = 0; j < b.size(); ++j) {
        uint64_t t = (uint64_t)a[i] * b[j] + r[i + j] + carry;
        r[i + j] = (uint32_t)t;
        carry = t >> 32;
      }
      size_t k = i + b.size();
      while (carry) {
        uint64_t t = (uint64_t)r[k] + carry;
        r[k] = (uint32_t)t;
        carry = t >> 32;
        ++k;
      }
    }
    return r;
  }
  // Knuth Algorithm D on magnitudes: u = q v + r, 0 <= r < v.
  static void divmod_mag(const std::vector<uint32_t>& u_in, const std::vector<uint32_t>& v_in,
                         std::vector<uint32_t>& q, std::vector<uint32_t>& r) {
    std::vector<uint32_t> u = u_in, v = v_in;
    trim(u);
    trim(v);
    if (cmp_mag(u, v) < 0) {
      q.clear();
      r = u;
      return;
    }
    const size_t n = v.size(), m = u.size() - v.size();
    if (n == 1) {
      q.assign(u.size(), 0);
      uint64_t rem = 0;
      for (size_t i = u.size(); i-- > 0;) {
        uint64_t cur = (rem << 32) | u[i];
        q[i] = (uint32_t)(cur / v[0]);
        rem = cur % v[0];
      }
      r.assign(1, (uint32_t)rem);
      trim(q);
      trim(r);
      return;
    }
    const int s = __builtin_clz(v[n - 1]);
    std::vector<uint32_t> vn(n), un(u.size() + 1);
    for (size_t i = n - 1; i > 0; --i)
      vn[i] = (v[i] << s) | (s ? (uint32_t)((uint64_t)v[i - 1] >> (32 - s)) : 0);
    vn[0] = v[0] << s;
    un[u.size()] = s ? (uint32_t)((uint64_t)u[u.size() - 1] >> (32 - s)) : 0;
    for (size_t i = u.size() - 1; i > 0; --i)
      un[i] = (u[i] << s) | (s ? (uint32_t)((uint64_t)u[i - 1] >> (32 - s)) : 0);
    un[0] = u[0] << s;
    q.assign(m + 1, 0);
    const uint64_t B = (uint64_t)1 << 32;
    for (size_t jj = m + 1; jj-- > 0;) {
      const size_t j = jj;
      uint64_t num = ((uint64_t)un[j + n] << 32) | un[j + n - 1];
      uint64_t qhat = num / vn[n - 1];
      uint64_t rhat = num % vn[n - 1];
      while (qhat >= B || qhat * vn[n - 2] > ((rhat << 32) | un[j + n - 2])) {
        qhat -= 1;
        rhat += vn[n - 1];
        if (rhat >= B) break;
      }
      int64_t borrow = 0;
      uint64_t carry = 0;
      for (size_t i = 0; i < n; ++i) {
        uint64_t p = qhat * vn[i] + carry;
        carry = p >> 32;
        int64_t t = (int64_t)un[i + j] - borrow - (int64_t)(p & 0xFFFFFFFFu);
        un[i + j] = (uint32_t)t;
        borrow = t < 0 ? 1 : 0;
      }
      int64_t t = (int64_t)un[j + n] - borrow - (int64_t)carry;
      un[j + n] = (uint32_t)t;
      if (t < 0) {  // add back
        qhat -= 1;
        uint64_t c = 0;
        for (size_t i = 0; i < n; ++i) {
          uint64_t s2 = (uint64_t)un[i + j] + vn[i] + c;
          un[i + j] = (uint32_t)s2;
          c = s2 >> 32;
        }
        un[j + n] = (uint32_t)((uint64_t)un[j + n] + c);
      }
      q[j] = (uint32_t)qhat;
    }
    r.assign(n, 0);
    for (size_t i = 0; i < n; ++i)
      r[i] = (un[i] >> s) | (s ? (uint32_t)((uint64_t)un[i + 1] << (32 - s)) : 0);
    trim(q);
    trim(r);
  }
};

}  // namespace graver
