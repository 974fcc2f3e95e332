// hostbig.hpp - the library's host-side big integers, used once per plan to
// derive constants (Montgomery -q^-1 mod 2^32, R mod q, R^2 mod q, Barrett mu,
// omega^-1, n^-1, twiddle ladders).  Not on the hot path: simple shift-subtract
// division and square-and-multiply are enough.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

namespace moma {

class HBig {
 public:
  std::vector<uint32_t> w;  // little-endian limbs, no trailing zero limbs

  HBig() {}
  explicit HBig(uint64_t v) {
    if (v) w.push_back((uint32_t)v);
    if (v >> 32) w.push_back((uint32_t)(v >> 32));
  }
  static HBig from_limbs(const uint32_t* p, int n) {
    HBig r;
    r.w.assign(p, p + n);
    r.trim();
    return r;
  }
  void to_limbs(uint32_t* p, int n) const {
    for (int i = 0; i < n; i++) p[i] = i < (int)w.size() ? w[i] : 0;
  }
  void trim() {
    while (!w.empty() && w.back() == 0) w.pop_back();
  }
  bool is_zero() const { return w.empty(); }
  bool is_odd() const { return !w.empty() && (w[0] & 1); }
  int bitlen() const {
    if (w.empty()) return 0;
    return 32 * ((int)w.size() - 1) + (32 - __builtin_clz(w.back()));
  }
  bool bit(int i) const {
    int k = i / 32;
    return k < (int)w.size() && ((w[k] >> (i % 32)) & 1);
  }
  static int cmp(const HBig& a, const HBig& b) {
    if (a.w.size() != b.w.size()) return a.w.size() < b.w.size() ? -1 : 1;
    for (int i = (int)a.w.size() - 1; i >= 0; i--)
      if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
  }
  static HBig add(const HBig& a, const HBig& b) {
    HBig r;
    size_t n = std::max(a.w.size(), b.w.size());
    r.w.resize(n + 1);
    uint64_t c = 0;
    for (size_t i = 0; i < n; i++) {
      c += (uint64_t)(i < a.w.size() ? a.w[i] : 0) + (i < b.w.size() ? b.w[i] : 0);
      r.w[i] = (uint32_t)c;
      c >>= 32;
    }
    r.w[n] = (uint32_t)c;
    r.trim();
    return r;
  }
  // a - b, requires a >= b
  static HBig sub(const HBig& a, const HBig& b) {
    HBig r;
    r.w.resize(a.w.size());
    int64_t br = 0;
    for (size_t i = 0; i < a.w.size(); i++) {
      int64_t t = (int64_t)a.w[i] - (i < b.w.size() ? b.w[i] : 0) - br;
      br = t < 0;
      r.w[i] = (uint32_t)t;
    }
    r.trim();
    return r;
  }
  static HBig mul(const HBig& a, const HBig& b) {
    HBig r;
    if (a.is_zero() || b.is_zero()) return r;
    r.w.assign(a.w.size() + b.w.size(), 0);
    for (size_t i = 0; i < a.w.size(); i++) {
      uint64_t c = 0;
      for (size_t j = 0; j < b.w.size(); j++) {
        c += (uint64_t)a.w[i] * b.w[j] + r.w[i + j];
        r.w[i + j] = (uint32_t)c;
        c >>= 32;
      }
      r.w[i + b.w.size()] = (uint32_t)c;
    }
    r.trim();
    return r;
  }
  static HBig shl(const HBig& a, int s) {
    if (a.is_zero()) return a;
    HBig r;
    int ws = s / 32, bs = s % 32;
    r.w.assign(a.w.size() + ws + 1, 0);
    for (size_t i = 0; i < a.w.size(); i++) {
      uint64_t v = (uint64_t)a.w[i] << bs;
      r.w[i + ws] |= (uint32_t)v;
      r.w[i + ws + 1] |= (uint32_t)(v >> 32);
    }
    r.trim();
    return r;
  }
  static HBig shr(const HBig& a, int s) {
    HBig r;
    int ws = s / 32, bs = s % 32;
    if (ws >= (int)a.w.size()) return r;
    r.w.assign(a.w.size() - ws, 0);
    for (size_t i = 0; i < r.w.size(); i++) {
      uint64_t lo = a.w[i + ws];
      uint64_t hi = i + ws + 1 < a.w.size() ? a.w[i + ws + 1] : 0;
      r.w[i] = (uint32_t)(((hi << 32) | lo) >> bs);
    }
    r.trim();
    return r;
  }
  static HBig pow2(int e) { return shl(HBig(1), e); }
  // quotient and remainder by shift-subtract long division, one bit at a time
  static void divmod(const HBig& a, const HBig& b, HBig* quo, HBig* rem) {
    HBig q, r;
    int nb = a.bitlen();
    if (quo) q.w.assign((nb + 31) / 32 + 1, 0);
    for (int i = nb - 1; i >= 0; i--) {
      r = shl(r, 1);
      if (a.bit(i)) {
        if (r.w.empty()) r.w.push_back(0);
        r.w[0] |= 1;
      }
      if (cmp(r, b) >= 0) {
        r = sub(r, b);
        if (quo) q.w[i / 32] |= 1u << (i % 32);
      }
    }
    if (quo) {
      q.trim();
      *quo = q;
    }
    if (rem) *rem = r;
  }
  static HBig mod(const HBig& a, const HBig& m) {
    HBig r;
    divmod(a, m, nullptr, &r);
    return r;
  }
  static HBig mulmod(const HBig& a, const HBig& b, const HBig& m) { return mod(mul(a, b), m); }
  static HBig powmod(const HBig& a, const HBig& e, const HBig& m) {
    HBig r = mod(HBig(1), m), base = mod(a, m);
    for (int i = e.bitlen() - 1; i >= 0; i--) {
      r = mulmod(r, r, m);
      if (e.bit(i)) r = mulmod(r, base, m);
    }
    return r;
  }
  std::string hex() const {
    static const char* d = "0123456789abcdef";
    if (w.empty()) return "0x0";
    std::string s;
    for (int i = (int)w.size() - 1; i >= 0; i--)
      for (int k = 7; k >= 0; k--) s.push_back(d[(w[i] >> (4 * k)) & 15]);
    size_t nz = s.find_first_not_of('0');
    return "0x" + s.substr(nz);
  }
};

// -q^{-1} mod 2^32 for odd q0 (Newton iteration: each step doubles the correct bits)
inline uint32_t neg_inv32(uint32_t q0) {
  uint32_t x = q0;  // correct to 3 bits for odd q0
  for (int i = 0; i < 5; i++) x *= 2u - q0 * x;
  return 0u - x;
}

}  // namespace moma
