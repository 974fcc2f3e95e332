// limb.hpp - device-side multi-word modular arithmetic on 32-bit limbs (gfx950).
//
// A residue is L little-endian 32-bit limbs held in VGPRs (one lane = one
// element).  The modulus and its constants are uniform per launch and live in
// SGPRs (kernel arguments), so every word product has one SGPR operand.
//
// The paper decomposes a 2w-bit operation into w-bit operations recursively
// (Section 3, Table 1).  On gfx950 the machine word is the 32-bit VGPR lane,
// and the recursion is flattened into straight L-limb loops, unrolled at
// compile time (L is a template parameter), so no intermediate word size is
// materialised:
//   * add / subtract with carry and borrow chains (Section 2.2, rules (adc),
//     (addqdd), (subddd)) map to v_add_co_u32 / v_addc_co_u32 and
//     v_sub_co_u32 / v_subb_co_u32, with the carry bit delta held as a
//     64-bit lane mask in an SGPR pair;
//   * the conditional selects of Eqs. (saddmod) / (ssubmod) and rule
//     (moddq_add) map to v_cndmask_b32 on that mask;
//   * each 32x32->64 word product plus accumulation (rule (mulqdd)) is one
//     v_mad_u64_u32, whose carry-out feeds a third accumulator word through
//     one v_addc_co_u32 (product scanning, one column at a time).
// The instructions are written as small inline-asm statements because the
// compiler does not use the carry-out of v_mad_u64_u32 on its own; carries
// between statements travel in named SGPR-pair variables, never in VCC.
// gfx950 allows one constant-bus (SGPR) read per VALU instruction and the
// carry-in already uses it, so chained limbs take the modulus from a VGPR copy.
//
// Comparisons are canonical (>= q subtracts), not the strict comparisons
// printed in Eq. (saddmod) and Listing 1, so every output lies in [0, q).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace moma {

typedef uint32_t u32;
typedef uint64_t u64;

// A pointer that a kernel reads from memory (a batch record) is generic to the
// compiler, which then accesses it with flat loads and stores.  Those count on
// the LDS wait counter as well, so every wait for an LDS access also waits for
// the HBM accesses in flight.  The records hold device global addresses:
// reading the field as a global-space pointer lets the compiler use global
// loads and stores wherever the pointer goes.
template <class T>
__device__ __forceinline__ T* load_global_ptr(T* const* slot) {
  typedef __attribute__((address_space(1))) T* GlobalPtr;
  return (T*)*static_cast<const GlobalPtr*>(static_cast<const void*>(slot));
}

// ----------------------------------------------------------------- word ops

// acc(64) += x * y; hi += carry-out.  x in a VGPR, y in a VGPR.
__device__ __forceinline__ void mac_vv(u64& acc, u32& hi, u32 x, u32 y) {
  u64 cy;
  asm("v_mad_u64_u32 %0, %1, %3, %4, %0\n\t"
      "v_addc_co_u32 %2, %1, %2, 0, %1"
      : "+v"(acc), "=&s"(cy), "+v"(hi)
      : "v"(x), "v"(y));
}

// acc(64) += x * y; hi += carry-out.  x in a VGPR, y uniform (SGPR).
__device__ __forceinline__ void mac_vs(u64& acc, u32& hi, u32 x, u32 y) {
  u64 cy;
  asm("v_mad_u64_u32 %0, %1, %3, %4, %0\n\t"
      "v_addc_co_u32 %2, %1, %2, 0, %1"
      : "+v"(acc), "=&s"(cy), "+v"(hi)
      : "v"(x), "s"(y));
}

// acc(64) += x1 * y1 + x2 * y2 with carries into hi; x in VGPRs, y1 VGPR, y2 uniform.
// One asm statement for two products halves the wait states the compiler
// inserts after every inline-asm block.
__device__ __forceinline__ void mac2_vv_vs(u64& acc, u32& hi, u32 x1, u32 y1, u32 x2, u32 y2) {
  u64 cy;
  asm("v_mad_u64_u32 %0, %1, %3, %4, %0\n\t"
      "v_addc_co_u32 %2, %1, %2, 0, %1\n\t"
      "v_mad_u64_u32 %0, %1, %5, %6, %0\n\t"
      "v_addc_co_u32 %2, %1, %2, 0, %1"
      : "+v"(acc), "=&s"(cy), "+v"(hi)
      : "v"(x1), "v"(y1), "v"(x2), "s"(y2));
}

// First products of a column: hi = carry-out (instead of hi += carry-out), so the
// carry word needs no zeroing move.
__device__ __forceinline__ void mac2_vv_vs_first(u64& acc, u32& hi, u32 x1, u32 y1, u32 x2, u32 y2) {
  u64 cy;
  asm("v_mad_u64_u32 %0, %1, %3, %4, %0\n\t"
      "v_addc_co_u32 %2, %1, 0, 0, %1\n\t"
      "v_mad_u64_u32 %0, %1, %5, %6, %0\n\t"
      "v_addc_co_u32 %2, %1, %2, 0, %1"
      : "+v"(acc), "=&s"(cy), "=&v"(hi)
      : "v"(x1), "v"(y1), "v"(x2), "s"(y2));
}

__device__ __forceinline__ void mac_vv_first(u64& acc, u32& hi, u32 x, u32 y) {
  u64 cy;
  asm("v_mad_u64_u32 %0, %1, %3, %4, %0\n\t"
      "v_addc_co_u32 %2, %1, 0, 0, %1"
      : "+v"(acc), "=&s"(cy), "=&v"(hi)
      : "v"(x), "v"(y));
}

// acc(64) += x * y with no carry-out (caller guarantees no overflow).
__device__ __forceinline__ void mad_vv(u64& acc, u32 x, u32 y) {
  u64 cy;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc), "=s"(cy) : "v"(x), "v"(y));
}

// move the 96-bit column accumulator one word down: {acc, hi} >>= 32
__device__ __forceinline__ void shift_col(u64& acc, u32& hi) {
  acc = (acc >> 32) | ((u64)hi << 32);
  hi = 0;
}

// r = a + b over L limbs (a, b VGPR); returns the carry-out lane mask
template <int L>
__device__ __forceinline__ u64 add_vv(u32* r, const u32* a, const u32* b) {
  u64 cy;
  asm("v_add_co_u32 %0, %1, %2, %3" : "=v"(r[0]), "=s"(cy) : "v"(a[0]), "v"(b[0]));
#pragma unroll
  for (int i = 1; i < L; i++) asm("v_addc_co_u32 %0, %1, %2, %3, %1" : "=v"(r[i]), "+s"(cy) : "v"(a[i]), "v"(b[i]));
  return cy;
}

// r = a + q over L limbs (q uniform); returns the carry-out lane mask
template <int L>
__device__ __forceinline__ u64 add_vs(u32* r, const u32* a, const u32* q) {
  u64 cy;
  asm("v_add_co_u32 %0, %1, %2, %3" : "=v"(r[0]), "=s"(cy) : "v"(a[0]), "s"(q[0]));
#pragma unroll
  for (int i = 1; i < L; i++) asm("v_addc_co_u32 %0, %1, %2, %3, %1" : "=v"(r[i]), "+s"(cy) : "v"(a[i]), "v"(q[i]));
  return cy;
}

// r = a - b over L limbs (a, b VGPR); returns the borrow-out lane mask
template <int L>
__device__ __forceinline__ u64 sub_vv(u32* r, const u32* a, const u32* b) {
  u64 br;
  asm("v_sub_co_u32 %0, %1, %2, %3" : "=v"(r[0]), "=s"(br) : "v"(a[0]), "v"(b[0]));
#pragma unroll
  for (int i = 1; i < L; i++) asm("v_subb_co_u32 %0, %1, %2, %3, %1" : "=v"(r[i]), "+s"(br) : "v"(a[i]), "v"(b[i]));
  return br;
}

// r = a - q over L limbs (q uniform); returns the borrow-out lane mask
template <int L>
__device__ __forceinline__ u64 sub_vs(u32* r, const u32* a, const u32* q) {
  u64 br;
  asm("v_sub_co_u32 %0, %1, %2, %3" : "=v"(r[0]), "=s"(br) : "v"(a[0]), "s"(q[0]));
#pragma unroll
  for (int i = 1; i < L; i++) asm("v_subb_co_u32 %0, %1, %2, %3, %1" : "=v"(r[i]), "+s"(br) : "v"(a[i]), "v"(q[i]));
  return br;
}

// r[i] = mask ? x[i] : y[i] per lane
template <int L>
__device__ __forceinline__ void select(u32* r, u64 mask, const u32* x, const u32* y) {
#pragma unroll
  for (int i = 0; i < L; i++) asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r[i]) : "v"(y[i]), "v"(x[i]), "s"(mask));
}

// ----------------------------------------------------------------- modular ops

// r = (a + b) mod q for a, b in [0, q), q < 2^(32L-1): sum, trial subtraction, select.
template <int L>
__device__ __forceinline__ void mod_add(u32* r, const u32* a, const u32* b, const u32* q) {
  u32 s[L], d[L];
  add_vv<L>(s, a, b);            // no carry-out: a + b < 2q < 2^(32L)
  u64 br = sub_vs<L>(d, s, q);   // borrow set  <=>  s < q
  select<L>(r, br, s, d);
}

// r = (a - b) mod q for a, b in [0, q): difference, add q back where it borrowed.
template <int L>
__device__ __forceinline__ void mod_sub(u32* r, const u32* a, const u32* b, const u32* q) {
  u32 d[L], e[L];
  u64 br = sub_vv<L>(d, a, b);
  add_vs<L>(e, d, q);
  select<L>(r, br, e, d);
}

// r = x mod q for x in [0, 2q): one trial subtraction.
template <int L>
__device__ __forceinline__ void reduce_once(u32* r, const u32* x, const u32* q) {
  u32 d[L];
  u64 br = sub_vs<L>(d, x, q);
  select<L>(r, br, x, d);
}

// Montgomery product t = a * b * 2^(-32L) (mod q), left in [0, 2q) (Montgomery,
// Math. Comp. 1985), product-scanning form: column i accumulates every a_j*b_{i-j}
// and m_j*q_{i-j}, then m_i = (column low word) * (-q^-1 mod 2^32) zeroes the low
// word.  Requires a*b < 4q^2 (e.g. a < 4q, b < q) and 4q <= 2^(32L); then
// t = (ab + mq) / 2^(32L) < 2q.  qinv = -q^{-1} mod 2^32.
// 2L^2 + L word products (as counted for Montgomery multiplication).
template <int L>
__device__ __forceinline__ void mont_mul_lazy(u32* t, const u32* a, const u32* b, const u32* q, u32 qinv) {
  u32 m[L];
  u64 acc = 0;
  u32 hi;
#pragma unroll
  for (int i = 0; i < L; i++) {
    if (i == 0) {
      mac_vv_first(acc, hi, a[0], b[0]);
    } else {
      mac2_vv_vs_first(acc, hi, a[0], b[i], m[0], q[i]);
#pragma unroll
      for (int j = 1; j < i; j++) mac2_vv_vs(acc, hi, a[j], b[i - j], m[j], q[i - j]);
      mac_vv(acc, hi, a[i], b[0]);
    }
    m[i] = (u32)acc * qinv;
    mac_vs(acc, hi, m[i], q[0]);
    acc = (acc >> 32) | ((u64)hi << 32);
  }
#pragma unroll
  for (int i = L; i < 2 * L; i++) {
    if (i - L + 1 < L) {
      mac2_vv_vs_first(acc, hi, a[i - L + 1], b[L - 1], m[i - L + 1], q[L - 1]);
#pragma unroll
      for (int j = i - L + 2; j < L; j++) mac2_vv_vs(acc, hi, a[j], b[i - j], m[j], q[i - j]);
      t[i - L] = (u32)acc;
      acc = (acc >> 32) | ((u64)hi << 32);
    } else {
      t[i - L] = (u32)acc;  // last column: no products left, only the carried word
    }
  }
  // t < 2q < 2^(32L): the final carry word is zero
}

// Montgomery product reduced to [0, q): a, b in [0, q).
template <int L>
__device__ __forceinline__ void mont_mul(u32* r, const u32* a, const u32* b, const u32* q, u32 qinv) {
  u32 t[L];
  mont_mul_lazy<L>(t, a, b, q, qinv);
  reduce_once<L>(r, t, q);
}

// ----------------------------------------------------------------- digit form
//
// The paper's multi-digit numbers may use any digit base z (Eq. (def_mp)).  For
// the transform's twiddle multiply, residues are re-expressed in base 2^b with
// b = 29 (28 above 28 limbs) and D digits, chosen so that a column of 2D digit
// products plus the carried word stays below 2^64.  Every word product is then
// one v_mad_u64_u32 into a 64-bit accumulator with no carry handling, which the
// compiler emits from plain C.  Operands stay in 32-bit limbs everywhere else;
// the multiply converts on the way in and out.
template <int L, bool FW = false>
struct Digits {
  static constexpr int b = digit_bits(L);
  static constexpr int D = digit_count(L, FW);
  static constexpr u32 mask = (1u << b) - 1;
};

// d = y in base 2^b (y < 2^(b*D))
template <int L, bool FW = false>
__device__ __forceinline__ void to_digits(u32* d, const u32* y) {
  constexpr int b = Digits<L, FW>::b, D = Digits<L, FW>::D;
#pragma unroll
  for (int i = 0; i < D; i++) {
    constexpr u32 m = Digits<L, FW>::mask;
    const int pos = b * i, l = pos / 32, s = pos % 32;
    u32 lo = l < L ? y[l] : 0u, hi = l + 1 < L ? y[l + 1] : 0u;
    u32 v = s ? __builtin_amdgcn_alignbit(hi, lo, s) : lo;
    d[i] = v & m;
  }
}

// y = the value of digits d, as L 32-bit limbs (the value fits 32L bits)
template <int L, bool FW = false>
__device__ __forceinline__ void from_digits(u32* y, const u32* d) {
  constexpr int b = Digits<L, FW>::b, D = Digits<L, FW>::D;
#pragma unroll
  for (int j = 0; j < L; j++) {
    const int pos = 32 * j, i = pos / b, s = pos % b;
    u32 v = d[i] >> s;
    if (i + 1 < D && b - s < 32) v |= d[i + 1] << (b - s);
    if (i + 2 < D && 2 * b - s < 32) v |= d[i + 2] << (2 * b - s);
    y[j] = v;
  }
}

// t = y * w * 2^(-bD) mod q in [0, 2q), w given as digits (Montgomery form for
// R = 2^(bD)), y < 4q in 32-bit limbs (y < q for a full-width modulus, FW).
// Product scanning: column i sums every digit product y_j w_{i-j} and
// m_j q_{i-j}; m_i = (low b bits) * qinvd mod 2^b clears the low b bits, then
// the column shifts right by b.  2D^2 products.  FW: the result may reach
// 2^(32L); *top receives its bit 32L (0 or 1).
template <int L, bool FW = false>
__device__ __forceinline__ void mont_mul_digits(u32* t, const u32* y, const u32* wd, const u32* qd, u32 qinvd,
                                                u32* top = nullptr) {
  constexpr int b = Digits<L, FW>::b, D = Digits<L, FW>::D;
  constexpr u32 mask = Digits<L, FW>::mask;
  static_assert(b * D >= 32 * L - (FW ? 0 : 2), "the digits cover the result limbs");
  u32 a[D], m[D];
  to_digits<L, FW>(a, y);
  u64 acc = 0;
#pragma unroll
  for (int i = 0; i < D; i++) {
#pragma unroll
    for (int j = 0; j <= i; j++) acc += (u64)a[j] * wd[i - j];
#pragma unroll
    for (int j = 0; j < i; j++) acc += (u64)m[j] * qd[i - j];
    m[i] = ((u32)acc * qinvd) & mask;
    acc += (u64)m[i] * qd[0];
    acc >>= b;
  }
  // the upper columns give the result digits; each result limb leaves as soon
  // as its 32 bits are known (digit positions are compile-time constants), so
  // the digits are never all live at once
  u64 bits = 0;
  int nb = 0, j = 0;
#pragma unroll
  for (int i = D; i < 2 * D; i++) {
    u32 dig;
    if (i < 2 * D - 1) {
#pragma unroll
      for (int jj = i - D + 1; jj < D; jj++) acc += (u64)a[jj] * wd[i - jj] + (u64)m[jj] * qd[i - jj];
      dig = (u32)acc & mask;
      acc >>= b;
    } else {
      dig = (u32)acc;  // the last digit carries everything above
    }
    bits |= (u64)dig << nb;
    nb += b;
    while (nb >= 32 && j < L) {
      t[j++] = (u32)bits;
      bits >>= 32;
      nb -= 32;
    }
  }
  // bD is at least 32L - 2 (at least 32L for a full-width modulus), so at most
  // the top limb is still in the buffer here: its bits above bD come from the
  // last digit, which is wider than b
  if (j < L) t[j] = (u32)bits;
  if constexpr (FW) *top = (u32)bits;  // bit 32L of a full-width result below 2q
}

// The same product with its first half (the digit product y w) by one level
// of Karatsuba (Eq. (mulk)) on the digits: with y = y1 B^h + y0 and
// w = w1 B^h + w0 (B = 2^b, h = ceil(D/2)), y w = z2 B^(2h) + z1 B^h + z0 where
// z1 = (y0 + y1)(w0 + w1) - z0 - z2.  The digit sums have b + 1 bits and need
// no carry; every product column is gathered as an exact 64-bit sum (it
// equals the schoolbook column, below D 2^(2b)), so the Montgomery
// reduction that follows is unchanged.  Word products: 2h^2 + (D - h)^2
// instead of D^2, for 2D - 1 extra column additions and 2h - 1 column
// subtractions.
template <int L>
__device__ __forceinline__ void mont_mul_digits_kara(u32* t, const u32* y, const u32* wd, const u32* qd, u32 qinvd) {
  constexpr int b = Digits<L>::b, D = Digits<L>::D, h = (D + 1) / 2, g = D - h;
  constexpr u32 mask = Digits<L>::mask;
  u32 a[D], m[D], r[D], sa[h], sw[h];
  to_digits<L>(a, y);
#pragma unroll
  for (int i = 0; i < h; i++) {
    sa[i] = a[i] + (i < g ? a[h + i] : 0u);
    sw[i] = wd[i] + (i < g ? wd[h + i] : 0u);
  }
  u64 p[2 * D - 1];
#pragma unroll
  for (int c = 0; c < 2 * D - 1; c++) p[c] = 0;
#pragma unroll
  for (int c = 0; c < 2 * h - 1; c++) {
    u64 z0 = 0, zm = 0, z2 = 0;
#pragma unroll
    for (int i = (c < h ? 0 : c - h + 1); i <= (c < h ? c : h - 1); i++) {
      z0 += (u64)a[i] * wd[c - i];
      zm += (u64)sa[i] * sw[c - i];
    }
    if (c <= 2 * g - 2) {
#pragma unroll
      for (int i = (c < g ? 0 : c - g + 1); i <= (c < g ? c : g - 1); i++) z2 += (u64)a[h + i] * wd[h + c - i];
      p[c + 2 * h] += z2;
    }
    p[c] += z0;
    p[c + h] += zm - z0 - z2;  // the cross terms: exact, non-negative
  }
  u64 acc = 0;
#pragma unroll
  for (int i = 0; i < D; i++) {
    acc += p[i];
#pragma unroll
    for (int j = 0; j < i; j++) acc += (u64)m[j] * qd[i - j];
    m[i] = ((u32)acc * qinvd) & mask;
    acc += (u64)m[i] * qd[0];
    acc >>= b;
  }
#pragma unroll
  for (int i = D; i < 2 * D - 1; i++) {
    acc += p[i];
#pragma unroll
    for (int j = i - D + 1; j < D; j++) acc += (u64)m[j] * qd[i - j];
    r[i - D] = (u32)acc & mask;
    acc >>= b;
  }
  r[D - 1] = (u32)acc;
  from_digits<L>(t, r);
}

// Lazy butterfly with the Karatsuba form of the twiddle multiply.
template <int L>
__device__ __forceinline__ void ct_butterfly_kara(u32* x, u32* y, const u32* wd, const u32* qd, u32 qinvd,
                                                  const u32* q2v) {
  u32 xr[L], t[L], d[L], s[L];
  u64 br = sub_vv<L>(s, x, q2v);  // x - 2q; borrow <=> x < 2q
  select<L>(xr, br, x, s);
  mont_mul_digits_kara<L>(t, y, wd, qd, qinvd);
  add_vv<L>(x, xr, t);
  sub_vv<L>(d, xr, t);
  add_vv<L>(y, d, q2v);
}

// ----------------------------------------------------------------- full width
//
// A full-width modulus (bitlen(q) > 32L - 4) leaves no headroom for the lazy
// reductions: operands stay canonical in [0, q), and a sum or a Montgomery
// product below 2q can carry out of the top limb, so that bit travels in a
// word of its own beside the L limbs (Section 5.2 names Montgomery
// multiplication for such moduli).

// r = (top 2^(32L) + t) mod q for a value below 2q (top in {0, 1}): the
// (L+1)-word trial subtraction's final borrow says whether the value is < q.
template <int L>
__device__ __forceinline__ void reduce_top(u32* r, const u32* t, u32 top, const u32* qv) {
  u32 d[L], dt;
  u64 br = sub_vv<L>(d, t, qv);
  asm("v_subb_co_u32 %0, %1, %2, 0, %1" : "=v"(dt), "+s"(br) : "v"(top));
  select<L>(r, br, t, d);
}

// r = (a + b) mod q for a, b in [0, q), q < 2^(32L) (the sum may carry out)
template <int L>
__device__ __forceinline__ void mod_add_fw(u32* r, const u32* a, const u32* b, const u32* qv) {
  u32 s[L], top;
  u64 cy = add_vv<L>(s, a, b);
  asm("v_addc_co_u32 %0, %1, 0, 0, %1" : "=v"(top), "+s"(cy));
  reduce_top<L>(r, s, top, qv);
}

// r = (a - b) mod q for a, b in [0, q): the difference wraps below zero by
// exactly 2^(32L), which adding q takes back (no headroom needed)
template <int L>
__device__ __forceinline__ void mod_sub_v(u32* r, const u32* a, const u32* b, const u32* qv) {
  u32 d[L], e[L];
  u64 br = sub_vv<L>(d, a, b);
  add_vv<L>(e, d, qv);
  select<L>(r, br, e, d);
}

// Canonical butterfly for a full-width modulus: x, y in [0, q), twiddle in
// digit form; x' = (x + wy) mod q, y' = (x - wy) mod q.
template <int L>
__device__ __forceinline__ void ct_butterfly_fw(u32* x, u32* y, const u32* wd, const u32* qd, u32 qinvd,
                                                const u32* qv) {
  u32 t[L], tr[L], top;
  mont_mul_digits<L, true>(t, y, wd, qd, qinvd, &top);
  reduce_top<L>(tr, t, top, qv);
  u32 s[L], d[L];
#pragma unroll
  for (int j = 0; j < L; j++) s[j] = x[j];
  mod_add_fw<L>(x, s, tr, qv);
  mod_sub_v<L>(d, s, tr, qv);
#pragma unroll
  for (int j = 0; j < L; j++) y[j] = d[j];
}

// The same with twiddle 1: (x + y, x - y) mod q.
template <int L>
__device__ __forceinline__ void ct_butterfly_one_fw(u32* x, u32* y, const u32* qv) {
  u32 s[L], d[L];
#pragma unroll
  for (int j = 0; j < L; j++) s[j] = x[j];
  mod_add_fw<L>(x, s, y, qv);
  mod_sub_v<L>(d, s, y, qv);
#pragma unroll
  for (int j = 0; j < L; j++) y[j] = d[j];
}

// Montgomery product for a full-width modulus, 32-bit limbs (the form of
// mont_mul_lazy): t = a b 2^(-32L) mod q in [0, q) for a, b in [0, q).  The
// value (ab + mq) / 2^(32L) < 2q may reach 2^(32L); its carry word is kept and
// folded into the final trial subtraction.
template <int L>
__device__ __forceinline__ void mont_mul_fw(u32* r, const u32* a, const u32* b, const u32* q, u32 qinv,
                                            const u32* qv) {
  u32 m[L], t[L];
  u64 acc = 0;
  u32 hi;
#pragma unroll
  for (int i = 0; i < L; i++) {
    if (i == 0) {
      mac_vv_first(acc, hi, a[0], b[0]);
    } else {
      mac2_vv_vs_first(acc, hi, a[0], b[i], m[0], q[i]);
#pragma unroll
      for (int j = 1; j < i; j++) mac2_vv_vs(acc, hi, a[j], b[i - j], m[j], q[i - j]);
      mac_vv(acc, hi, a[i], b[0]);
    }
    m[i] = (u32)acc * qinv;
    mac_vs(acc, hi, m[i], q[0]);
    acc = (acc >> 32) | ((u64)hi << 32);
  }
  u32 top = 0;
#pragma unroll
  for (int i = L; i < 2 * L; i++) {
    if (i - L + 1 < L) {
      mac2_vv_vs_first(acc, hi, a[i - L + 1], b[L - 1], m[i - L + 1], q[L - 1]);
#pragma unroll
      for (int j = i - L + 2; j < L; j++) mac2_vv_vs(acc, hi, a[j], b[i - j], m[j], q[i - j]);
      t[i - L] = (u32)acc;
      acc = (acc >> 32) | ((u64)hi << 32);
    } else {
      t[i - L] = (u32)acc;  // last column: only the carried words are left
      top = (u32)(acc >> 32);
    }
  }
  reduce_top<L>(r, t, top, qv);
}

// Copy uniform words into VGPRs once, opaquely, so carry chains that need the
// operand in a VGPR do not re-copy it from SGPRs at every use.
template <int L>
__device__ __forceinline__ void to_vgprs(u32* dst, const u32* src) {
#pragma unroll
  for (int i = 0; i < L; i++) asm volatile("v_mov_b32 %0, %1" : "=v"(dst[i]) : "s"(src[i]));
}

// Cooley-Tukey butterfly with lazy reduction (Harvey, "Faster arithmetic for
// number-theoretic transforms", J. Symb. Comp. 2014): inputs and outputs in
// [0, 4q), twiddle w < q in Montgomery form, q2 = 2q.
//   x <- x mod 2q;  t <- w*y in [0, 2q);  x' = x + t;  y' = x - t + 2q.
// Same residues as (x + wy, x - wy) mod q; 5L add-class ops instead of 8L.
template <int L>
__device__ __forceinline__ void ct_butterfly_lazy(u32* x, u32* y, const u32* w, const u32* q, const u32* q2,
                                                  u32 qinv) {
  u32 xr[L], t[L], d[L];
  reduce_once<L>(xr, x, q2);
  mont_mul_lazy<L>(t, y, w, q, qinv);
  add_vv<L>(x, xr, t);
  sub_vv<L>(d, xr, t);
  add_vs<L>(y, d, q2);
}

// Lazy butterfly with twiddle 1 (the first stages of a transform): the same
// residues as the multiplying butterfly, with t = y mod 2q in [0, 2q) in place
// of the Montgomery product w*y.
template <int L>
__device__ __forceinline__ void ct_butterfly_one(u32* x, u32* y, const u32* q2v) {
  u32 xr[L], t[L], d[L], s[L];
  u64 br = sub_vv<L>(s, x, q2v);
  select<L>(xr, br, x, s);
  br = sub_vv<L>(s, y, q2v);
  select<L>(t, br, y, s);
  add_vv<L>(x, xr, t);
  sub_vv<L>(d, xr, t);
  add_vv<L>(y, d, q2v);
}

// Lazy butterfly with the twiddle in digit form (mont_mul_digits) and 2q in VGPRs.
template <int L>
__device__ __forceinline__ void ct_butterfly_digits(u32* x, u32* y, const u32* wd, const u32* qd, u32 qinvd,
                                                    const u32* q2v) {
  u32 xr[L], t[L], d[L], s[L];
  u64 br = sub_vv<L>(s, x, q2v);  // x - 2q; borrow <=> x < 2q
  select<L>(xr, br, x, s);
  mont_mul_digits<L>(t, y, wd, qd, qinvd);
  add_vv<L>(x, xr, t);
  sub_vv<L>(d, xr, t);
  add_vv<L>(y, d, q2v);
}

// The same butterfly with 2q already in VGPRs (q2v); q stays uniform for the
// multiply's products.
template <int L>
__device__ __forceinline__ void ct_butterfly_lazy_v(u32* x, u32* y, const u32* w, const u32* q, const u32* q2v,
                                                    u32 qinv) {
  u32 xr[L], t[L], d[L], s[L];
  u64 br = sub_vv<L>(s, x, q2v);  // x - 2q; borrow <=> x < 2q
  select<L>(xr, br, x, s);
  mont_mul_lazy<L>(t, y, w, q, qinv);
  add_vv<L>(x, xr, t);
  sub_vv<L>(d, xr, t);
  add_vv<L>(y, d, q2v);
}

// The additions of the lazy butterfly once its product t = w*y in [0, 2q) is
// known: x <- x mod 2q; y = x - t + 2q; x = x + t.
template <int L>
__device__ __forceinline__ void ct_lazy_tail(u32* x, u32* y, const u32* t, const u32* q2v) {
  u32 xr[L], d[L], s[L];
  u64 br = sub_vv<L>(s, x, q2v);
  select<L>(xr, br, x, s);
  add_vv<L>(x, xr, t);
  sub_vv<L>(d, xr, t);
  add_vv<L>(y, d, q2v);
}

// The same for a full-width modulus: t (with its carry word) reduced, then
// (x + t, x - t) mod q.
template <int L>
__device__ __forceinline__ void ct_fw_tail(u32* x, u32* y, const u32* t, u32 top, const u32* qv) {
  u32 tr[L], s[L];
  reduce_top<L>(tr, t, top, qv);
#pragma unroll
  for (int j = 0; j < L; j++) s[j] = x[j];
  mod_add_fw<L>(x, s, tr, qv);
  mod_sub_v<L>(y, s, tr, qv);
}

// Barrett constants for r = a*b mod q, following Listings 1 and 4 generalised to
// L limbs.  The modulus is pre-scaled to qn = q * 2^d with bitlen(qn) = M = 32L-4,
// so the paper's shifts by M-2 and M+5 fall at fixed limb/bit positions:
// mu = floor(2^(2M+3) / qn) < 2^(M+4) = 2^(32L).
template <int L>
struct BarrettC {
  u32 qn[L];
  u32 mu[L];
  u32 d;
};

// t[0 .. M+N) = a[0 .. M) * b[0 .. N), product scanning, both operands in VGPRs
template <int M, int N>
__device__ __forceinline__ void mul_ps(u32* t, const u32* a, const u32* b) {
  u64 acc = 0;
  u32 hi = 0;
#pragma unroll
  for (int k = 0; k < M + N - 1; k++) {
#pragma unroll
    for (int i = (k < N ? 0 : k - N + 1); i <= (k < M ? k : M - 1); i++) mac_vv(acc, hi, a[i], b[k - i]);
    t[k] = (u32)acc;
    shift_col(acc, hi);
  }
  t[M + N - 1] = (u32)acc;
}

// t[0 .. 2L) = a * b by one level of Karatsuba (Eq. (mulk)), subtractive form:
// with a = a1 B^h + a0, b = b1 B^h + b0 (B = 2^32, h = ceil(L/2)),
//   a b = z2 B^(2h) + (z0 + z2 - s |a0 - a1| |b0 - b1|) B^h + z0,
//   z0 = a0 b0, z2 = a1 b1, s = sign((a0 - a1)(b0 - b1)).
// Three half-size products (3 ceil(L/2)^2 word products instead of L^2); the
// differences need no carry bit, at the price of the sign selects.
template <int L>
__device__ __forceinline__ void kara_mul(u32* t, const u32* a, const u32* b) {
  constexpr int h = (L + 1) / 2, g = L - h;  // a0, b0: h limbs; a1, b1: g <= h limbs
  u32 z0[2 * h], z2[2 * g], p[2 * h];
  mul_ps<h, h>(z0, a, b);
  mul_ps<g, g>(z2, a + h, b + h);
  u32 a1[h], b1[h], da[h], da2[h], db[h], db2[h];
#pragma unroll
  for (int i = 0; i < h; i++) {
    a1[i] = i < g ? a[h + i] : 0u;
    b1[i] = i < g ? b[h + i] : 0u;
  }
  u64 sa = sub_vv<h>(da, a, a1);  // borrow <=> a0 < a1
  sub_vv<h>(da2, a1, a);
  select<h>(da, sa, da2, da);
  u64 sb = sub_vv<h>(db, b, b1);
  sub_vv<h>(db2, b1, b);
  select<h>(db, sb, db2, db);
  mul_ps<h, h>(p, da, db);
  // mid = z0 + z2 -/+ p: a0 b1 + a1 b0 >= 0, at most 2h + 1 limbs
  constexpr int W = 2 * h + 1;
  u32 x0[W], x2[W], xp[W], m[W], mp[W], mm[W];
#pragma unroll
  for (int i = 0; i < W; i++) {
    x0[i] = i < 2 * h ? z0[i] : 0u;
    x2[i] = i < 2 * g ? z2[i] : 0u;
    xp[i] = i < 2 * h ? p[i] : 0u;
  }
  add_vv<W>(m, x0, x2);
  add_vv<W>(mp, m, xp);
  sub_vv<W>(mm, m, xp);
  select<W>(m, sa ^ sb, mp, mm);  // signs differ: the product of the differences is negative
  // t = z0 + z2 B^(2h) + mid B^h; the true value fits 2L limbs
  constexpr int T = 2 * L - h;
  u32 lo[T], mx[T];
#pragma unroll
  for (int i = 0; i < 2 * h; i++) t[i] = z0[i];
#pragma unroll
  for (int i = 0; i < 2 * g; i++) t[2 * h + i] = z2[i];
#pragma unroll
  for (int i = 0; i < T; i++) {
    lo[i] = t[h + i];
    mx[i] = i < W ? m[i] : 0u;
  }
  add_vv<T>(t + h, lo, mx);
}

// r = a*b mod q by Barrett reduction (Eq. (barrett), Listing 4 generalised):
//   a' = a*2^d, t = a'*b < qn^2, r1 = t >> (M-2), r2 = (r1*mu) >> (M+5),
//   t - r2*qn in [0, 2qn) (one correction), result = (that mod qn) >> d.
// The subtraction uses only the low L limbs, as in _dmulmod: the difference
// fits in L limbs.  Products: L^2 (a*b) + L^2 (r1*mu) + L(L+1)/2 (r2*qn).
// KARA: the two full products by one level of Karatsuba (kara_mul).
template <int L, bool KARA = false>
__device__ __forceinline__ void barrett_mul(u32* r, const u32* a, const u32* b, const BarrettC<L>& c) {
  // a' = a << d (a < q so a' < qn < 2^(32L-4): no overflow past L limbs)
  u32 as[L];
  if (c.d == 0) {
#pragma unroll
    for (int i = 0; i < L; i++) as[i] = a[i];
  } else {
    as[0] = a[0] << c.d;
#pragma unroll
    for (int i = 1; i < L; i++) as[i] = __builtin_amdgcn_alignbit(a[i], a[i - 1], 32 - c.d);
  }
  // t = a' * b, 2L limbs
  u32 t[2 * L];
  if constexpr (KARA) {
    kara_mul<L>(t, as, b);
  } else {
    u64 acc = 0;
    u32 hi = 0;
#pragma unroll
    for (int k = 0; k < 2 * L - 1; k++) {
#pragma unroll
      for (int i = (k < L ? 0 : k - L + 1); i <= (k < L ? k : L - 1); i++) mac_vv(acc, hi, as[i], b[k - i]);
      t[k] = (u32)acc;
      shift_col(acc, hi);
    }
    t[2 * L - 1] = (u32)acc;
  }
  // r1 = t >> (M - 2) = t >> (32(L-1) + 26): limbs L-1 .. 2L-1, bit offset 26
  u32 r1[L];
#pragma unroll
  for (int i = 0; i < L; i++) r1[i] = __builtin_amdgcn_alignbit(t[L + i], t[L - 1 + i], 26);
  // r2 = (r1 * mu) >> (M + 5) = >> (32L + 1): need product limbs L .. 2L-1 exactly
  u32 p[2 * L];
  if constexpr (KARA) {
    u32 muv[L];
    to_vgprs<L>(muv, c.mu);
    kara_mul<L>(p, r1, muv);
  } else {
    u64 acc = 0;
    u32 hi = 0;
#pragma unroll
    for (int k = 0; k < 2 * L - 1; k++) {
#pragma unroll
      for (int i = (k < L ? 0 : k - L + 1); i <= (k < L ? k : L - 1); i++) mac_vs(acc, hi, r1[i], c.mu[k - i]);
      p[k] = (u32)acc;
      shift_col(acc, hi);
    }
    p[2 * L - 1] = (u32)acc;
  }
  u32 r2[L];
#pragma unroll
  for (int i = 0; i < L - 1; i++) r2[i] = __builtin_amdgcn_alignbit(p[L + i + 1], p[L + i], 1);
  r2[L - 1] = p[2 * L - 1] >> 1;
  // low L limbs of r2 * qn
  u32 s[L];
  {
    u64 acc = 0;
    u32 hi = 0;
#pragma unroll
    for (int k = 0; k < L; k++) {
#pragma unroll
      for (int i = 0; i <= k; i++) mac_vs(acc, hi, r2[i], c.qn[k - i]);
      s[k] = (u32)acc;
      shift_col(acc, hi);
    }
  }
  u32 dlt[L], red[L];
  sub_vv<L>(dlt, t, s);               // t - r2*qn mod 2^(32L), true value in [0, 2qn)
  reduce_once<L>(red, dlt, c.qn);
  // undo the scaling: exact, the low d bits are zero
  if (c.d == 0) {
#pragma unroll
    for (int i = 0; i < L; i++) r[i] = red[i];
  } else {
#pragma unroll
    for (int i = 0; i < L - 1; i++) r[i] = __builtin_amdgcn_alignbit(red[i + 1], red[i], c.d);
    r[L - 1] = red[L - 1] >> c.d;
  }
}

}  // namespace moma
