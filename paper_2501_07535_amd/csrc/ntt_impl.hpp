// ntt_impl.hpp - number theoretic transform kernels (paper Eq. (ntt),
// Section 5.3) and their per-limb-count launchers, as templates.  ntt.hip
// dispatches on the limb count at run time; the instantiations for each limb
// count live in the ntt_inst_*.hip units, so they compile in parallel.
//
// Algorithm: radix-2 Cooley-Tukey butterflies (U + V*W, U - V*W), natural-order
// input.  Stage s (s = 0 .. log2 n - 1) has 2^s blocks; block i pairs elements
// t = n / 2^(s+1) apart and multiplies by W = w_{2m}^{rev_s(i)} with m = 2^s,
// w_{2m} = w^(n/2m).  After the last stage element p holds y[rev(p)].
//
// Data movement (MI355X-first): stages are grouped into passes of k stages that
// run in LDS, so each pass reads and writes every element once in HBM.
//   * Between passes the logical element p is stored at address rev_n(p).  The
//     first pass reads natural order and writes bit-reversed; later passes read
//     and write the same addresses (in place); after the last pass address j
//     holds y[j]: the output comes out in natural order with no extra pass.
//   * A pass over stages [K, K+k) works on groups of 2^k elements that share a
//     level-K block and an offset.  A tile is C groups whose addresses are
//     consecutive (C >= 16 words per limb plane per row), so global loads and
//     stores are coalesced in every pass.
//   * Inside a tile, each thread runs radix-2^r units in registers: 2^r
//     elements spanning r consecutive stages, so LDS is read and written, and
//     the workgroup synchronised, once per r stages instead of once per stage.
//   * Twiddle table: entry m + i' (m = 2^s) holds w_{2m}^{i'} in Montgomery form
//     for R = 2^(bD), as D b-bit digits padded to an even word count (level s
//     stores the first m powers of w_{2m}).  With that order the C
//     groups of a tile read C consecutive entries, and the first pass reads a
//     table prefix shared by every tile.
// Butterflies use lazy reduction: values stay in [0, 4q) between stages and
// between passes, and the last pass stores canonical residues in [0, q).
#pragma once
#include <string.h>

#include <atomic>

#include "common.hpp"
#include "limb.hpp"

namespace moma {

// FW: a full-width modulus (no headroom): canonical values, digits over 32L bits
template <int L, bool FW = false>
struct NttC {
  u32 q[L];
  u32 q2[L];                        // 2q (unused for a full-width modulus)
  u32 qinv;
  u32 nscaled[Digits<L, FW>::D];    // last-pass scale of the inverse, digit Montgomery form
  u32 qd[Digits<L, FW>::D];         // q in b-bit digits (twiddle multiply)
  u32 qinvd;                        // -q^-1 mod 2^b
};

__device__ __forceinline__ u32 rev_bits(u32 x, u32 b) { return b ? (__brev(x) >> (32 - b)) : 0u; }

template <int L>
__device__ __forceinline__ void load_entry(u32* r, const u32* __restrict__ p) {
  if constexpr (L % 4 == 0) {
    const uint4* v = reinterpret_cast<const uint4*>(p);
#pragma unroll
    for (int i = 0; i < L / 4; i++) {
      uint4 t = v[i];
      r[4 * i] = t.x;
      r[4 * i + 1] = t.y;
      r[4 * i + 2] = t.z;
      r[4 * i + 3] = t.w;
    }
  } else if constexpr (L % 2 == 0) {
    const uint2* v = reinterpret_cast<const uint2*>(p);
#pragma unroll
    for (int i = 0; i < L / 2; i++) {
      uint2 t = v[i];
      r[2 * i] = t.x;
      r[2 * i + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < L; i++) r[i] = p[i];
  }
}

// one twiddle entry: digit_stride(L, FW) words, 8-byte aligned
template <int L, bool FW = false>
__device__ __forceinline__ void load_digits(u32* r, const u32* __restrict__ p) {
  const uint2* v = reinterpret_cast<const uint2*>(p);
#pragma unroll
  for (int i = 0; i < digit_stride(L, FW) / 2; i++) {
    uint2 t = v[i];
    r[2 * i] = t.x;
    r[2 * i + 1] = t.y;
  }
}

// Tile geometry shared by the load, compute and store phases.
struct TileGeo {
  u32 k, logc, K, rows, C, E;
  u64 n, S, o0, ro, b0;
};

// twiddle table position for local stage sg, local block lb of group g
__device__ __forceinline__ u64 tw_pos(const TileGeo& t, u32 sg, u32 lb, u32 g) {
  return (t.K == 0) ? ((1ull << sg) + rev_bits(lb, sg))
                    : ((1ull << (t.K + sg)) + ((u64)rev_bits(lb, sg) << t.K) + t.b0 + g);
}

// One round of R stages [sg0, sg0+R) on every radix-2^R unit of the tile.
// FIRST: the transform's first round (first pass, sg0 = 0).  There every unit
// lies in block 0, so a pair whose local block index is 0 has twiddle
// w^0 = 1 (table entry 2^s) and skips the multiply: all pairs of stage 0, half
// of stage 1, a quarter of stage 2.
// STORE: the pass's last round in a later pass (K > 0) with at least 16
// columns (and at most 10 limbs): each unit writes its finished elements straight to their HBM
// addresses (the rows of one column are consecutive across lanes, so every
// store instruction covers 64-byte runs) instead of back to LDS, so the pass
// has no separate store phase and the stores drain while other units compute.
template <int L, bool FW = false>
__device__ __forceinline__ void finish_elem(u32* x, const NttPassArgs& a, const NttC<L, FW>& c) {
  if constexpr (FW) {
    // values are canonical throughout; only the inverse's scale remains
    if (a.last && a.scale) {
      u32 y[L], top;
      mont_mul_digits<L, true>(y, x, c.nscaled, c.qd, c.qinvd, &top);
      reduce_top<L>(x, y, top, c.q);
    }
    return;
  }
  if (a.last) {
    u32 y[L];
    if (a.scale) {
      mont_mul_digits<L>(y, x, c.nscaled, c.qd, c.qinvd);  // x < 4q, scale < q: y in [0, 2q)
    } else {
      reduce_once<L>(y, x, c.q2);                           // [0, 4q) -> [0, 2q)
    }
    reduce_once<L>(x, y, c.q);                              // -> [0, q)
  }
}

// LOADG: the pass's first round reads its elements straight from the input in
// HBM (the addresses the load phase would have filled the LDS rows from)
// instead of from LDS, so the pass has no separate load phase.
// Wide limbs, radix-2 units: registers, not instructions, bound these kernels
// (one or two waves per SIMD), so a unit reads the bottom element, forms the
// product w*y, and only then reads the top element and copies 2q (or q) into
// VGPRs for the additions; neither is live across the multiply.
constexpr int kLateLoadLimbs = 11;

template <int L, bool FIRST, bool STORE, int AR>
__device__ __forceinline__ void round_late(u32* lds, const TileGeo& t, u32 sg0, const NttPassArgs& a,
                                           const NttC<L, AR == kArithFull>& c) {
  constexpr bool FW = AR == kArithFull;
  const u32* __restrict__ tw = a.tw;
  const u32 k = t.k;
  const u32 B = 1u << (k - sg0);  // block size (rows) at stage sg0; the pair is B/2 rows apart
  const u32 units = t.E >> 1;
  for (u32 b = threadIdx.x; b < units; b += blockDim.x) {
    u32 g = b & (t.C - 1), v = b >> t.logc;
    u32 lb = v >> (k - sg0 - 1);
    u32 p0 = lb * B + (v & ((B >> 1) - 1));
    const u32 r0 = p0, r1 = p0 + (B >> 1);
    u32 x[L], y[L];
    if (FIRST && lb == 0) {
      // twiddle 1: no multiply
#pragma unroll
      for (int j = 0; j < L; j++) {
        x[j] = lds[(j * t.rows + r0) * t.C + g];
        y[j] = lds[(j * t.rows + r1) * t.C + g];
      }
      u32 qv[L];
      to_vgprs<L>(qv, FW ? c.q : c.q2);
      if constexpr (FW)
        ct_butterfly_one_fw<L>(x, y, qv);
      else
        ct_butterfly_one<L>(x, y, qv);
    } else {
      u32 w[digit_stride(L, FW)], p[L], top = 0;
      load_digits<L, FW>(w, tw + tw_pos(t, sg0, lb, g) * digit_stride(L, FW));
#pragma unroll
      for (int j = 0; j < L; j++) y[j] = lds[(j * t.rows + r1) * t.C + g];
      if constexpr (FW)
        mont_mul_digits<L, true>(p, y, w, c.qd, c.qinvd, &top);
      else if constexpr (AR == kArithKara)
        mont_mul_digits_kara<L>(p, y, w, c.qd, c.qinvd);
      else
        mont_mul_digits<L>(p, y, w, c.qd, c.qinvd);
#pragma unroll
      for (int j = 0; j < L; j++) x[j] = lds[(j * t.rows + r0) * t.C + g];
      u32 qv[L];
      to_vgprs<L>(qv, FW ? c.q : c.q2);
      if constexpr (FW)
        ct_fw_tail<L>(x, y, p, top, qv);
      else
        ct_lazy_tail<L>(x, y, p, qv);
    }
    if constexpr (STORE) {
      const u64 base = (t.ro << (t.K + k)) + t.b0 + g;
      finish_elem<L, FW>(x, a, c);
      finish_elem<L, FW>(y, a, c);
      const u64 d0 = base + ((u64)rev_bits(r0, k) << t.K), d1 = base + ((u64)rev_bits(r1, k) << t.K);
#pragma unroll
      for (int j = 0; j < L; j++) {
        a.out[(u64)j * t.n + d0] = x[j];
        a.out[(u64)j * t.n + d1] = y[j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < L; j++) {
        lds[(j * t.rows + r0) * t.C + g] = x[j];
        lds[(j * t.rows + r1) * t.C + g] = y[j];
      }
    }
  }
}

// AR: the kernel's arithmetic (NttArith)
template <int L, int R, bool FIRST, bool STORE, bool LOADG = false, int AR = kArithLazy>
__device__ __forceinline__ void ntt_round(u32* lds, const TileGeo& t, u32 sg0, const NttPassArgs& a,
                                          const NttC<L, AR == kArithFull>& c) {
  constexpr bool FW = AR == kArithFull;
  const u32* __restrict__ tw = a.tw;
  const u32 k = t.k;
  const u32 B = 1u << (k - sg0);        // block size (rows) at stage sg0
  const u32 sub = B >> R;                // row spacing of a unit's elements
  const u32 units = (t.E >> R);
  if constexpr (R == 1 && !LOADG && L >= kLateLoadLimbs) {
    round_late<L, FIRST, STORE, AR>(lds, t, sg0, a, c);
    return;
  }
  u32 q2v[L];  // 2q (lazy butterflies), or q (full width)
  to_vgprs<L>(q2v, FW ? c.q : c.q2);
  for (u32 b = threadIdx.x; b < units; b += blockDim.x) {
    u32 g = b & (t.C - 1), v = b >> t.logc;
    u32 lb = v >> (k - sg0 - R);
    u32 p0 = lb * B + (v & (sub - 1));
    u32 x[1 << R][L];
    // LOADG: the first stage's twiddle (one per unit) is loaded before the
    // elements, and the elements pair by pair of the first stage, (e, e +
    // 2^(R-1)): a wave's loads complete in issue order, so the first pair's
    // butterfly can start while the later pairs are still in flight
    u32 w0[LOADG ? digit_stride(L, FW) : 1];
    if constexpr (LOADG) {
      if constexpr (!FIRST) load_digits<L, FW>(w0, tw + tw_pos(t, sg0, lb, g) * digit_stride(L, FW));
#pragma unroll
      for (int pp = 0; pp < (1 << R); pp++) {
        const int e = (pp >> 1) + (pp & 1) * (1 << (R - 1));
        const u32 u = p0 + e * sub;  // LDS row; global row u (first pass) or rev(u) (later passes)
        const u64 src = (t.K == 0) ? (u64)u * t.S + t.o0 + g
                                   : (t.ro << (t.K + k)) + ((u64)rev_bits(u, k) << t.K) + t.b0 + g;
#pragma unroll
        for (int j = 0; j < L; j++) x[e][j] = a.in[(u64)j * t.n + src];
      }
    } else {
#pragma unroll
      for (int e = 0; e < (1 << R); e++)
#pragma unroll
        for (int j = 0; j < L; j++) x[e][j] = lds[(j * t.rows + p0 + e * sub) * t.C + g];
    }
#pragma unroll
    for (int s = 0; s < R; s++) {
      const int kb = R - 1 - s, half = 1 << kb;
#pragma unroll
      for (int p = 0; p < (1 << (R - 1)); p++) {
        // p with a zero bit inserted at position kb: the pair (e, e + half) of this stage
        const int e = ((p >> kb) << (kb + 1)) | (p & (half - 1));
        auto bfly = [&](const u32* w) {
          if constexpr (FW)
            ct_butterfly_fw<L>(x[e], x[e + half], w, c.qd, c.qinvd, q2v);
          else if constexpr (AR == kArithKara)
            ct_butterfly_kara<L>(x[e], x[e + half], w, c.qd, c.qinvd, q2v);
          else
            ct_butterfly_digits<L>(x[e], x[e + half], w, c.qd, c.qinvd, q2v);
        };
        if (FIRST && (e >> (R - s)) == 0) {
          if constexpr (FW)
            ct_butterfly_one_fw<L>(x[e], x[e + half], q2v);
          else
            ct_butterfly_one<L>(x[e], x[e + half], q2v);
        } else if (LOADG && s == 0) {
          bfly(w0);  // stage 0: every pair of the unit has block lb
        } else {
          u32 lbk = (lb << s) + (u32)(e >> (R - s));
          u32 w[digit_stride(L, FW)];
          load_digits<L, FW>(w, tw + tw_pos(t, sg0 + s, lbk, g) * digit_stride(L, FW));
          bfly(w);
        }
      }
    }
    if constexpr (STORE) {
      const u64 base = (t.ro << (t.K + k)) + t.b0 + g;
#pragma unroll
      for (int e = 0; e < (1 << R); e++) {
        const u64 dst = base + ((u64)rev_bits(p0 + e * sub, k) << t.K);
        finish_elem<L, FW>(x[e], a, c);
#pragma unroll
        for (int j = 0; j < L; j++) a.out[(u64)j * t.n + dst] = x[e][j];
      }
    } else {
#pragma unroll
      for (int e = 0; e < (1 << R); e++)
#pragma unroll
        for (int j = 0; j < L; j++) lds[(j * t.rows + p0 + e * sub) * t.C + g] = x[e][j];
    }
  }
}

// Exchange of a final-stage round: a <-> the partner lane's b, where the
// partner of lane l is l ^ 32 (C = 32 groups per tile) or l ^ 16 (C = 16).
// v_permlane32_swap / v_permlane16_swap swap the upper (odd) 32- (16-) lane
// rows of the first operand with the lower (even) rows of the second.
__device__ __forceinline__ void swap_with_partner(u32& a, u32& b, bool c32) {
  if (c32) {
    auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  } else {
    auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  }
}

// The pass's last R + 1 stages [sg0, k) without an LDS round trip before the
// last one.  A radix-2^R round on stages sg0 .. k - 2 leaves element e of unit
// v at row p0 + 2e of its block (p0 = block start + (v & 1)), so the partners
// of the last stage, rows 2m and 2m + 1, sit in units v and v ^ 1: the same
// group g, in lanes C apart of one wavefront (the units of a round are laid
// out g-fastest).  Swapping the upper half of one unit's elements with the
// lower half of its partner's puts both rows of a pair in one lane: lane half
// h = v & 1 then holds pair j (elements j and j + 2^(R-1)) = rows
// 2j + 2^R h and 2j + 2^R h + 1 of the block, whose last-stage block index is
// 2^R lb + 2^(R-1) h + j.  Requires C in {16, 32}, whole wavefronts of units,
// and a round that is not the transform's first.
template <int L, int R, bool STORE>
__device__ __forceinline__ void ntt_round_last(u32* lds, const TileGeo& t, u32 sg0, const NttPassArgs& a,
                                               const NttC<L>& c) {
  const u32* __restrict__ tw = a.tw;
  const u32 k = t.k;
  const u32 B = 1u << (k - sg0);        // block size (rows) at stage sg0: 2^(R+1)
  const u32 units = (t.E >> R);
  const bool c32 = t.logc == 5;
  constexpr int H = 1 << (R - 1);
  u32 q2v[L];
  to_vgprs<L>(q2v, c.q2);
  for (u32 b = threadIdx.x; b < units; b += blockDim.x) {
    u32 g = b & (t.C - 1), v = b >> t.logc;
    u32 lb = v >> 1;
    u32 p0 = lb * B + (v & 1u);
    u32 x[1 << R][L];
#pragma unroll
    for (int e = 0; e < (1 << R); e++)
#pragma unroll
      for (int j = 0; j < L; j++) x[e][j] = lds[(j * t.rows + p0 + 2 * e) * t.C + g];
#pragma unroll
    for (int s = 0; s < R; s++) {
      const int kb = R - 1 - s, half = 1 << kb;
#pragma unroll
      for (int p = 0; p < (1 << (R - 1)); p++) {
        const int e = ((p >> kb) << (kb + 1)) | (p & (half - 1));
        u32 lbk = (lb << s) + (u32)(e >> (R - s));
        u32 w[digit_stride(L)];
        load_digits<L>(w, tw + tw_pos(t, sg0 + s, lbk, g) * digit_stride(L));
        ct_butterfly_digits<L>(x[e], x[e + half], w, c.qd, c.qinvd, q2v);
      }
    }
#pragma unroll
    for (int e = 0; e < H; e++)
#pragma unroll
      for (int j = 0; j < L; j++) swap_with_partner(x[e][j], x[e + H][j], c32);
    const u32 h = v & 1u;
#pragma unroll
    for (int jp = 0; jp < H; jp++) {
      u32 lbk = (lb << R) + (h << (R - 1)) + (u32)jp;
      u32 w[digit_stride(L)];
      load_digits<L>(w, tw + tw_pos(t, k - 1, lbk, g) * digit_stride(L));
      ct_butterfly_digits<L>(x[jp], x[jp + H], w, c.qd, c.qinvd, q2v);
    }
    const u32 r0 = lb * B + (h << R);
    if constexpr (STORE) {
      const u64 base = (t.ro << (t.K + k)) + t.b0 + g;
#pragma unroll
      for (int jp = 0; jp < H; jp++)
#pragma unroll
        for (int o = 0; o < 2; o++) {
          u32* y = x[jp + o * H];
          const u64 dst = base + ((u64)rev_bits(r0 + 2 * jp + o, k) << t.K);
          finish_elem<L>(y, a, c);
#pragma unroll
          for (int j = 0; j < L; j++) a.out[(u64)j * t.n + dst] = y[j];
        }
    } else {
#pragma unroll
      for (int jp = 0; jp < H; jp++)
#pragma unroll
        for (int o = 0; o < 2; o++)
#pragma unroll
          for (int j = 0; j < L; j++) lds[(j * t.rows + r0 + 2 * jp + o) * t.C + g] = x[jp + o * H][j];
    }
  }
}

// One tile of one pass: stages [K, K+k) on C = 2^logc groups of 2^k elements.
// LDS holds the tile limb-planar: word (j * 2^k + u) * C + g is limb j of row u
// of group g, so lanes with consecutive g touch consecutive banks.
// the fused store keeps a unit's finished elements live while it stores them
// (up to 10 limbs, 9 for a full-width modulus: at 11 to 16 limbs it measured
// no faster than the store from LDS)
template <int L, bool FW = false>
constexpr bool kFuseStore = L <= (FW ? 9 : 10);

template <int L, int R, int AR = kArithLazy>
__device__ __forceinline__ void round_at(u32* lds, const TileGeo& t, u32 sg0, const NttPassArgs& a,
                                         const NttC<L, AR == kArithFull>& c, bool store) {
  if constexpr (kFuseStore<L, AR == kArithFull>) {
    if (store) {
      ntt_round<L, R, false, true, false, AR>(lds, t, sg0, a, c);
      return;
    }
  }
  if (t.K == 0 && sg0 == 0)
    ntt_round<L, R, true, false, false, AR>(lds, t, sg0, a, c);
  else
    ntt_round<L, R, false, false, false, AR>(lds, t, sg0, a, c);
}

// Fused pointwise product of a cyclic product's first inverse pass:
// r = x * y * 2^(-bD) mod q in [0, 2q) for x, y < q (the digit-form multiply
// with y converted to digits; the last pass's scale constant carries 2^(bD)).
template <int L, bool FW = false>
__device__ __forceinline__ void pointwise_digits(u32* r, const u32* x, const u32* y, const NttC<L, FW>& c) {
  u32 yd[Digits<L, FW>::D];
  to_digits<L, FW>(yd, y);
  if constexpr (FW) {
    // canonical result for a full-width modulus
    u32 t[L], top;
    mont_mul_digits<L, true>(t, x, yd, c.qd, c.qinvd, &top);
    reduce_top<L>(r, t, top, c.q);
  } else {
    mont_mul_digits<L>(r, x, yd, c.qd, c.qinvd);
  }
}

// MUL: the pass also multiplies its input by a.in2 element by element as it
// loads (first pass of the inverse transform inside a cyclic product).
// LASTX: the pass ends with ntt_round_last (radix-4 units only; the launcher
// sets it when fused_last_applies holds, so other launches run unchanged code).
template <int L, int R, bool MUL, bool LASTX = false, int AR = kArithLazy>
__device__ __forceinline__ void pass_tile(u32* lds, const NttPassArgs& a, const NttC<L, AR == kArithFull>& c,
                                          u64 tile) {
  constexpr bool FW = AR == kArithFull;
  static_assert(AR == kArithLazy || !LASTX, "only the lazy schoolbook kernels have the cross-lane variant");
  TileGeo t;
  t.k = a.k;
  t.logc = a.logc;
  t.K = a.K;
  t.C = 1u << t.logc;
  t.rows = 1u << t.k;
  t.E = t.rows << t.logc;
  t.n = a.n;
  t.S = t.n >> (t.K + t.k);
  t.o0 = t.ro = t.b0 = 0;
  if (t.K == 0) {
    t.o0 = tile << t.logc;
  } else {
    u64 per = (1ull << t.K) >> t.logc;
    t.ro = tile / per;
    t.b0 = (tile % per) << t.logc;
  }
  const u32 tid = threadIdx.x, T = blockDim.x;
  const u64 n = t.n;
  // LASTX passes without a fused product read their first round straight from HBM
  const bool direct = LASTX && !MUL && a.direct != 0;

  // ---- load (natural order in the first pass, bit-reversed storage after).
  // Each lane moves 4 consecutive words per limb: 4 groups of one row when the
  // tile has C >= 4 groups, else 4 consecutive rows of a one-pass transform.
  const bool vec_g = t.C >= 4, vec_u = (t.C == 1 && t.S == 1 && t.rows >= 4);
  if (direct) {
    // the first round loads its own elements
  } else if (vec_g || vec_u) {
    for (u32 e4 = tid; e4 < (t.E >> 2); e4 += T) {
      u32 e = e4 << 2;
      u32 g = e & (t.C - 1), v = e >> t.logc;
      u64 src;
      u32 u;
      if (t.K == 0) {
        u = v;
        src = (u64)u * t.S + t.o0 + g;
      } else {
        u = rev_bits(v, t.k);
        src = (t.ro << (t.K + t.k)) + ((u64)v << t.K) + t.b0 + g;
      }
      if constexpr (MUL && L <= 8) {
        // 4 elements of each input in registers, multiplied pointwise
        u32 x[4][L], y[4][L];
#pragma unroll
        for (int j = 0; j < L; j++) {
          uint4 w = *reinterpret_cast<const uint4*>(a.in + (u64)j * n + src);
          uint4 z = *reinterpret_cast<const uint4*>(a.in2 + (u64)j * n + src);
          x[0][j] = w.x; x[1][j] = w.y; x[2][j] = w.z; x[3][j] = w.w;
          y[0][j] = z.x; y[1][j] = z.y; y[2][j] = z.z; y[3][j] = z.w;
        }
        u32 r[4][L];
#pragma unroll
        for (int q4 = 0; q4 < 4; q4++) pointwise_digits<L, FW>(r[q4], x[q4], y[q4], c);
#pragma unroll
        for (int j = 0; j < L; j++)
          *reinterpret_cast<uint4*>(lds + (j * t.rows + u) * t.C + g) = make_uint4(r[0][j], r[1][j], r[2][j], r[3][j]);
      } else if constexpr (MUL) {
        // wider limbs, fewer live registers: stage the first input in LDS as
        // the plain load does, then multiply one element at a time; each lane
        // rereads only the 4 consecutive LDS words (4 groups of one row, or 4
        // rows when C == 1) that it wrote itself
#pragma unroll
        for (int j = 0; j < L; j++) {
          uint4 w = *reinterpret_cast<const uint4*>(a.in + (u64)j * n + src);
          *reinterpret_cast<uint4*>(lds + (j * t.rows + u) * t.C + g) = w;
        }
#pragma unroll 1
        for (u32 q4 = 0; q4 < 4; q4++) {
          u32 x[L], y[L], r[L];
#pragma unroll
          for (int j = 0; j < L; j++) {
            x[j] = lds[(j * t.rows + u) * t.C + g + q4];
            y[j] = a.in2[(u64)j * n + src + q4];
          }
          pointwise_digits<L, FW>(r, x, y, c);
#pragma unroll
          for (int j = 0; j < L; j++) lds[(j * t.rows + u) * t.C + g + q4] = r[j];
        }
      } else {
#pragma unroll
        for (int j = 0; j < L; j++) {
          uint4 w = *reinterpret_cast<const uint4*>(a.in + (u64)j * n + src);
          *reinterpret_cast<uint4*>(lds + (j * t.rows + u) * t.C + g) = w;
        }
      }
    }
  } else {
    for (u32 e = tid; e < t.E; e += T) {
      u32 g = e & (t.C - 1), v = e >> t.logc;
      u64 src;
      u32 u;
      if (t.K == 0) {
        u = v;
        src = (u64)u * t.S + t.o0 + g;
      } else {
        u = rev_bits(v, t.k);
        src = (t.ro << (t.K + t.k)) + ((u64)v << t.K) + t.b0 + g;
      }
      if constexpr (MUL) {
        u32 x[L], y[L], r[L];
#pragma unroll
        for (int j = 0; j < L; j++) {
          x[j] = a.in[(u64)j * n + src];
          y[j] = a.in2[(u64)j * n + src];
        }
        pointwise_digits<L, FW>(r, x, y, c);
#pragma unroll
        for (int j = 0; j < L; j++) lds[(j * t.rows + u) * t.C + g] = r[j];
      } else {
#pragma unroll
        for (int j = 0; j < L; j++) lds[(j * t.rows + u) * t.C + g] = a.in[(u64)j * n + src];
      }
    }
  }
  if (!direct) __syncthreads();

  // ---- stages, R at a time in registers
  // later passes with 16+ columns store from the last round's registers
  const bool fuse = kFuseStore<L, FW> && t.K > 0 && t.C >= 16;
  u32 sg = 0;
  while (sg < t.k) {
    u32 rem = t.k - sg;
    if constexpr (LASTX && !MUL) {
      if (direct && sg == 0) {
        if (t.K == 0)
          ntt_round<L, R, true, false, true>(lds, t, 0, a, c);
        else
          ntt_round<L, R, false, false, true>(lds, t, 0, a, c);
        sg = R;
        __syncthreads();
        continue;
      }
    }
    if constexpr ((R == 2 || R == 3) && LASTX) {
      // the last R + 1 stages with a cross-lane exchange before the last one
      if (rem == (u32)R + 1 && (t.logc == 4 || t.logc == 5) && ((t.E >> R) & 63u) == 0 &&
          (t.E >> R) >= blockDim.x && !(t.K == 0 && sg == 0)) {
        if constexpr (kFuseStore<L>) {
          if (fuse) {
            ntt_round_last<L, R, true>(lds, t, sg, a, c);
            return;
          }
        }
        ntt_round_last<L, R, false>(lds, t, sg, a, c);
        __syncthreads();
        break;
      }
    }
    const u32 rr = rem < (u32)R ? rem : (u32)R;
    const bool store = fuse && sg + rr == t.k;
    if (rr == 4) {
      round_at<L, (R >= 4 ? 4 : 1), AR>(lds, t, sg, a, c, store);
    } else if (rr == 3) {
      round_at<L, (R >= 3 ? 3 : 1), AR>(lds, t, sg, a, c, store);
    } else if (rr == 2) {
      round_at<L, (R >= 2 ? 2 : 1), AR>(lds, t, sg, a, c, store);
    } else {
      round_at<L, 1, AR>(lds, t, sg, a, c, store);
    }
    sg += rr;
    if (!store) __syncthreads();
  }
  if (fuse) return;

  // ---- store (canonical residues on the last pass), 4 words per lane per limb
  const u32 logn = a.logn;
  auto finish = [&](u32* x) { finish_elem<L, FW>(x, a, c); };
  // 4 elements of L limbs (and the scale multiply) stay in registers
  // (up to 10 limbs: at 11 to 16 limbs the 4L live words cost occupancy, and
  // 2^16-point transforms measured 3 to 10% slower)
  constexpr bool kVecStore = L <= (FW ? 9 : 10);
  if (kVecStore && t.K > 0 && vec_g) {
    // same addresses as the load: 4 consecutive groups of one row
    for (u32 e4 = tid; e4 < (t.E >> 2); e4 += T) {
      u32 e = e4 << 2;
      u32 g = e & (t.C - 1), v = e >> t.logc;
      u32 u = rev_bits(v, t.k);
      u64 dst = (t.ro << (t.K + t.k)) + ((u64)v << t.K) + t.b0 + g;
      u32 x[4][L];
#pragma unroll
      for (int j = 0; j < L; j++) {
        uint4 w = *reinterpret_cast<const uint4*>(lds + (j * t.rows + u) * t.C + g);
        x[0][j] = w.x;
        x[1][j] = w.y;
        x[2][j] = w.z;
        x[3][j] = w.w;
      }
#pragma unroll
      for (int q4 = 0; q4 < 4; q4++) finish(x[q4]);
#pragma unroll
      for (int j = 0; j < L; j++)
        *reinterpret_cast<uint4*>(a.out + (u64)j * n + dst) = make_uint4(x[0][j], x[1][j], x[2][j], x[3][j]);
    }
  } else if (kVecStore && t.K == 0 && t.rows >= 4) {
    // 4 consecutive output addresses inside one group's run of 2^k
    for (u32 e4 = tid; e4 < (t.E >> 2); e4 += T) {
      u32 e = e4 << 2;
      u32 g = e >> t.k, v = e & (t.rows - 1);
      u64 dst = ((u64)rev_bits((u32)(t.o0 + g), logn - t.k) << t.k) + v;
      u32 x[4][L];
#pragma unroll
      for (int q4 = 0; q4 < 4; q4++) {
        u32 u = rev_bits(v + q4, t.k);
#pragma unroll
        for (int j = 0; j < L; j++) x[q4][j] = lds[(j * t.rows + u) * t.C + g];
        finish(x[q4]);
      }
#pragma unroll
      for (int j = 0; j < L; j++)
        *reinterpret_cast<uint4*>(a.out + (u64)j * n + dst) = make_uint4(x[0][j], x[1][j], x[2][j], x[3][j]);
    }
  } else {
    for (u32 e = tid; e < t.E; e += T) {
      u32 g, v, u;
      u64 dst;
      if (t.K == 0) {
        g = e >> t.k;
        v = e & (t.rows - 1);
        u = rev_bits(v, t.k);
        dst = ((u64)rev_bits((u32)(t.o0 + g), logn - t.k) << t.k) + v;
      } else {
        g = e & (t.C - 1);
        v = e >> t.logc;
        u = rev_bits(v, t.k);
        dst = (t.ro << (t.K + t.k)) + ((u64)v << t.K) + t.b0 + g;
      }
      u32 x[L];
#pragma unroll
      for (int j = 0; j < L; j++) x[j] = lds[(j * t.rows + u) * t.C + g];
      finish(x);
#pragma unroll
      for (int j = 0; j < L; j++) a.out[(u64)j * n + dst] = x[j];
    }
  }
}

// Workgroup size cap per instantiation: a radix-2^R unit keeps 2^R elements of
// L limbs live, so wider units get fewer threads and more VGPRs per lane.
template <int L, int R>
struct PassTraits {
  static constexpr int live = L << R;
  static constexpr int max_threads = live <= 16 ? 1024 : (live <= 32 ? 512 : 256);
};

// One pass of one transform: workgroup b runs tile b.
template <int L, int R, bool MUL, bool LASTX, int AR = kArithLazy>
__global__ __launch_bounds__((PassTraits<L, R>::max_threads)) void ntt_pass_kernel(NttPassArgs a,
                                                                                 NttC<L, AR == kArithFull> c) {
  extern __shared__ u32 lds[];
  pass_tile<L, R, MUL, LASTX, AR>(lds, a, c, blockIdx.x);
}

// Whether a pass with radix-4 units ends with ntt_round_last: its stage count
// is odd (rounds 2, 2, ..., then 3), the tile has 16 or 32 groups, the units
// fill whole wavefronts and every thread has one, and the fused round is not
// the transform's first round.  Measured against the separate radix-2 round:
// transforms 1 to 4% faster at 2^20 and 2^21 points from 64 to 256 bits; where
// a thread would have no radix-4 unit the separate round, which keeps twice as
// many threads busy, is faster.
inline bool fused_last_applies(const NttPassArgs& a, uint32_t threads, uint32_t radix_log) {
  const uint32_t r = radix_log;
  if (a.k < r + 1 || (a.k - r - 1) % r != 0 || (a.logc != 4 && a.logc != 5)) return false;
  const uint64_t units = (1ull << (a.k + a.logc)) >> r;
  return units % 64 == 0 && units >= threads && !(a.K == 0 && a.k == r + 1);
}

// One phase of a batch: items[i] = (pass record, tile); every pass record names
// its own transform (buffers, size, stages, twiddles) and its modulus constants.
// Workgroup i runs item i; items are sorted by decreasing cost, so the
// dispatcher hands out the largest tiles first.
template <int L, int R, bool MUL, bool LASTX, bool FW = false>
__global__ __launch_bounds__((PassTraits<L, R>::max_threads)) void ntt_batch_kernel(
    const NttPassArgs* __restrict__ passes, const NttC<L, FW>* __restrict__ consts, const uint2* __restrict__ items,
    u32 nitems) {
  extern __shared__ u32 lds[];
  const u32 i = blockIdx.x;
  if (i >= nitems) return;
  const uint2 it = items[i];
  const NttPassArgs* rec = passes + it.x;
  NttPassArgs a = *rec;
  a.in = load_global_ptr(&rec->in);
  a.in2 = load_global_ptr(&rec->in2);
  a.out = load_global_ptr(&rec->out);
  a.tw = load_global_ptr(&rec->tw);
  const NttC<L, FW> c = consts[it.x];
  pass_tile<L, R, MUL, LASTX, FW ? kArithFull : kArithLazy>(lds, a, c, it.y);
}

// Twiddle table: entry e = 2^s + i' holds w^(i' * 2^(logn-s-1)) * 2^(32L) mod q.
// ladder[b] = w^(2^b) * 2^(32L) mod q; the product of the ladder entries for the
// set bits of the exponent stays in Montgomery form.
// FW (full-width modulus): the products keep the carry out of the top limb.
template <int L, bool FW = false>
__global__ __launch_bounds__(256) void twiddle_kernel(u32* __restrict__ tw, u64 n, u32 logn,
                                                      const u32* __restrict__ ladder, NttC<L, FW> c,
                                                      const u32* __restrict__ one_m, const u32* __restrict__ adj) {
  u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  u32 acc[L];
#pragma unroll
  for (int j = 0; j < L; j++) acc[j] = one_m[j];
  if (e > 0) {
    u32 s = 63 - __builtin_clzll(e);
    u64 ip = e - (1ull << s);
    u64 x = ip << (logn - s - 1);
    for (u32 bit = 0; bit < logn; bit++) {
      if ((x >> bit) & 1) {
        u32 w[L], t[L];
#pragma unroll
        for (int j = 0; j < L; j++) w[j] = ladder[bit * L + j];
        if constexpr (FW)
          mont_mul_fw<L>(t, acc, w, c.q, c.qinv, c.q);
        else
          mont_mul<L>(t, acc, w, c.q, c.qinv);
#pragma unroll
        for (int j = 0; j < L; j++) acc[j] = t[j];
      }
    }
  }
  // acc = w^x * 2^(32L); times 2^(bD) * 2^(-32L) gives the digit-form Montgomery value
  constexpr int S = digit_stride(L, FW);
  u32 ad[L], wm[L], d[S];
#pragma unroll
  for (int j = 0; j < L; j++) ad[j] = adj[j];
  if constexpr (FW)
    mont_mul_fw<L>(wm, acc, ad, c.q, c.qinv, c.q);
  else
    mont_mul<L>(wm, acc, ad, c.q, c.qinv);
  to_digits<L, FW>(d, wm);
  if (S > Digits<L, FW>::D) d[S - 1] = 0;
#pragma unroll
  for (int j = 0; j < S; j++) tw[e * S + j] = d[j];
}

template <int L, bool FW = false>
inline NttC<L, FW> make_consts(const FieldRaw& f, const DigitConsts& dc, const NttConsts* nc) {
  NttC<L, FW> c;
  for (int j = 0; j < Digits<L, FW>::D; j++) c.qd[j] = dc.qd[j];
  c.qinvd = dc.qinvd;
  u64 carry = 0;
  for (int j = 0; j < L; j++) {
    c.q[j] = f.q[j];
    u64 d = ((u64)f.q[j] << 1) + carry;  // 2q limb by limb (wraps for a full-width q, where it is unused)
    c.q2[j] = (u32)d;
    carry = d >> 32;
  }
  for (int j = 0; j < Digits<L, FW>::D; j++) c.nscaled[j] = nc ? nc->nscale_d[j] : 0;
  c.qinv = f.qinv;
  return c;
}

template <int L, int R, bool MUL, bool LASTX, int AR = kArithLazy>
int launch_pass_LRM(const NttC<L, AR == kArithFull>& c, const NttPassArgs& a, uint32_t threads, uint64_t tiles,
                    hipStream_t s) {
  size_t lds = (size_t)L * ((size_t)1 << (a.k + a.logc)) * sizeof(u32);
  static std::atomic<bool> attr_set{false};  // several host threads may launch at once
  if (lds > 65536 && !attr_set.load(std::memory_order_acquire)) {
    (void)hipFuncSetAttribute((const void*)ntt_pass_kernel<L, R, MUL, LASTX, AR>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set.store(true, std::memory_order_release);
  }
  hipLaunchKernelGGL((ntt_pass_kernel<L, R, MUL, LASTX, AR>), dim3((unsigned)tiles), dim3(threads), lds, s, a, c);
  return (int)hipGetLastError();
}

// (up to 8 limbs: at 10 limbs the fused round measured level at 2^20 points
// and 3% slower at 2^18)
template <int L>
constexpr bool kFusedLast = L <= 8;

// Whether a pass's first round reads its elements straight from HBM (the
// LASTX variant does when it has no fused product): 16 or 32 groups per tile
// (each load instruction then covers 64- or 128-byte runs, as the load phase's
// do), more than one round, and at least two tiles per compute unit.  Measured:
// 1 to 7% faster transforms from 64 to 256 bits at 2^19 to 2^25 points; with
// one tile per compute unit (2^18 points, 256 bits) the load phase's wider
// loads were 4% faster.
uint32_t device_cu_count();
inline bool direct_load_applies(const NttPassArgs& a, uint32_t radix_log, uint64_t tiles) {
  return !a.in2 && (a.logc == 4 || a.logc == 5) && a.k > radix_log && tiles >= 2ull * device_cu_count();
}

// The batch executor's choice for one pass record: the variant kernel when the
// pass would take the cross-lane last stage or the direct first round (a batch
// launch holds many tiles, so the tile-count rule of a lone call is not applied).
inline bool batch_variant(int L, uint32_t radix_log, uint32_t threads, NttPassArgs* a) {
  if ((radix_log != 2 && radix_log != 3) || L > 8) return false;
  const bool direct = !a->in2 && (a->logc == 4 || a->logc == 5) && a->k > radix_log;
  a->direct = direct ? 1u : 0u;
  return direct || fused_last_applies(*a, threads, radix_log);
}

template <int L, int R, bool MUL>
int launch_pass_LRX(const NttC<L>& c, const NttPassArgs& a, uint32_t threads, uint64_t tiles, hipStream_t s) {
  if constexpr ((R == 2 || R == 3) && kFusedLast<L>) {
    const bool direct = direct_load_applies(a, R, tiles);
    if (direct || fused_last_applies(a, threads, R)) {
      NttPassArgs b = a;
      b.direct = direct ? 1u : 0u;
      return launch_pass_LRM<L, R, MUL, true>(c, b, threads, tiles, s);
    }
  }
  return launch_pass_LRM<L, R, MUL, false>(c, a, threads, tiles, s);
}

template <int L, int R>
int launch_pass_LR(const NttC<L>& c, const NttPassArgs& a, uint32_t threads, uint64_t tiles, hipStream_t s) {
  return a.in2 ? launch_pass_LRX<L, R, true>(c, a, threads, tiles, s)
               : launch_pass_LRX<L, R, false>(c, a, threads, tiles, s);
}

// full-width modulus: radix-2 and radix-4 units, no cross-lane variant
template <int L>
int launch_pass_fw(const FieldRaw& f, const DigitConsts& dc, const NttPassArgs& a, const NttConsts& nc,
                   uint32_t threads, uint64_t tiles, uint32_t radix_log, hipStream_t s) {
  NttC<L, true> c = make_consts<L, true>(f, dc, &nc);
  if (radix_log == 1)
    return a.in2 ? launch_pass_LRM<L, 1, true, false, kArithFull>(c, a, threads, tiles, s)
                 : launch_pass_LRM<L, 1, false, false, kArithFull>(c, a, threads, tiles, s);
  if constexpr (L <= kMaxLimbsRadix4Fw) {
    if (radix_log == 2)
      return a.in2 ? launch_pass_LRM<L, 2, true, false, kArithFull>(c, a, threads, tiles, s)
                   : launch_pass_LRM<L, 2, false, false, kArithFull>(c, a, threads, tiles, s);
  }
  return (int)hipErrorInvalidValue;
}

template <int L>
int launch_pass_L(const FieldRaw& f, const DigitConsts& dc, const NttPassArgs& a, const NttConsts& nc,
                  uint32_t threads, uint64_t tiles, uint32_t radix_log, uint32_t kara, hipStream_t s) {
  if (f.fw)
    return kara ? (int)hipErrorInvalidValue : launch_pass_fw<L>(f, dc, a, nc, threads, tiles, radix_log, s);
  NttC<L> c = make_consts<L>(f, dc, &nc);
  if (kara) {
    // the Karatsuba butterfly: radix-2 units, 2 to 24 limbs, no cross-lane variant
    if constexpr (L >= 2 && L <= kMaxLimbsKara) {
      if (radix_log == 1)
        return a.in2 ? launch_pass_LRM<L, 1, true, false, kArithKara>(c, a, threads, tiles, s)
                     : launch_pass_LRM<L, 1, false, false, kArithKara>(c, a, threads, tiles, s);
    }
    return (int)hipErrorInvalidValue;
  }
  // register blocking is limited by the VGPR budget: 2^r elements of L limbs
  if (radix_log == 1) return launch_pass_LR<L, 1>(c, a, threads, tiles, s);
  if constexpr (L <= kMaxLimbsRadix4) {
    if (radix_log == 2) return launch_pass_LR<L, 2>(c, a, threads, tiles, s);
  }
  if constexpr (L <= kMaxLimbsRadix8) {
    if (radix_log == 3) return launch_pass_LR<L, 3>(c, a, threads, tiles, s);
  }
  if constexpr (L <= kMaxLimbsRadix16) {
    if (radix_log == 4) return launch_pass_LR<L, 4>(c, a, threads, tiles, s);
  }
  return (int)hipErrorInvalidValue;
}

template <int L, int R, bool LASTX, bool FW = false>
int launch_batch_LRX(bool mul, uint32_t threads, size_t lds, uint32_t grid, const NttPassArgs* d_passes,
                     const void* d_consts, const uint2* d_items, uint32_t nitems, hipStream_t s) {
  if (mul)
    hipLaunchKernelGGL((ntt_batch_kernel<L, R, true, LASTX, FW>), dim3(grid), dim3(threads), lds, s, d_passes,
                       (const NttC<L, FW>*)d_consts, d_items, nitems);
  else
    hipLaunchKernelGGL((ntt_batch_kernel<L, R, false, LASTX, FW>), dim3(grid), dim3(threads), lds, s, d_passes,
                       (const NttC<L, FW>*)d_consts, d_items, nitems);
  return (int)hipGetLastError();
}

template <int L, int R>
int launch_batch_LR(bool mul, bool lastx, uint32_t threads, size_t lds, uint32_t grid, const NttPassArgs* d_passes,
                    const void* d_consts, const uint2* d_items, uint32_t nitems, hipStream_t s) {
  if constexpr ((R == 2 || R == 3) && kFusedLast<L>) {
    if (lastx)
      return launch_batch_LRX<L, R, true>(mul, threads, lds, grid, d_passes, d_consts, d_items, nitems, s);
  }
  if (lastx) return (int)hipErrorInvalidValue;
  return launch_batch_LRX<L, R, false>(mul, threads, lds, grid, d_passes, d_consts, d_items, nitems, s);
}

template <int L>
int launch_batch_L(uint32_t radix_log, bool mul, bool lastx, bool fw, uint32_t threads, size_t lds, uint32_t grid,
                   const NttPassArgs* d_passes, const void* d_consts, const uint2* d_items, uint32_t nitems,
                   hipStream_t s) {
  if (fw) {
    // full-width modulus: radix-2 and radix-4 units, no cross-lane variant
    if (lastx) return (int)hipErrorInvalidValue;
    if (radix_log == 1)
      return launch_batch_LRX<L, 1, false, true>(mul, threads, lds, grid, d_passes, d_consts, d_items, nitems, s);
    if constexpr (L <= kMaxLimbsRadix4Fw) {
      if (radix_log == 2)
        return launch_batch_LRX<L, 2, false, true>(mul, threads, lds, grid, d_passes, d_consts, d_items, nitems, s);
    }
    return (int)hipErrorInvalidValue;
  }
  if (radix_log == 1)
    return launch_batch_LR<L, 1>(mul, lastx, threads, lds, grid, d_passes, d_consts, d_items, nitems, s);
  if constexpr (L <= kMaxLimbsRadix4) {
    if (radix_log == 2)
      return launch_batch_LR<L, 2>(mul, lastx, threads, lds, grid, d_passes, d_consts, d_items, nitems, s);
  }
  if constexpr (L <= kMaxLimbsRadix8) {
    if (radix_log == 3)
      return launch_batch_LR<L, 3>(mul, lastx, threads, lds, grid, d_passes, d_consts, d_items, nitems, s);
  }
  if constexpr (L <= kMaxLimbsRadix16) {
    if (radix_log == 4)
      return launch_batch_LR<L, 4>(mul, lastx, threads, lds, grid, d_passes, d_consts, d_items, nitems, s);
  }
  return (int)hipErrorInvalidValue;
}

// allow the batch kernels more than 64 KiB of dynamic LDS; called before graph
// capture so that nothing but launches is recorded
template <int L, int R>
void batch_attr_LR() {
  (void)hipFuncSetAttribute((const void*)ntt_batch_kernel<L, R, false, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipFuncSetAttribute((const void*)ntt_batch_kernel<L, R, true, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if constexpr ((R == 2 || R == 3) && kFusedLast<L>) {
    (void)hipFuncSetAttribute((const void*)ntt_batch_kernel<L, R, false, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void*)ntt_batch_kernel<L, R, true, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  }
}

template <int L>
void batch_attr_L(uint32_t radix_log, bool fw) {
  if (fw) {
    const void* k[4] = {(const void*)ntt_batch_kernel<L, 1, false, false, true>,
                        (const void*)ntt_batch_kernel<L, 1, true, false, true>, nullptr, nullptr};
    if constexpr (L <= kMaxLimbsRadix4Fw) {
      k[2] = (const void*)ntt_batch_kernel<L, 2, false, false, true>;
      k[3] = (const void*)ntt_batch_kernel<L, 2, true, false, true>;
    }
    for (const void* f : k)
      if (f) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    return;
  }
  if (radix_log == 1) batch_attr_LR<L, 1>();
  if constexpr (L <= kMaxLimbsRadix4) {
    if (radix_log == 2) batch_attr_LR<L, 2>();
  }
  if constexpr (L <= kMaxLimbsRadix8) {
    if (radix_log == 3) batch_attr_LR<L, 3>();
  }
  if constexpr (L <= kMaxLimbsRadix16) {
    if (radix_log == 4) batch_attr_LR<L, 4>();
  }
}

template <int L>
int launch_tw_L(const FieldRaw& f, const DigitConsts& dc, uint32_t* tw, uint64_t n, uint32_t logn,
                       const uint32_t* d_ladder, hipStream_t s) {
  // the ladder buffer carries one_m and then adj after the logn ladder entries
  const u32* one_m = d_ladder + (size_t)logn * L;
  const u32* adj = one_m + L;
  u64 blocks = (n + 255) / 256;
  if (f.fw) {
    NttC<L, true> c = make_consts<L, true>(f, dc, nullptr);
    hipLaunchKernelGGL((twiddle_kernel<L, true>), dim3((unsigned)blocks), dim3(256), 0, s, tw, n, logn, d_ladder, c,
                       one_m, adj);
  } else {
    NttC<L> c = make_consts<L>(f, dc, nullptr);
    hipLaunchKernelGGL((twiddle_kernel<L>), dim3((unsigned)blocks), dim3(256), 0, s, tw, n, logn, d_ladder, c,
                       one_m, adj);
  }
  return (int)hipGetLastError();
}

// the per-limb-count entry points, instantiated once (in ntt_inst_*.hip)
#define MOMA_NTT_DECLARE(PREFIX, LL)                                                                              \
  PREFIX template int launch_pass_L<LL>(const FieldRaw&, const DigitConsts&, const NttPassArgs&, const NttConsts&, \
                                        uint32_t, uint64_t, uint32_t, uint32_t, hipStream_t);                       \
  PREFIX template int launch_batch_L<LL>(uint32_t, bool, bool, bool, uint32_t, size_t, uint32_t,                  \
                                         const NttPassArgs*, const void*, const uint2*, uint32_t, hipStream_t);     \
  PREFIX template void batch_attr_L<LL>(uint32_t, bool);                                                            \
  PREFIX template int launch_tw_L<LL>(const FieldRaw&, const DigitConsts&, uint32_t*, uint64_t, uint32_t,          \
                                      const uint32_t*, hipStream_t);
#define MOMA_NTT_INSTANTIATE(LL) MOMA_NTT_DECLARE(, LL)
#define MOMA_NTT_EXTERN(LL) MOMA_NTT_DECLARE(extern, LL)

}  // namespace moma
