// ntt.hip - number theoretic transform kernels (paper Eq. (ntt), Section 5.3).
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
//   * Twiddle table: entry m + i' (m = 2^s) holds w_{2m}^{i'} in Montgomery form
//     (level s stores the first m powers of w_{2m}).  With that order the C
//     groups of a tile read C consecutive entries, and the first pass reads a
//     table prefix shared by every tile.
// Every butterfly is one mont_mul (V*W), one mod_add and one mod_sub.
#include "common.hpp"
#include "limb.hpp"

namespace moma {

template <int L>
struct NttC {
  u32 q[L];
  u32 qinv;
  u32 nscale[L];  // n^-1 in Montgomery form (inverse transform, last pass)
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

// One pass: stages [K, K+k) on tiles of C = 2^logc groups of 2^k elements.
// LDS holds the tile limb-planar: word (j * 2^k + u) * C + g is limb j of row u
// of group g, so lanes with consecutive g touch consecutive banks.
template <int L>
__global__ __launch_bounds__(256) void ntt_pass_kernel(NttPassArgs a, NttC<L> c) {
  extern __shared__ u32 lds[];
  const u32 k = a.k, logc = a.logc, K = a.K;
  const u32 C = 1u << logc;
  const u32 rows = 1u << k;
  const u32 E = rows << logc;
  const u64 n = a.n;
  const u32 T = blockDim.x;
  const u32 tid = threadIdx.x;
  const u64 tile = blockIdx.x;

  // tile -> (base address, first group); see the file comment for the layout
  u64 o0 = 0, ro = 0, b0 = 0;
  u64 S = n >> (K + k);
  if (K == 0) {
    o0 = tile << logc;
  } else {
    u64 per = (1ull << K) >> logc;
    ro = tile / per;
    b0 = (tile % per) << logc;
  }

  // ---- load
  for (u32 e = tid; e < E; e += T) {
    u32 g = e & (C - 1), v = e >> logc;
    u64 src;
    u32 u;
    if (K == 0) {
      u = v;
      src = (u64)u * S + o0 + g;
    } else {
      u = rev_bits(v, k);
      src = (ro << (K + k)) + ((u64)v << K) + b0 + g;
    }
#pragma unroll
    for (int j = 0; j < L; j++) lds[(j * rows + u) * C + g] = a.in[(u64)j * n + src];
  }
  __syncthreads();

  // ---- stages
  for (u32 sg = 0; sg < k; sg++) {
    const u32 hb = k - sg - 1;
    const u32 h = 1u << hb;
    for (u32 b = tid; b < (E >> 1); b += T) {
      u32 g = b & (C - 1), r = b >> logc;
      u32 lb = r >> hb, pos = r & (h - 1);
      u32 u1 = (lb << (hb + 1)) + pos, u2 = u1 + h;
      u64 twpos = (K == 0) ? ((1ull << sg) + rev_bits(lb, sg))
                           : ((1ull << (K + sg)) + ((u64)rev_bits(lb, sg) << K) + b0 + g);
      u32 w[L], x[L], y[L], t[L];
      load_entry<L>(w, a.tw + twpos * L);
#pragma unroll
      for (int j = 0; j < L; j++) {
        x[j] = lds[(j * rows + u1) * C + g];
        y[j] = lds[(j * rows + u2) * C + g];
      }
      mont_mul<L>(t, y, w, c.q, c.qinv);
      u32 s0[L], s1[L];
      mod_add<L>(s0, x, t, c.q);
      mod_sub<L>(s1, x, t, c.q);
#pragma unroll
      for (int j = 0; j < L; j++) {
        lds[(j * rows + u1) * C + g] = s0[j];
        lds[(j * rows + u2) * C + g] = s1[j];
      }
    }
    __syncthreads();
  }

  // ---- store
  const u32 logn = a.logn;
  for (u32 e = tid; e < E; e += T) {
    u32 g, v, u;
    u64 dst;
    if (K == 0) {
      // consecutive lanes write consecutive addresses inside one group's run
      g = e >> k;
      v = e & (rows - 1);
      u = rev_bits(v, k);
      dst = ((u64)rev_bits((u32)(o0 + g), logn - k) << k) + v;
    } else {
      g = e & (C - 1);
      v = e >> logc;
      u = rev_bits(v, k);
      dst = (ro << (K + k)) + ((u64)v << K) + b0 + g;
    }
    u32 x[L];
#pragma unroll
    for (int j = 0; j < L; j++) x[j] = lds[(j * rows + u) * C + g];
    if (a.scale) {
      u32 s[L];
      mont_mul<L>(s, x, c.nscale, c.q, c.qinv);
#pragma unroll
      for (int j = 0; j < L; j++) a.out[(u64)j * n + dst] = s[j];
    } else {
#pragma unroll
      for (int j = 0; j < L; j++) a.out[(u64)j * n + dst] = x[j];
    }
  }
}

// Twiddle table: entry e = 2^s + i' holds w^(i' * 2^(logn-s-1)) * 2^(32L) mod q.
// ladder[b] = w^(2^b) * 2^(32L) mod q; the product of the ladder entries for the
// set bits of the exponent stays in Montgomery form.
template <int L>
__global__ __launch_bounds__(256) void twiddle_kernel(u32* __restrict__ tw, u64 n, u32 logn,
                                                      const u32* __restrict__ ladder, NttC<L> c,
                                                      const u32* __restrict__ one_m) {
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
        mont_mul<L>(t, acc, w, c.q, c.qinv);
#pragma unroll
        for (int j = 0; j < L; j++) acc[j] = t[j];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < L; j++) tw[e * L + j] = acc[j];
}

uint32_t ntt_tile_elems(int L) {
  // 64 KiB of LDS per tile keeps two or more workgroups resident per CU
  uint32_t words = 16384u / (uint32_t)L;
  uint32_t e = 1;
  while (e * 2 <= words) e *= 2;
  return e;
}

template <int L>
static NttC<L> make_consts(const FieldRaw& f, const NttConsts* nc) {
  NttC<L> c;
  for (int j = 0; j < L; j++) {
    c.q[j] = f.q[j];
    c.nscale[j] = nc ? nc->nscale_m[j] : 0;
  }
  c.qinv = f.qinv;
  return c;
}

template <int L>
static int launch_pass_L(const FieldRaw& f, const NttPassArgs& a, const NttConsts& nc, uint32_t threads,
                         uint64_t tiles, hipStream_t s) {
  NttC<L> c = make_consts<L>(f, &nc);
  size_t lds = (size_t)L * ((size_t)1 << (a.k + a.logc)) * sizeof(u32);
  hipLaunchKernelGGL((ntt_pass_kernel<L>), dim3((unsigned)tiles), dim3(threads), lds, s, a, c);
  return (int)hipGetLastError();
}

int launch_ntt_pass(const FieldRaw& f, const NttPassArgs& a, const NttConsts& c, uint32_t threads, uint64_t tiles,
                    hipStream_t s) {
  switch (f.L) {
#define CASE(LL) \
  case LL: return launch_pass_L<LL>(f, a, c, threads, tiles, s);
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
  return (int)hipErrorInvalidValue;
}

template <int L>
static int launch_tw_L(const FieldRaw& f, uint32_t* tw, uint64_t n, uint32_t logn, const uint32_t* d_ladder,
                       hipStream_t s) {
  NttC<L> c = make_consts<L>(f, nullptr);
  // the ladder buffer carries one_m after the logn ladder entries
  const u32* one_m = d_ladder + (size_t)logn * L;
  u64 blocks = (n + 255) / 256;
  hipLaunchKernelGGL((twiddle_kernel<L>), dim3((unsigned)blocks), dim3(256), 0, s, tw, n, logn, d_ladder, c, one_m);
  return (int)hipGetLastError();
}

int launch_twiddle_gen(const FieldRaw& f, uint32_t* tw, uint64_t n, uint32_t logn, const uint32_t* d_ladder,
                       hipStream_t s) {
  switch (f.L) {
#define CASE(LL) \
  case LL: return launch_tw_L<LL>(f, tw, n, logn, d_ladder, s);
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
  return (int)hipErrorInvalidValue;
}

}  // namespace moma
