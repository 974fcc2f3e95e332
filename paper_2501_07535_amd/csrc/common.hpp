// common.hpp - declarations shared by the host runtime and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace moma {

constexpr int kMaxLimbs = 32;
// Digit form of the transform's twiddle multiply: b-bit digits (b = 29, or 28
// above 28 limbs), D of them, so that 2D products of two digits plus a carry
// stay below 2^64 and b*D >= 32L - 2 covers every operand below 4q.
// A full-width modulus (fw: bitlen(q) > 32L - 4) keeps canonical operands
// below q < 2^(32L), so its digits cover 32L bits.
constexpr int digit_bits(int L) { return L <= 28 ? 29 : 28; }
constexpr int digit_count(int L, bool fw = false) {
  return (32 * L - (fw ? 0 : 2) + digit_bits(L) - 1) / digit_bits(L);
}
constexpr int digit_stride(int L, bool fw = false) {  // table words per entry
  return digit_count(L, fw) + (digit_count(L, fw) & 1);
}

// widest limb counts that get radix-4 / radix-8 / radix-16 register units
// (radix 4 up to 16 limbs: 4 elements of 16 limbs plus the digit multiply fit
// the 256 VGPRs of a lane at two waves per SIMD)
constexpr int kMaxLimbsRadix4 = 16;
constexpr int kMaxLimbsRadix8 = 5;
constexpr int kMaxLimbsRadix16 = 2;
// the Karatsuba form of the butterfly's multiply (Eq. (mulk)): radix-2 units,
// 2 to 24 limbs (up to 768 bits, the widths its comparison with schoolbook
// covers; its 2D - 1 live column sums cost registers the wider units lack)
constexpr int kMaxLimbsKara = 24;
// full-width moduli: radix-4 units up to 16 limbs as well
constexpr int kMaxLimbsRadix4Fw = 16;

// Constants of one modulus, sized for the largest limb count; the launchers copy
// the first L words of each array into a compile-time sized kernel argument.
struct FieldRaw {
  int L;                   // compute limbs: ceil((bitlen(q) + 4) / 32), or the storage limbs for a full-width q
  int Ls;                  // storage limbs (planes) given by the caller, >= L
  int fw;                  // full width: bitlen(q) > 32 L - 4, no headroom for lazy reduction
  uint32_t q[kMaxLimbs];
  uint32_t qinv;           // -q^{-1} mod 2^32 (Montgomery)
  uint32_t one_m[kMaxLimbs];  // 2^(32L) mod q (1 in Montgomery form)
  uint32_t qn[kMaxLimbs];  // q * 2^d, bitlen 32L - 4 (Barrett)
  uint32_t mu[kMaxLimbs];  // floor(2^(2(32L-4)+3) / qn)
  uint32_t d;              // Barrett pre-scale shift
  uint32_t r2[kMaxLimbs];  // 2^(64L) mod q: full-width vmul (two Montgomery products)
};

enum BlasOp { OP_VADD = 0, OP_VSUB = 1, OP_VMUL = 2, OP_AXPY = 3 };

struct BlasArgs {
  const uint32_t* a;
  const uint32_t* b;
  uint32_t* out;
  uint64_t n;
  uint32_t alpha_m[kMaxLimbs];  // axpy: alpha * 2^(32L) mod q (Montgomery form)
  uint32_t variant;              // vmul: 0 schoolbook products, 1 Karatsuba (L >= 2)
  uint32_t ls;                   // storage planes (>= L; the planes above L are written as zero)
};

// One pass of the transform: k radix-2 stages [K, K+k) over tiles of C groups.
struct NttPass {
  uint32_t K, k, logc;
  uint64_t tiles;
};

struct NttPassArgs {
  const uint32_t* in;
  const uint32_t* in2;  // first inverse pass of a cyclic product: multiply by in2 pointwise while loading, else NULL
  uint32_t* out;
  const uint32_t* tw;  // twiddle table, element-major, digit_stride(L) words per entry
  uint64_t n;
  uint32_t logn, K, k, logc;
  uint32_t last;       // last pass: store canonical residues in [0, q)
  uint32_t scale;      // multiply by n^-1 on store (last pass of the inverse)
  uint32_t direct;     // set by the pass launcher: the first round reads straight from `in`
};

// Launch shape of a transform: LDS tile of 2^tile_log elements, 2^col_log
// groups per tile in multi-pass plans, threads per workgroup, stages per
// register unit (radix 2^radix_log), and the butterfly's word-product form
// (kara: one level of Karatsuba, Eq. (mulk); 0: schoolbook).
struct NttSchedule {
  uint32_t tile_log, col_log, threads, radix_log;
  uint32_t kara = 0;
};

// arithmetic of a transform kernel: lazy butterflies with the schoolbook or
// the Karatsuba digit product, or canonical ones for a full-width modulus
enum NttArith { kArithLazy = 0, kArithFull = 1, kArithKara = 2 };


struct NttConsts {
  // last-pass scale of the inverse transform, as D b-bit digits: n^{-1} 2^(bD)
  // mod q (times another 2^(bD) after a fused pointwise product)
  uint32_t nscale_d[40];
};

// per-modulus constants of the digit-form multiply
struct DigitConsts {
  uint32_t qd[40];   // q in b-bit digits (digit_count(L, fw) of them)
  uint32_t qinvd;    // -q^{-1} mod 2^b
  uint32_t adj[kMaxLimbs];  // 2^(b*D) mod q, converts a table entry to digit Montgomery form
};

// set the thread's error detail and return code
int set_error(int code, const std::string& detail);

// launchers (return hipError_t as int)
int launch_blas(int op, const FieldRaw& f, const BlasArgs& a, hipStream_t s);
int launch_zero_planes(uint32_t* out, uint64_t n, int from_plane, int to_plane, hipStream_t s);
int launch_ntt_pass(const FieldRaw& f, const DigitConsts& dc, const NttPassArgs& a, const NttConsts& c,
                    uint32_t threads, uint64_t tiles, uint32_t radix_log, uint32_t kara, hipStream_t s);
// batched transforms: one launch runs items (pass record, tile) of many plans
// (fw: full-width moduli, whose kernels and constants are of their own kind)
size_t ntt_consts_bytes(int L, bool fw);
void ntt_batch_prepare(int L, uint32_t radix_log, bool fw, size_t lds);
void ntt_fill_consts(const FieldRaw& f, const DigitConsts& dc, const NttConsts* nc, void* dst);
int launch_ntt_batch(int L, uint32_t radix_log, bool mul, bool variant, bool fw, uint32_t threads, size_t lds,
                     uint32_t grid, const NttPassArgs* d_passes, const void* d_consts, const uint2* d_items,
                     uint32_t nitems, hipStream_t s);
// whether a batch pass record runs the variant kernel (direct first round,
// cross-lane last stage); sets the record's `direct` flag
bool ntt_batch_variant(int L, uint32_t radix_log, uint32_t threads, NttPassArgs* a);
// largest workgroup the pass kernel for (L, radix_log) was compiled for
uint32_t ntt_max_threads(int L, uint32_t radix_log);
int launch_twiddle_gen(const FieldRaw& f, const DigitConsts& dc, uint32_t* tw, uint64_t n, uint32_t logn,
                       const uint32_t* d_ladder, hipStream_t s);


}  // namespace moma

// expand CASE(L) for every supported compute limb count
#define MOMA_FOR_EACH_L(CASE)                                                                                     \
  CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13)    \
  CASE(14) CASE(15) CASE(16) CASE(17) CASE(18) CASE(19) CASE(20) CASE(21) CASE(22) CASE(23) CASE(24) CASE(25)    \
  CASE(26) CASE(27) CASE(28) CASE(29) CASE(30) CASE(31) CASE(32)
