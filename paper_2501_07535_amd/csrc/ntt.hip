// ntt.hip - run-time dispatch of the transform kernels on the compute limb
// count; the kernels and their launchers are in ntt_impl.hpp.
#include <atomic>

#include "ntt_impl.hpp"

namespace moma {

MOMA_FOR_EACH_L(MOMA_NTT_EXTERN)

// compute units of the current device (cached per device ordinal; several
// host threads may ask at once)
uint32_t device_cu_count() {
  static std::atomic<uint32_t> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  uint32_t c = cache[dev].load(std::memory_order_relaxed);
  if (!c) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    c = (uint32_t)v;
    cache[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

uint32_t ntt_max_threads(int L, uint32_t radix_log) {
  int live = L << radix_log;
  return live <= 16 ? 1024u : (live <= 32 ? 512u : 256u);
}

int launch_ntt_pass(const FieldRaw& f, const DigitConsts& dc, const NttPassArgs& a, const NttConsts& c,
                    uint32_t threads, uint64_t tiles, uint32_t radix_log, uint32_t kara, hipStream_t s) {
  switch (f.L) {
#define CASE(LL) \
  case LL: return launch_pass_L<LL>(f, dc, a, c, threads, tiles, radix_log, kara, s);
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
  return (int)hipErrorInvalidValue;
}

bool ntt_batch_variant(int L, uint32_t radix_log, uint32_t threads, NttPassArgs* a) {
  return batch_variant(L, radix_log, threads, a);
}

int launch_ntt_batch(int L, uint32_t radix_log, bool mul, bool variant, bool fw, uint32_t threads, size_t lds,
                     uint32_t grid, const NttPassArgs* d_passes, const void* d_consts, const uint2* d_items,
                     uint32_t nitems, hipStream_t s) {
  switch (L) {
#define CASE(LL)                                                                                                 \
  case LL:                                                                                                       \
    return launch_batch_L<LL>(radix_log, mul, variant, fw, threads, lds, grid, d_passes, d_consts, d_items,      \
                              nitems, s);
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
  return (int)hipErrorInvalidValue;
}

void ntt_batch_prepare(int L, uint32_t radix_log, bool fw, size_t lds) {
  if (lds <= 65536) return;
  switch (L) {
#define CASE(LL) \
  case LL: batch_attr_L<LL>(radix_log, fw); return;
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
}

size_t ntt_consts_bytes(int L, bool fw) {
  switch (L) {
#define CASE(LL) \
  case LL: return fw ? sizeof(NttC<LL, true>) : sizeof(NttC<LL>);
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
  return 0;
}

void ntt_fill_consts(const FieldRaw& f, const DigitConsts& dc, const NttConsts* nc, void* dst) {
  switch (f.L) {
#define CASE(LL)                                          \
  case LL: {                                              \
    if (f.fw) {                                           \
      NttC<LL, true> c = make_consts<LL, true>(f, dc, nc); \
      memcpy(dst, &c, sizeof(c));                         \
    } else {                                              \
      NttC<LL> c = make_consts<LL>(f, dc, nc);            \
      memcpy(dst, &c, sizeof(c));                         \
    }                                                     \
    return;                                               \
  }
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
}

int launch_twiddle_gen(const FieldRaw& f, const DigitConsts& dc, uint32_t* tw, uint64_t n, uint32_t logn,
                       const uint32_t* d_ladder, hipStream_t s) {
  switch (f.L) {
#define CASE(LL) \
  case LL: return launch_tw_L<LL>(f, dc, tw, n, logn, d_ladder, s);
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
  return (int)hipErrorInvalidValue;
}

}  // namespace moma
