// probe.hip - measured issue rates and bandwidths that price the roofline of
// the transform and BLAS kernels (moma_measure_peaks).
//
// The integer work of a modular multiply is word products and carry
// propagation (Section 2.2's rules (mulqdd), (adc)); on gfx950 a word product
// with its 64-bit accumulation is one v_mad_u64_u32, a carry step one
// v_addc_co_u32.  The vendor peak counts full-rate 32-bit lane operations
// (256 CUs x 4 SIMDs x 16 lanes x clock); how fast each of these instructions
// actually issues is measured here, on independent chains spread over every
// SIMD so that latency is hidden and only issue throughput counts.  The HBM
// probes stream large buffers with one and two reads per write.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string.h>
#include <vector>

#include "../../include/moma.h"
#include "common.hpp"
#include "plan.hpp"

namespace moma {

typedef uint32_t u32;
typedef uint64_t u64;

enum ProbeOp { PR_ADD = 0, PR_ADDC = 1, PR_MAD64 = 2, PR_MULLO = 3, PR_MULHI = 4, PR_MADC = 5 };
constexpr int kChains = 8;  // independent dependency chains per lane
constexpr int kUnroll = 4;  // rounds per loop iteration (keeps loop control off the count)

// Each lane runs kUnroll * iters rounds of kChains independent instructions of one
// kind (PR_ADDC: an add and an add-with-carry per chain; PR_MADC: a word product
// and the add-with-carry that takes its carry-out; both count two instructions).
// The result is folded into one word per lane and written, so nothing is dead.
template <int OP>
__global__ __launch_bounds__(256) void probe_valu_kernel(u32* __restrict__ out, u32 iters, u32 seed) {
  const u32 gid = blockIdx.x * blockDim.x + threadIdx.x;
  u32 y = seed ^ (gid * 0x9e3779b9u);
  u32 a[kChains], b[kChains];
  u64 acc[kChains];
#pragma unroll
  for (int k = 0; k < kChains; k++) {
    a[k] = gid * (2u * k + 3u) + seed;
    b[k] = a[k] ^ 0x5bd1e995u;
    acc[k] = a[k];
  }
  for (u32 i = 0; i < iters; i++) {
#pragma unroll
    for (int kk = 0; kk < kUnroll * kChains; kk++) {
      const int k = kk % kChains;
      if constexpr (OP == PR_ADD) {
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[k]) : "v"(y));
      } else if constexpr (OP == PR_ADDC) {
        u64 cy;
        asm volatile(
            "v_add_co_u32 %0, %2, %0, %3\n\t"
            "v_addc_co_u32 %1, %2, %1, %3, %2"
            : "+v"(a[k]), "+v"(b[k]), "=&s"(cy)
            : "v"(y));
      } else if constexpr (OP == PR_MAD64) {
        u64 cy;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[k]), "=s"(cy) : "v"(a[k]), "v"(y));
      } else if constexpr (OP == PR_MADC) {
        // a word product accumulated into 64 bits whose carry-out moves into a
        // third word: one step of product scanning with carries
        u64 cy;
        asm volatile(
            "v_mad_u64_u32 %0, %2, %3, %4, %0\n\t"
            "v_addc_co_u32 %1, %2, %1, 0, %2"
            : "+v"(acc[k]), "+v"(b[k]), "=&s"(cy)
            : "v"(a[k]), "v"(y));
      } else if constexpr (OP == PR_MULLO) {
        asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[k]) : "v"(y));
      } else {
        asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[k]) : "v"(y));
      }
    }
  }
  u32 r = 0;
#pragma unroll
  for (int k = 0; k < kChains; k++) r ^= a[k] ^ b[k] ^ (u32)acc[k] ^ (u32)(acc[k] >> 32);
  out[gid] = r;
}

// dst[i] = src[i], 16 bytes per lane per step, grid-stride over `vecs` uint4s
__global__ __launch_bounds__(256) void probe_copy_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                         u64 vecs) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < vecs; i += (u64)gridDim.x * blockDim.x) dst[i] = src[i];
}

// dst[i] = a[i] + b[i] (word-wise), two reads per write
__global__ __launch_bounds__(256) void probe_triad_kernel(uint4* __restrict__ dst, const uint4* __restrict__ a,
                                                          const uint4* __restrict__ b, u64 vecs) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < vecs; i += (u64)gridDim.x * blockDim.x) {
    uint4 x = a[i], y = b[i];
    dst[i] = make_uint4(x.x + y.x, x.y + y.y, x.z + y.z, x.w + y.w);
  }
}

// Best of `reps` timed launches (after one warm-up) of fn, in seconds.
template <class F>
static int best_time(F fn, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1, double* sec) {
  int e = fn();
  if (e) return e;
  double best = 1e30;
  for (int r = 0; r < reps; r++) {
    if ((e = (int)hipEventRecord(e0, s))) return e;
    if ((e = fn())) return e;
    if ((e = (int)hipEventRecord(e1, s))) return e;
    if ((e = (int)hipEventSynchronize(e1))) return e;
    float ms = 0;
    if ((e = (int)hipEventElapsedTime(&ms, e0, e1))) return e;
    best = std::min(best, (double)ms * 1e-3);
  }
  *sec = best;
  return 0;
}

template <int OP>
static int probe_valu(u32* d_out, u32 blocks, u32 iters, hipStream_t s, hipEvent_t e0, hipEvent_t e1, double* rate) {
  double sec = 0;
  int e = best_time(
      [&]() {
        hipLaunchKernelGGL((probe_valu_kernel<OP>), dim3(blocks), dim3(256), 0, s, d_out, iters, 12345u);
        return (int)hipGetLastError();
      },
      3, s, e0, e1, &sec);
  if (e) return e;
  const double per_chain = (OP == PR_ADDC || OP == PR_MADC) ? 2.0 : 1.0;
  *rate = (double)blocks * 256.0 * iters * kUnroll * kChains * per_chain / sec;
  return 0;
}

}  // namespace moma

using namespace moma;

extern "C" int moma_measure_peaks(moma_peak_rates_t* out, uint64_t hbm_bytes, void* stream) {
  if (!out) return set_error(MOMA_E_ARG, "out is NULL");
  if (hbm_bytes == 0) hbm_bytes = 1ull << 30;
  if (hbm_bytes < (1ull << 20) || hbm_bytes > (16ull << 30))
    return set_error(MOMA_E_ARG, "hbm_bytes must be in [1 MiB, 16 GiB]");
  memset(out, 0, sizeof(*out));
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  // 16 workgroups of 4 waves per compute unit: 16 waves per SIMD, enough
  // independent chains to hide every latency
  const u32 blocks = (u32)cus * 16u;
  const u32 iters = 2048;
  const u64 vecs = hbm_bytes / 16;
  u32* d_valu = nullptr;
  uint4 *d_a = nullptr, *d_b = nullptr, *d_c = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int e = (int)hipMalloc((void**)&d_valu, (size_t)blocks * 256 * sizeof(u32));
  if (!e) e = (int)hipMalloc((void**)&d_a, vecs * 16);
  if (!e) e = (int)hipMalloc((void**)&d_b, vecs * 16);
  if (!e) e = (int)hipMalloc((void**)&d_c, vecs * 16);
  if (e) {
    (void)hipFree(d_valu);
    (void)hipFree(d_a);
    (void)hipFree(d_b);
    (void)hipFree(d_c);
    return set_error(MOMA_E_NOMEM, "probe buffers");
  }
  if (!e) e = (int)hipMemsetAsync(d_a, 1, vecs * 16, s);
  if (!e) e = (int)hipMemsetAsync(d_b, 2, vecs * 16, s);
  if (!e) e = (int)hipEventCreate(&e0);
  if (!e) e = (int)hipEventCreate(&e1);
  if (!e) e = probe_valu<PR_ADD>(d_valu, blocks, iters, s, e0, e1, &out->add_u32);
  if (!e) e = probe_valu<PR_ADDC>(d_valu, blocks, iters, s, e0, e1, &out->add_co_addc_u32);
  if (!e) e = probe_valu<PR_MAD64>(d_valu, blocks, iters, s, e0, e1, &out->mad_u64_u32);
  if (!e) e = probe_valu<PR_MADC>(d_valu, blocks, iters, s, e0, e1, &out->mad_addc_u32);
  if (!e) e = probe_valu<PR_MULLO>(d_valu, blocks, iters, s, e0, e1, &out->mul_lo_u32);
  if (!e) e = probe_valu<PR_MULHI>(d_valu, blocks, iters, s, e0, e1, &out->mul_hi_u32);
  // bandwidth: a grid of 4096 workgroups striding over the buffers
  const u32 hb = 4096;
  double sec = 0;
  if (!e)
    e = best_time(
        [&]() {
          hipLaunchKernelGGL(probe_copy_kernel, dim3(hb), dim3(256), 0, s, d_c, (const uint4*)d_a, vecs);
          return (int)hipGetLastError();
        },
        5, s, e0, e1, &sec);
  if (!e) out->hbm_copy = 2.0 * vecs * 16 / sec;
  if (!e)
    e = best_time(
        [&]() {
          hipLaunchKernelGGL(probe_triad_kernel, dim3(hb), dim3(256), 0, s, d_c, (const uint4*)d_a, (const uint4*)d_b,
                             vecs);
          return (int)hipGetLastError();
        },
        5, s, e0, e1, &sec);
  if (!e) out->hbm_triad = 3.0 * vecs * 16 / sec;
  if (!e) e = (int)hipStreamSynchronize(s);
  out->compute_units = (uint32_t)cus;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d_valu);
  (void)hipFree(d_a);
  (void)hipFree(d_b);
  (void)hipFree(d_c);
  return e ? hip_fail(e, "peak probes") : MOMA_OK;
}
