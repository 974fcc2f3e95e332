// noalloc.hip - the cyclic product for callers that cannot allocate device
// memory (code under graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  It runs the same kernels as moma_ntt_cyclic_mul; only the
// buffers of the two spectra come from a fixed library-wide device array
// instead of the plan.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/moma.h"
#include "plan.hpp"

namespace moma {

// Library-wide scratch of the allocation-free cyclic product.  Each GPU the
// library runs on holds its own copy (the code object's global memory on that
// device) until the process ends.  In host code `scratch` names a host-side
// stand-in, not a device address: kernels and copies only ever get the address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint32_t scratch[MOMA_NOALLOC_SCRATCH_WORDS];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint32_t* g_scratch_ptr[kMaxDevices];  // per device ordinal; NULL until looked up

// The current device's copy of `scratch`, looked up once per device (with that
// device current) on its first call.
static int scratch_on_current_device(uint32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail((int)e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return set_error(MOMA_E_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail((int)e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(MOMA_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return MOMA_OK;
}

}  // namespace moma

using namespace moma;

extern "C" int moma_ntt_cyclic_mul_noalloc(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs,
                                           const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_out,
                                           void* stream) {
  if (!d_a || !d_b || !d_out) return set_error(MOMA_E_ARG, "device pointer is NULL");
  std::shared_ptr<NttPlan> p;
  int rc = find_plan(q, omega, n, limbs, &p);
  if (rc) return rc;
  const uint64_t need = cyclic_mul_scratch_words(*p);
  if (need > (uint64_t)MOMA_NOALLOC_SCRATCH_WORDS)
    return set_error(MOMA_E_ARG, "the allocation-free cyclic product needs " + std::to_string(need) +
                                     " scratch words, more than its fixed " +
                                     std::to_string((uint64_t)MOMA_NOALLOC_SCRATCH_WORDS));
  uint32_t* ws = nullptr;
  rc = scratch_on_current_device(&ws);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (input_check_on()) {
    // the per-workgroup counts use the head of the scratch; the check waits
    // for the stream before the spectra are enqueued over it
    const uint32_t* xs[2] = {d_a, d_b};
    rc = check_inputs(p->fe->f, xs, 2, n, s, ws);
    if (rc) return rc;
  }
  return run_cyclic_mul(*p, d_a, d_b, d_out, s, ws);
}
