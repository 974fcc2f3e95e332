// blas.hip - elementwise modular BLAS kernels (paper Section 2.3 / Section 5.2).
//
// One lane per element, limb-planar layout: a wavefront's load of limb j is 64
// consecutive words (256 bytes), so every access is fully coalesced.  vadd and
// vsub are HBM-bound (3 * 4L bytes per element against ~3L VALU ops); vmul and
// axpy carry an L-limb modular multiply per element.
#include <string.h>

#include "common.hpp"
#include "limb.hpp"
#include "plan.hpp"

namespace moma {

template <int L>
struct BlasC {
  u32 q[L];
  u32 qinv;
  BarrettC<L> bc;
  u32 alpha_m[L];
  u32 r2[L];  // 2^(64L) mod q (full-width vmul)
};

// One element's operation.  A full-width modulus (FW: no headroom for Barrett's
// pre-scaled modulus) multiplies by Montgomery products that keep the carry
// out of the top limb: vmul = mont(mont(a, b), 2^(64L) mod q).
template <int L, int OP, bool KARA, bool FW>
__device__ __forceinline__ void blas_elem(u32* r, const u32* a, const u32* b, const BlasC<L>& c) {
  if constexpr (FW) {
    u32 qv[L];
    to_vgprs<L>(qv, c.q);
    if constexpr (OP == OP_VADD) {
      mod_add_fw<L>(r, a, b, qv);
    } else if constexpr (OP == OP_VSUB) {
      mod_sub_v<L>(r, a, b, qv);
    } else if constexpr (OP == OP_VMUL) {
      u32 t[L], r2v[L];
      mont_mul_fw<L>(t, a, b, c.q, c.qinv, qv);    // a b 2^(-32L)
      to_vgprs<L>(r2v, c.r2);
      mont_mul_fw<L>(r, t, r2v, c.q, c.qinv, qv);  // times 2^(64L) 2^(-32L)
    } else {
      u32 t[L], av[L];
      to_vgprs<L>(av, c.alpha_m);
      mont_mul_fw<L>(t, a, av, c.q, c.qinv, qv);   // alpha * x
      mod_add_fw<L>(r, t, b, qv);                  // + y
    }
  } else {
    if constexpr (OP == OP_VADD) {
      mod_add<L>(r, a, b, c.q);
    } else if constexpr (OP == OP_VSUB) {
      mod_sub<L>(r, a, b, c.q);
    } else if constexpr (OP == OP_VMUL) {
      barrett_mul<L, KARA>(r, a, b, c.bc);
    } else {
      u32 t[L];
      mont_mul<L>(t, a, c.alpha_m, c.q, c.qinv);  // alpha * x
      mod_add<L>(r, t, b, c.q);                   // + y
    }
  }
}

// One element per lane.  Every word is streamed once, so loads and stores are
// nontemporal (no reuse to keep in the caches).  Four elements per lane with
// 16-byte accesses was measured at n = 2^24: vadd at 256 bits took 333 us
// against 280 us with one element per lane.
template <int L, int OP, bool KARA, bool FW>
__global__ __launch_bounds__(256) void blas_kernel(const u32* __restrict__ pa, const u32* __restrict__ pb,
                                                   u32* __restrict__ pout, u64 n, BlasC<L> c) {
  const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  u32 a[L], b[L], r[L];
#pragma unroll
  for (int j = 0; j < L; j++) {
    a[j] = __builtin_nontemporal_load(pa + (u64)j * n + i);
    b[j] = __builtin_nontemporal_load(pb + (u64)j * n + i);
  }
  blas_elem<L, OP, KARA, FW>(r, a, b, c);
#pragma unroll
  for (int j = 0; j < L; j++) __builtin_nontemporal_store(r[j], pout + (u64)j * n + i);
}

template <int L, int OP, bool KARA, bool FW>
static int launch_blas_LK(const BlasArgs& a, const BlasC<L>& c, hipStream_t s) {
  const unsigned T = 256;
  const u64 blocks = (a.n + T - 1) / T;
  hipLaunchKernelGGL((blas_kernel<L, OP, KARA, FW>), dim3((unsigned)blocks), dim3(T), 0, s, a.a, a.b, a.out, a.n,
                     c);
  return (int)hipGetLastError();
}

template <int L>
static BlasC<L> blas_consts(const FieldRaw& f, const BlasArgs& a) {
  BlasC<L> c;
  memset(&c, 0, sizeof(c));
  for (int j = 0; j < L; j++) {
    c.q[j] = f.q[j];
    c.bc.qn[j] = f.qn[j];
    c.bc.mu[j] = f.mu[j];
    c.alpha_m[j] = a.alpha_m[j];
    c.r2[j] = f.r2[j];
  }
  c.qinv = f.qinv;
  c.bc.d = f.d;
  return c;
}

// A full-width modulus runs the Montgomery products (the product variant is a
// choice of Barrett's products and does not apply).
template <int L, int OP>
static int launch_blas_L(const FieldRaw& f, const BlasArgs& a, hipStream_t s) {
  BlasC<L> c = blas_consts<L>(f, a);
  if (f.fw) return launch_blas_LK<L, OP, false, true>(a, c, s);
  if constexpr (OP == OP_VMUL && L >= 2) {
    if (a.variant == 1) return launch_blas_LK<L, OP, true, false>(a, c, s);
  }
  return launch_blas_LK<L, OP, false, false>(a, c, s);
}

template <int L>
static int launch_blas_op(int op, const FieldRaw& f, const BlasArgs& a, hipStream_t s) {
  switch (op) {
    case OP_VADD: return launch_blas_L<L, OP_VADD>(f, a, s);
    case OP_VSUB: return launch_blas_L<L, OP_VSUB>(f, a, s);
    case OP_VMUL: return launch_blas_L<L, OP_VMUL>(f, a, s);
    case OP_AXPY: return launch_blas_L<L, OP_AXPY>(f, a, s);
  }
  return (int)hipErrorInvalidValue;
}

int launch_blas(int op, const FieldRaw& f, const BlasArgs& a, hipStream_t s) {
  if (a.n == 0) return 0;
  switch (f.L) {
#define CASE(LL) \
  case LL: return launch_blas_op<LL>(op, f, a, s);
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
  return (int)hipErrorInvalidValue;
}

// ---------------------------------------------------------------- batched
//
// Many BLAS calls of one (op, compute limbs, product variant) in one launch:
// workgroup w runs item w = (job record, block of 256 elements); every record
// carries its own vectors, length and modulus constants.  Items are ordered
// job by job, so the blocks of a vector stay together.

template <int L, int OP, bool KARA, bool FW>
__global__ __launch_bounds__(256) void blas_batch_kernel(const BlasJobRec* __restrict__ recs,
                                                         const BlasC<L>* __restrict__ consts,
                                                         const uint2* __restrict__ items, u32 nitems) {
  const u32 w = blockIdx.x;
  if (w >= nitems) return;
  const uint2 it = items[w];
  const BlasJobRec* rec = recs + it.x;
  BlasJobRec r = *rec;
  r.a = load_global_ptr(&rec->a);
  r.b = load_global_ptr(&rec->b);
  r.out = load_global_ptr(&rec->out);
  const BlasC<L> c = consts[it.x];
  const u64 i = (u64)it.y * blockDim.x + threadIdx.x;
  if (i >= r.n) return;
  const u64 n = r.n;
  u32 a[L], bb[L], res[L];
#pragma unroll
  for (int j = 0; j < L; j++) {
    a[j] = r.a[(u64)j * n + i];
    bb[j] = r.b[(u64)j * n + i];
  }
  blas_elem<L, OP, KARA, FW>(res, a, bb, c);
#pragma unroll
  for (int j = 0; j < L; j++) r.out[(u64)j * n + i] = res[j];
}

size_t blas_consts_bytes(int L) {
  switch (L) {
#define CASE(LL) \
  case LL: return sizeof(BlasC<LL>);
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
  return 0;
}

void blas_fill_consts(const FieldRaw& f, const BlasArgs& a, void* dst) {
  switch (f.L) {
#define CASE(LL)                                  \
  case LL: {                                      \
    BlasC<LL> c = blas_consts<LL>(f, a);          \
    memcpy(dst, &c, sizeof(c));                   \
    return;                                       \
  }
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
}

template <int L, int OP, bool KARA, bool FW = false>
static int launch_blas_batch_LOK(const void* recs, const void* consts, const uint2* items, uint32_t nitems,
                                 hipStream_t s) {
  hipLaunchKernelGGL((blas_batch_kernel<L, OP, KARA, FW>), dim3(nitems), dim3(256), 0, s, (const BlasJobRec*)recs,
                     (const BlasC<L>*)consts, items, nitems);
  return (int)hipGetLastError();
}

template <int L>
static int launch_blas_batch_L(int op, uint32_t variant, bool fw, const void* recs, const void* consts,
                               const uint2* items, uint32_t nitems, hipStream_t s) {
  if (fw) {
    switch (op) {
      case OP_VADD: return launch_blas_batch_LOK<L, OP_VADD, false, true>(recs, consts, items, nitems, s);
      case OP_VSUB: return launch_blas_batch_LOK<L, OP_VSUB, false, true>(recs, consts, items, nitems, s);
      case OP_VMUL: return launch_blas_batch_LOK<L, OP_VMUL, false, true>(recs, consts, items, nitems, s);
      case OP_AXPY: return launch_blas_batch_LOK<L, OP_AXPY, false, true>(recs, consts, items, nitems, s);
    }
    return (int)hipErrorInvalidValue;
  }
  switch (op) {
    case OP_VADD: return launch_blas_batch_LOK<L, OP_VADD, false>(recs, consts, items, nitems, s);
    case OP_VSUB: return launch_blas_batch_LOK<L, OP_VSUB, false>(recs, consts, items, nitems, s);
    case OP_VMUL:
      if constexpr (L >= 2) {
        if (variant == 1) return launch_blas_batch_LOK<L, OP_VMUL, true>(recs, consts, items, nitems, s);
      }
      return launch_blas_batch_LOK<L, OP_VMUL, false>(recs, consts, items, nitems, s);
    case OP_AXPY: return launch_blas_batch_LOK<L, OP_AXPY, false>(recs, consts, items, nitems, s);
  }
  return (int)hipErrorInvalidValue;
}

int launch_blas_batch(int op, int L, uint32_t variant, bool fw, const void* recs, const void* consts,
                      const uint2* items, uint32_t nitems, hipStream_t s) {
  if (nitems == 0) return 0;
  switch (L) {
#define CASE(LL) \
  case LL: return launch_blas_batch_L<LL>(op, variant, fw, recs, consts, items, nitems, s);
    MOMA_FOR_EACH_L(CASE)
#undef CASE
  }
  return (int)hipErrorInvalidValue;
}

__global__ __launch_bounds__(256) void zero_planes_kernel(u32* out, u64 n, int from, int to) {
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = from; j < to; j++) out[(u64)j * n + i] = 0;
}

int launch_zero_planes(uint32_t* out, uint64_t n, int from_plane, int to_plane, hipStream_t s) {
  if (n == 0 || from_plane >= to_plane) return 0;
  u64 blocks = (n + 255) / 256;
  hipLaunchKernelGGL(zero_planes_kernel, dim3((unsigned)blocks), dim3(256), 0, s, out, n, from_plane, to_plane);
  return (int)hipGetLastError();
}

}  // namespace moma

namespace moma {

// Timing inputs: word i of plane j is a hash of (i, seed); planes below the
// top limb of q are uniform, the top limb is masked below q's top limb, the
// planes above it are zero, so every element is a residue below q.
__global__ __launch_bounds__(256) void fill_residues_kernel(u32* __restrict__ p, u64 n, int planes, int top,
                                                            u32 top_mask, u32 seed) {
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * (u64)planes) return;
  int j = (int)(i / n);
  u32 x = (u32)i ^ (u32)(i >> 32) * 0x9e3779b9u ^ seed;
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  p[i] = j < top ? x : (j == top ? (x & top_mask) : 0u);
}

int launch_fill_residues(uint32_t* p, uint64_t n, int planes, int top, uint32_t top_mask, uint32_t seed,
                         hipStream_t s) {
  u64 count = n * (u64)planes;
  if (count == 0) return 0;
  hipLaunchKernelGGL(fill_residues_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, n, planes, top,
                     top_mask, seed);
  return (int)hipGetLastError();
}

// Input check: counts the elements of a limb-planar vector that are not
// canonical, i.e. whose value over all `ls` storage planes is >= q.  Each
// workgroup writes its own count to partial[blockIdx.x]; there are no atomics.
struct QWords {
  u32 w[kMaxLimbs];
};

__global__ __launch_bounds__(256) void count_noncanonical_kernel(const u32* __restrict__ x, u64 n, int ls, QWords q,
                                                                 u32* __restrict__ partial) {
  __shared__ u32 red[256];
  u32 bad = 0;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
    // compare from the top word down: the first differing word decides
    int state = 0;  // 0 equal so far, 1 x > q, -1 x < q
    for (int j = ls - 1; j >= 0; j--) {
      u32 v = x[(u64)j * n + i];
      if (state == 0 && v != q.w[j]) state = v > q.w[j] ? 1 : -1;
    }
    bad += state >= 0 ? 1u : 0u;
  }
  red[threadIdx.x] = bad;
  __syncthreads();
  for (u32 s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

int launch_count_noncanonical(const uint32_t* q, int ls, const uint32_t* d_x, uint64_t n, uint32_t* d_partial,
                              uint32_t blocks, hipStream_t s) {
  if (ls < 1 || ls > kMaxLimbs || blocks == 0) return (int)hipErrorInvalidValue;
  QWords qw;
  memset(&qw, 0, sizeof(qw));
  for (int j = 0; j < ls; j++) qw.w[j] = q[j];
  hipLaunchKernelGGL(count_noncanonical_kernel, dim3(blocks), dim3(256), 0, s, d_x, n, ls, qw, d_partial);
  return (int)hipGetLastError();
}

// Layout conversion between element-major words (element i's limb j at
// i * L + j, the usual array of little-endian multi-word integers) and the
// library's limb-planar layout (j * n + i).  A workgroup moves 256 elements
// through LDS so that both the global reads and the global writes are
// consecutive words; the LDS row stride is odd, so the column-wise LDS
// accesses of one wavefront fall in distinct banks.
__global__ __launch_bounds__(256) void layout_kernel(const u32* __restrict__ src, u32* __restrict__ dst, u64 n,
                                                     u32 L, int to_planar) {
  extern __shared__ u32 tile[];
  const u32 S = L | 1u;
  const u64 base = (u64)blockIdx.x * 256;
  const u32 cnt = (u32)((n - base) < 256 ? (n - base) : 256);
  const u32 tid = threadIdx.x;
  if (to_planar) {
    for (u32 k = tid; k < cnt * L; k += 256) tile[(k / L) * S + (k % L)] = src[base * L + k];
    __syncthreads();
    if (tid < cnt)
      for (u32 j = 0; j < L; j++) dst[(u64)j * n + base + tid] = tile[tid * S + j];
  } else {
    if (tid < cnt)
      for (u32 j = 0; j < L; j++) tile[tid * S + j] = src[(u64)j * n + base + tid];
    __syncthreads();
    for (u32 k = tid; k < cnt * L; k += 256) dst[base * L + k] = tile[(k / L) * S + (k % L)];
  }
}

int launch_layout(const uint32_t* src, uint32_t* dst, uint64_t n, uint32_t L, bool to_planar, hipStream_t s) {
  if (n == 0) return 0;
  if (L < 1 || L > (uint32_t)kMaxLimbs) return (int)hipErrorInvalidValue;
  const u64 blocks = (n + 255) / 256;
  const size_t lds = (size_t)256 * (L | 1u) * sizeof(u32);
  hipLaunchKernelGGL(layout_kernel, dim3((unsigned)blocks), dim3(256), lds, s, src, dst, n, L, to_planar ? 1 : 0);
  return (int)hipGetLastError();
}

}  // namespace moma
