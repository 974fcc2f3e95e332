// plan.hpp - host runtime internals shared by the C ABI, the batch executor and
// the autotuner: per-modulus constants, transform plans and their schedules.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "hostbig.hpp"

namespace moma {

struct FieldEntry {
  FieldRaw f;
  DigitConsts dc;
  HBig Q, one_m;
  HBig adj;  // 2^(bD) mod q: R of the digit form
  // last axpy scalar, cached with its Montgomery form
  std::vector<uint32_t> alpha_key;
  std::vector<uint32_t> alpha_m;
};

struct DirTables {
  uint32_t* tw = nullptr;      // n entries x digit_stride(L) words, digit Montgomery form
  uint32_t* ladder = nullptr;  // (logn + 2) x L words: w^(2^b) in Montgomery form, then 1, then 2^(bD) mod q
};

struct NttPlan {
  std::shared_ptr<FieldEntry> fe;
  int device = 0;
  uint64_t n = 0;
  uint32_t logn = 0;
  DirTables fwd, inv;
  NttConsts inv_consts;
  NttConsts mul_consts;           // inverse after a fused pointwise product
  uint32_t* scratch = nullptr;    // for in-place multi-pass calls
  uint32_t* spectra = nullptr;    // 2 x n x L words: the two forward transforms of a cyclic product
  NttSchedule sched;
  std::vector<NttPass> passes;
  std::mutex mu;  // guards scratch allocation and schedule changes
  ~NttPlan() {
    (void)hipFree(fwd.tw);
    (void)hipFree(fwd.ladder);
    (void)hipFree(inv.tw);
    (void)hipFree(inv.ladder);
    (void)hipFree(scratch);
    (void)hipFree(spectra);
  }
};

extern std::mutex g_mu;              // guards the field and plan caches
extern thread_local std::string g_detail;

int hip_fail(int e, const char* what);
int build_field(const uint32_t* q, uint32_t limbs, std::shared_ptr<FieldEntry>* out);
int get_plan(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, std::shared_ptr<NttPlan>* out);
// fw: a full-width modulus, whose kernels have radix-2 and radix-4 units only
uint32_t max_radix_log(int L, bool fw = false);
int plan_passes(int L, uint32_t logn, const NttSchedule& s, std::vector<NttPass>* out, bool fw = false);
NttSchedule default_schedule(int L, uint32_t logn);
NttSchedule batch_schedule(int L, uint32_t logn);
int run_plan(NttPlan& p, bool inverse, const uint32_t* d_in, uint32_t* d_out, hipStream_t s);
// ext: NULL, or caller-provided device scratch of cyclic_mul_scratch_words(p)
// words used in place of the plan's spectra buffer, so the call
// allocates nothing
int run_cyclic_mul(NttPlan& p, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_out, hipStream_t s,
                   uint32_t* ext = nullptr);
uint64_t cyclic_mul_scratch_words(const NttPlan& p);
// the cached plan for these arguments, or MOMA_E_ARG when none has been built
// (allocates no device memory)
int find_plan(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, std::shared_ptr<NttPlan>* out);
// batched BLAS (blas.hip): one record per job, its constants, and items
// (record, block of 256 elements)
struct BlasJobRec {
  const uint32_t* a;
  const uint32_t* b;
  uint32_t* out;
  uint64_t n;
};
size_t blas_consts_bytes(int L);
void blas_fill_consts(const FieldRaw& f, const BlasArgs& a, void* dst);
int launch_blas_batch(int op, int L, uint32_t variant, bool fw, const void* recs, const void* consts,
                      const uint2* items, uint32_t nitems, hipStream_t s);
// vmul's product variant for a compute limb count (capi.cpp)
uint32_t vmul_variant(int L);
// alpha (storage limbs words) in Montgomery form for axpy, validated < q
int axpy_alpha(FieldEntry& fe, const uint32_t* alpha, uint32_t limbs, uint32_t* alpha_m);
// n pseudo-random residues below q in Ls = f.Ls storage planes (timing inputs for the tuners)
int fill_random_residues(const FieldRaw& f, uint32_t* d, uint64_t n, uint32_t seed, hipStream_t s);
int launch_fill_residues(uint32_t* p, uint64_t n, int planes, int top, uint32_t top_mask, uint32_t seed, hipStream_t s);
// per-workgroup counts of the elements >= q over `ls` storage planes
int launch_count_noncanonical(const uint32_t* q, int ls, const uint32_t* d_x, uint64_t n, uint32_t* d_partial,
                              uint32_t blocks, hipStream_t s);
// element-major <-> limb-planar words (to_planar: src is element-major)
int launch_layout(const uint32_t* src, uint32_t* dst, uint64_t n, uint32_t L, bool to_planar, hipStream_t s);
// the input check of every entry point (MOMA_CHECK_INPUTS / moma_set_input_check)
bool input_check_on();
// d_part: NULL (a buffer is allocated for the call) or at least 1024 device words
int count_noncanonical(const FieldRaw& f, const uint32_t* d_x, uint64_t n, hipStream_t s, uint64_t* bad,
                       uint32_t* d_part = nullptr);
int check_inputs(const FieldRaw& f, const uint32_t* const* d_x, int nx, uint64_t n, hipStream_t s,
                 uint32_t* d_part = nullptr);
// tuner (tune.cpp)
std::vector<NttSchedule> enumerate_schedules(int L, uint32_t logn, bool fw = false);
bool tune_db_best(const std::string& dev, int L, uint32_t logn, NttSchedule* out);
std::string current_device_name();
// cost model (costmodel.cpp): predicted log-time per schedule; MOMA_E_UNSUPPORTED without a model
int costmodel_scores(int L, uint32_t logn, const std::vector<NttSchedule>& cands, std::vector<float>* scores);
// the loaded model's fastest predicted schedule for (L, log2 n), cached per
// shape until the model changes; false when no model is loaded
bool costmodel_pick(int L, uint32_t logn, NttSchedule* out);
// a new plan's schedule: the timing database's best, else the cost model's
// pick, else the fixed rule of default_schedule
NttSchedule initial_schedule(int L, uint32_t logn, bool fw = false);

}  // namespace moma
