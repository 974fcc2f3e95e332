// batch.cpp - many transforms of mixed sizes, limb counts and moduli in one
// hipGraph launch (the paper runs batches of kernels to fill the GPU and
// reports steady-state time per transform, Section 5.1).
//
// Every job is split into the passes of its own plan.  Pass p of every job
// forms phase p (a cyclic product runs its two forward transforms in phases
// 0 .. P-1 and its inverse in phases P .. 2P-1); within a phase, jobs are
// grouped by compute limb count (the
// kernels are compiled per limb count) and by their plans' register radix and
// workgroup size, and each group becomes one launch of
// ntt_batch_kernel over a flat list of (pass record, tile) items, sorted by
// decreasing work, one workgroup per item (the dispatcher starts the largest
// tiles first).  Phases follow one
// another in stream order, which is the only dependency between a job's
// passes.  Jobs whose data is 16 MiB or more run in groups instead: the jobs
// of a group share phases, and each group's phases follow the previous
// group's, so that the passes of a group of one limb count revisit at most
// 256 MiB of data (one job if it is larger).  The launches are captured once
// into a graph; running the batch is one hipGraphLaunch.  The launches of
// different compute limb counts are captured on different streams (a job's
// passes all have its limb count), so they are independent chains of the
// graph, and groups of different limb counts may run side by side.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "../../include/moma.h"
#include "common.hpp"
#include "plan.hpp"

namespace moma {

struct BatchLaunch {
  int L;
  bool mul, variant, fw;
  uint32_t phase, radix_log, threads, grid, nitems;
  size_t lds;
  const NttPassArgs* d_passes;
  const void* d_consts;
  const uint2* d_items;
};

struct ZeroFill {
  uint32_t* out;
  uint64_t n;
  int from, to;
};

struct BlasLaunch {
  int op, L;
  bool fw;
  uint32_t variant, nitems;
  const void* d_recs;
  const void* d_consts;
  const uint2* d_items;
};

struct BatchImpl {
  std::vector<std::shared_ptr<NttPlan>> plans;  // keep tables alive
  std::vector<void*> dev_allocs;
  std::vector<BatchLaunch> launches;
  std::vector<BlasLaunch> blas;
  std::vector<ZeroFill> fills;
  // every job's inputs, counted before a run when the input check is on
  struct Input {
    std::shared_ptr<FieldEntry> fe;
    const uint32_t* x;
    uint64_t n;
    uint32_t job;
  };
  std::vector<Input> inputs;
  uint64_t items = 0;
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> side;  // further capture streams: launches of one phase run side by side
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~BatchImpl() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (hipStream_t st : side) (void)hipStreamDestroy(st);
    if (cap) (void)hipStreamDestroy(cap);
    for (void* p : dev_allocs) (void)hipFree(p);
  }
};

static int dev_upload(BatchImpl& b, const void* host, size_t bytes, void** out) {
  void* d = nullptr;
  if (hipMalloc(&d, bytes ? bytes : 4)) return set_error(MOMA_E_NOMEM, "batch table allocation failed");
  b.dev_allocs.push_back(d);
  if (bytes && hipMemcpy(d, host, bytes, hipMemcpyHostToDevice)) return hip_fail(1, "batch table upload");
  *out = d;
  return MOMA_OK;
}

static int batch_create(const moma_ntt_job_t* jobs, uint32_t njobs, BatchImpl& b) {
  if (!jobs && njobs) return set_error(MOMA_E_ARG, "jobs is NULL");
  // per limb count: pass records, their constants, and per-phase items
  struct Group {
    std::vector<NttPassArgs> recs;
    std::vector<uint8_t> consts;
    std::map<uint32_t, std::vector<std::pair<uint64_t, uint2>>> items;  // phase -> (cost, item)
    std::map<uint32_t, size_t> lds;                                     // phase -> max tile bytes
  };
  // key: (compute limbs, register radix, threads) of the job's schedule,
  // whether the pass multiplies two inputs (first inverse pass of a cyclic
  // product: a kernel variant of its own), and the tile's LDS bytes (a launch
  // reserves its largest tile for every workgroup, so mixing sizes would cut
  // the occupancy of the smaller tiles), and whether the pass runs the kernel
  // variant with the direct first round and the cross-lane last stage, and
  // whether the modulus is full width (kernels of their own)
  typedef std::tuple<int, uint32_t, uint32_t, bool, size_t, bool, bool> GKey;
  std::map<GKey, Group> groups;
  NttConsts none;
  memset(&none, 0, sizeof(none));
  // one transform of a job: its passes go to phases phase0, phase0 + 1, ...
  auto add = [&](NttPlan& p, const NttSchedule& sched, const std::vector<NttPass>& passes, const DirTables& t,
                 const NttConsts& nc, bool scale, const uint32_t* in, const uint32_t* in2, uint32_t* first_out,
                 uint32_t* out, uint32_t phase0) {
    const FieldRaw& f = p.fe->f;
    size_t cb = ntt_consts_bytes(f.L, f.fw != 0);
    for (size_t i = 0; i < passes.size(); i++) {
      const NttPass& ps = passes[i];
      const size_t tile_bytes = ((size_t)1 << (ps.k + ps.logc)) * f.L * sizeof(uint32_t);
      NttPassArgs a{};
      a.in = (i == 0) ? in : (i == 1 ? first_out : out);
      a.in2 = (i == 0) ? in2 : nullptr;
      a.out = (i == 0) ? first_out : out;
      a.tw = t.tw;
      a.n = p.n;
      a.logn = p.logn;
      a.K = ps.K;
      a.k = ps.k;
      a.logc = ps.logc;
      a.last = (i + 1 == passes.size()) ? 1u : 0u;
      a.scale = (scale && i + 1 == passes.size()) ? 1u : 0u;
      const bool variant = !f.fw && ntt_batch_variant(f.L, sched.radix_log, sched.threads, &a);
      Group& g = groups[GKey(f.L, sched.radix_log, sched.threads, i == 0 && in2 != nullptr, tile_bytes, variant,
                             f.fw != 0)];
      uint32_t rec = (uint32_t)g.recs.size();
      g.recs.push_back(a);
      size_t off = g.consts.size();
      g.consts.resize(off + cb);
      ntt_fill_consts(f, p.fe->dc, &nc, g.consts.data() + off);
      uint64_t E = 1ull << (ps.k + ps.logc);
      uint64_t cost = E * ps.k;
      uint32_t ph = phase0 + (uint32_t)i;
      auto& v = g.items[ph];
      for (uint64_t tl = 0; tl < ps.tiles; tl++) v.push_back({cost, make_uint2(rec, (uint32_t)tl)});
      size_t bytes = (size_t)E * f.L * sizeof(uint32_t);
      g.lds[ph] = std::max(g.lds[ph], bytes);
    }
  };
  // BLAS jobs: per (op, compute limbs, vmul variant, full width) the job
  // records, their constants and the (record, 256-element block) items
  struct BGroup {
    std::vector<BlasJobRec> recs;
    std::vector<uint8_t> consts;
    std::vector<uint2> items;
  };
  std::map<std::tuple<int, int, uint32_t, bool>, BGroup> bgroups;
  // groups of large jobs: the phases [group_phase, group_phase + group_span)
  constexpr uint64_t kGroupMinJobBytes = 16ull << 20, kGroupBytes = 256ull << 20;
  uint32_t group_phase = 0, group_span = 0;
  uint64_t group_bytes = 0;
  for (uint32_t j = 0; j < njobs; j++) {
    const moma_ntt_job_t& job = jobs[j];
    const std::string tag = "job " + std::to_string(j) + ": ";
    if (job.kind > MOMA_JOB_AXPY) return set_error(MOMA_E_ARG, tag + "unknown job kind");
    if (job.kind >= MOMA_JOB_VADD) {
      const int op = (int)job.kind - (int)MOMA_JOB_VADD;  // OP_VADD .. OP_AXPY
      std::shared_ptr<FieldEntry> fe;
      int rc = build_field(job.q, job.limbs, &fe);
      if (rc) return set_error(rc, tag + g_detail);
      if (job.n > (1ull << 31)) return set_error(MOMA_E_ARG, tag + "n must be <= 2^31");
      if (job.n == 0) continue;
      if (!job.d_in || !job.d_in2 || !job.d_out) return set_error(MOMA_E_ARG, tag + "NULL buffer");
      BlasArgs a;
      memset(&a, 0, sizeof(a));
      a.a = job.d_in;
      a.b = job.d_in2;
      a.out = job.d_out;
      a.n = job.n;
      a.ls = (uint32_t)fe->f.Ls;
      if (op == OP_VMUL && !fe->f.fw) a.variant = vmul_variant(fe->f.L);
      if (op == OP_AXPY) {
        rc = axpy_alpha(*fe, job.alpha, job.limbs, a.alpha_m);
        if (rc) return set_error(rc, tag + g_detail);
      }
      BGroup& g = bgroups[std::make_tuple(op, fe->f.L, a.variant, fe->f.fw != 0)];
      const uint32_t rec = (uint32_t)g.recs.size();
      g.recs.push_back({job.d_in, job.d_in2, job.d_out, job.n});
      size_t cb = blas_consts_bytes(fe->f.L), off = g.consts.size();
      g.consts.resize(off + cb);
      blas_fill_consts(fe->f, a, g.consts.data() + off);
      const uint64_t blocks = (job.n + 255) / 256;
      if (g.items.size() + blocks > 0x7fffffffull) return set_error(MOMA_E_UNSUPPORTED, tag + "too many blocks");
      for (uint64_t k = 0; k < blocks; k++) g.items.push_back(make_uint2(rec, (uint32_t)k));
      if (fe->f.Ls > fe->f.L && job.d_out != job.d_in && job.d_out != job.d_in2)
        b.fills.push_back({job.d_out, job.n, fe->f.L, fe->f.Ls});
      b.inputs.push_back({fe, job.d_in, job.n, j});
      b.inputs.push_back({fe, job.d_in2, job.n, j});
      continue;
    }
    if (!job.d_in || !job.d_out) return set_error(MOMA_E_ARG, tag + "NULL buffer");
    if (job.kind == MOMA_JOB_CYCLIC_MUL && !job.d_in2) return set_error(MOMA_E_ARG, tag + "NULL second input");
    std::shared_ptr<NttPlan> p;
    int rc = get_plan(job.q, job.omega, job.n, job.limbs, &p);
    if (rc) return set_error(rc, tag + g_detail);
    b.plans.push_back(p);
    b.inputs.push_back({p->fe, job.d_in, job.n, j});
    if (job.kind == MOMA_JOB_CYCLIC_MUL) b.inputs.push_back({p->fe, job.d_in2, job.n, j});
    const FieldRaw& f = p->fe->f;
    std::vector<NttPass> passes;
    NttSchedule sched;
    {
      std::lock_guard<std::mutex> lk(p->mu);
      passes = p->passes;
      sched = p->sched;
    }
    // the batch kernels run the schoolbook butterfly
    sched.kara = 0;
    // A plan's own schedule is chosen for a lone call, where small transforms
    // want small tiles to spread over the chip.  In a batch the other jobs
    // fill the chip, so jobs up to 2^18 points take large tiles (fewer passes
    // and workgroups); larger jobs keep their schedule, which measured faster
    // for them (2^24 points, and 1024-bit moduli at 2^20).
    if (p->n <= (1ull << 18)) {
      NttSchedule ds = batch_schedule(f.L, p->logn);
      std::vector<NttPass> dp;
      std::string keep = g_detail;
      if (plan_passes(f.L, p->logn, ds, &dp, f.fw) == MOMA_OK) {
        sched = ds;
        passes = dp;
      }
      g_detail = keep;
    }
    const size_t plane_words = (size_t)p->n * f.L;
    uint32_t ph0 = 0;
    {
      const uint32_t copies = job.kind == MOMA_JOB_CYCLIC_MUL ? 2u : 1u;
      const uint64_t bytes = (uint64_t)plane_words * sizeof(uint32_t) * copies;
      if (bytes >= kGroupMinJobBytes) {
        if (group_bytes > 0 && group_bytes + bytes > kGroupBytes) {
          group_phase += group_span;
          group_span = 0;
          group_bytes = 0;
        }
        ph0 = group_phase;
        group_bytes += bytes;
        group_span = std::max(group_span, (uint32_t)passes.size() * copies);
      }
    }
    auto alloc = [&](size_t words, uint32_t** outp) -> int {
      void* s = nullptr;
      if (hipMalloc(&s, words * sizeof(uint32_t))) return set_error(MOMA_E_NOMEM, tag + "job buffers");
      b.dev_allocs.push_back(s);
      *outp = (uint32_t*)s;
      return MOMA_OK;
    };
    if (job.kind == MOMA_JOB_CYCLIC_MUL) {
      uint32_t* sa = nullptr;
      int r = alloc(2 * plane_words, &sa);
      if (r) return r;
      uint32_t* sb = sa + plane_words;
      add(*p, sched, passes, p->fwd, none, false, job.d_in, nullptr, sa, sa, ph0);
      add(*p, sched, passes, p->fwd, none, false, job.d_in2, nullptr, sb, sb, ph0);
      add(*p, sched, passes, p->inv, p->mul_consts, true, sa, sb, job.d_out, job.d_out,
          ph0 + (uint32_t)passes.size());
      if (f.Ls > f.L) b.fills.push_back({job.d_out, p->n, f.L, f.Ls});
      continue;
    }
    const bool inverse = job.kind == MOMA_JOB_INVERSE;
    uint32_t* first_out = job.d_out;
    if (passes.size() > 1 && job.d_in == job.d_out) {
      int r = alloc(plane_words, &first_out);
      if (r) return r;
    }
    add(*p, sched, passes, inverse ? p->inv : p->fwd, inverse ? p->inv_consts : none, inverse, job.d_in, nullptr,
        first_out, job.d_out, ph0);
    if (f.Ls > f.L && job.d_out != job.d_in) b.fills.push_back({job.d_out, p->n, f.L, f.Ls});
  }
  // upload tables and build the launch list, phase by phase
  uint32_t max_phase = 0;
  for (auto& kv : groups)
    for (auto& it : kv.second.items) max_phase = std::max(max_phase, it.first + 1);
  std::map<GKey, std::pair<void*, void*>> dev_recs;
  for (auto& kv : groups) {
    void *dp = nullptr, *dc = nullptr;
    int rc = dev_upload(b, kv.second.recs.data(), kv.second.recs.size() * sizeof(NttPassArgs), &dp);
    if (rc) return rc;
    rc = dev_upload(b, kv.second.consts.data(), kv.second.consts.size(), &dc);
    if (rc) return rc;
    dev_recs[kv.first] = {dp, dc};
  }
  for (uint32_t ph = 0; ph < max_phase; ph++) {
    for (auto& kv : groups) {
      int L = std::get<0>(kv.first);
      auto it = kv.second.items.find(ph);
      if (it == kv.second.items.end() || it->second.empty()) continue;
      auto& v = it->second;
      std::stable_sort(v.begin(), v.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
      std::vector<uint2> items(v.size());
      for (size_t i = 0; i < v.size(); i++) items[i] = v[i].second;
      void* di = nullptr;
      int rc = dev_upload(b, items.data(), items.size() * sizeof(uint2), &di);
      if (rc) return rc;
      BatchLaunch bl;
      bl.L = L;
      bl.phase = ph;
      bl.mul = std::get<3>(kv.first);
      bl.variant = std::get<5>(kv.first);
      bl.fw = std::get<6>(kv.first);
      bl.radix_log = std::get<1>(kv.first);
      bl.threads = std::get<2>(kv.first);
      bl.lds = kv.second.lds[ph];
      bl.nitems = (uint32_t)items.size();
      if (items.size() > 0x7fffffffull) return set_error(MOMA_E_UNSUPPORTED, "batch phase has too many tiles");
      bl.grid = bl.nitems;  // one workgroup per item
      bl.d_passes = (const NttPassArgs*)dev_recs[kv.first].first;
      bl.d_consts = dev_recs[kv.first].second;
      bl.d_items = (const uint2*)di;
      b.launches.push_back(bl);
      b.items += bl.nitems;
    }
  }
  for (auto& kv : bgroups) {
    BGroup& g = kv.second;
    BlasLaunch bl;
    bl.op = std::get<0>(kv.first);
    bl.L = std::get<1>(kv.first);
    bl.variant = std::get<2>(kv.first);
    bl.fw = std::get<3>(kv.first);
    bl.nitems = (uint32_t)g.items.size();
    void *dr = nullptr, *dc = nullptr, *di = nullptr;
    int rc = dev_upload(b, g.recs.data(), g.recs.size() * sizeof(BlasJobRec), &dr);
    if (!rc) rc = dev_upload(b, g.consts.data(), g.consts.size(), &dc);
    if (!rc) rc = dev_upload(b, g.items.data(), g.items.size() * sizeof(uint2), &di);
    if (rc) return rc;
    bl.d_recs = dr;
    bl.d_consts = dc;
    bl.d_items = (const uint2*)di;
    b.blas.push_back(bl);
    b.items += bl.nitems;
  }
  for (const BatchLaunch& bl : b.launches) ntt_batch_prepare(bl.L, bl.radix_log, bl.fw, bl.lds);
  // Capture the launches into one graph.  All passes of a job have the job's
  // compute limb count, so each limb count gets one of up to kStreams streams
  // forked from the capture stream: launch order within a stream keeps every
  // job's passes in phase order, and the chains of different limb counts are
  // independent nodes of the graph that run side by side.  The streams join
  // before the zero fills.
  constexpr size_t kStreams = 4;
  if (hipStreamCreate(&b.cap)) return hip_fail(1, "batch stream");
  std::map<int, size_t> slot_of;  // compute limbs -> stream slot (0: the capture stream)
  for (const BatchLaunch& bl : b.launches)
    if (!slot_of.count(bl.L)) {
      const size_t slot = slot_of.size() % kStreams;
      slot_of[bl.L] = slot;
    }
  for (size_t k = 1; k < std::min(slot_of.size(), kStreams); k++) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) return hip_fail(1, "batch stream");
    b.side.push_back(st);
  }
  auto record = [&](hipStream_t st) -> hipEvent_t {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming)) return nullptr;
    b.events.push_back(e);
    return hipEventRecord(e, st) ? nullptr : e;
  };
  if (hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal)) return hip_fail(1, "begin capture");
  int err = 0;
  for (const BlasLaunch& bl : b.blas) {
    err = launch_blas_batch(bl.op, bl.L, bl.variant, bl.fw, bl.d_recs, bl.d_consts, bl.d_items, bl.nitems, b.cap);
    if (err) break;
  }
  if (!err && !b.side.empty()) {
    hipEvent_t fork = record(b.cap);
    if (!fork) err = 1;
    for (size_t k = 0; !err && k < b.side.size(); k++)
      if (hipStreamWaitEvent(b.side[k], fork, 0)) err = 1;
  }
  for (size_t k = 0; !err && k < b.launches.size(); k++) {
    const BatchLaunch& bl = b.launches[k];
    const size_t slot = slot_of[bl.L];
    err = launch_ntt_batch(bl.L, bl.radix_log, bl.mul, bl.variant, bl.fw, bl.threads, bl.lds, bl.grid, bl.d_passes,
                           bl.d_consts, bl.d_items, bl.nitems, slot ? b.side[slot - 1] : b.cap);
  }
  for (size_t k = 0; !err && k < b.side.size(); k++) {
    hipEvent_t join = record(b.side[k]);
    if (!join || hipStreamWaitEvent(b.cap, join, 0)) err = 1;
  }
  if (!err)
    for (const ZeroFill& z : b.fills) {
      err = launch_zero_planes(z.out, z.n, z.from, z.to, b.cap);
      if (err) break;
    }
  hipError_t ec = hipStreamEndCapture(b.cap, &b.graph);
  if (err) return hip_fail(err, "batch launch capture");
  if (ec) return hip_fail((int)ec, "end capture");
  if (hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0)) return hip_fail(1, "graph instantiate");
  return MOMA_OK;
}

}  // namespace moma

using namespace moma;

struct moma_batch {
  BatchImpl impl;
};

extern "C" {

int moma_batch_create(const moma_ntt_job_t* jobs, uint32_t njobs, moma_batch_t* out) {
  if (!out) return set_error(MOMA_E_ARG, "out is NULL");
  *out = nullptr;
  auto* b = new moma_batch();
  int rc = batch_create(jobs, njobs, b->impl);
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return MOMA_OK;
}

int moma_batch_run(moma_batch_t b, void* stream) {
  if (!b) return set_error(MOMA_E_ARG, "batch is NULL");
  if (input_check_on()) {
    for (const auto& in : b->impl.inputs) {
      int rc = check_inputs(in.fe->f, &in.x, 1, in.n, (hipStream_t)stream);
      if (rc) return set_error(rc, "job " + std::to_string(in.job) + ": " + g_detail);
    }
  }
  hipError_t e = hipGraphLaunch(b->impl.exec, (hipStream_t)stream);
  if (e) return hip_fail((int)e, "graph launch");
  return MOMA_OK;
}

int moma_batch_info(moma_batch_t b, uint32_t* launches, uint64_t* items) {
  if (!b) return set_error(MOMA_E_ARG, "batch is NULL");
  if (launches)
    *launches = (uint32_t)(b->impl.launches.size() + b->impl.blas.size() + b->impl.fills.size());
  if (items) *items = b->impl.items;
  return MOMA_OK;
}

int moma_batch_destroy(moma_batch_t b) {
  delete b;
  return MOMA_OK;
}

}  // extern "C"
