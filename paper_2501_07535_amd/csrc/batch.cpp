// batch.cpp - many transforms of mixed sizes, limb counts and moduli in one
// hipGraph launch (the paper runs batches of kernels to fill the GPU and
// reports steady-state time per transform, Section 5.1).
//
// Every job is split into the passes of its own plan.  Pass p of every job
// forms phase p; within a phase, jobs are grouped by compute limb count (the
// kernels are compiled per limb count) and each group becomes one launch of
// ntt_batch_kernel over a flat list of (pass record, tile) items, sorted by
// decreasing work and dealt round-robin to a fixed grid.  Phases follow one
// another in stream order, which is the only dependency between a job's
// passes.  The launches are captured once into a graph; running the batch is
// one hipGraphLaunch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <vector>

#include "../../include/moma.h"
#include "common.hpp"
#include "plan.hpp"

namespace moma {

struct BatchLaunch {
  int L;
  uint32_t radix_log, threads, grid, nitems;
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

struct BatchImpl {
  std::vector<std::shared_ptr<NttPlan>> plans;  // keep tables alive
  std::vector<void*> dev_allocs;
  std::vector<BatchLaunch> launches;
  std::vector<ZeroFill> fills;
  uint64_t items = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~BatchImpl() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
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
  std::map<int, Group> groups;
  for (uint32_t j = 0; j < njobs; j++) {
    const moma_ntt_job_t& job = jobs[j];
    if (!job.d_in || !job.d_out) return set_error(MOMA_E_ARG, "job " + std::to_string(j) + ": NULL buffer");
    if (job.inverse > 1) return set_error(MOMA_E_ARG, "job " + std::to_string(j) + ": inverse must be 0 or 1");
    std::shared_ptr<NttPlan> p;
    int rc = get_plan(job.q, job.omega, job.n, job.limbs, &p);
    if (rc) return set_error(rc, "job " + std::to_string(j) + ": " + g_detail);
    b.plans.push_back(p);
    const FieldRaw& f = p->fe->f;
    std::vector<NttPass> passes;
    {
      std::lock_guard<std::mutex> lk(p->mu);
      passes = p->passes;
    }
    uint32_t* first_out = job.d_out;
    if (passes.size() > 1 && job.d_in == job.d_out) {
      void* s = nullptr;
      if (hipMalloc(&s, (size_t)p->n * f.L * sizeof(uint32_t))) return set_error(MOMA_E_NOMEM, "job scratch");
      b.dev_allocs.push_back(s);
      first_out = (uint32_t*)s;
    }
    Group& g = groups[f.L];
    size_t cb = ntt_consts_bytes(f.L);
    NttConsts none;
    memset(&none, 0, sizeof(none));
    for (size_t i = 0; i < passes.size(); i++) {
      const NttPass& ps = passes[i];
      NttPassArgs a;
      a.in = (i == 0) ? job.d_in : (i == 1 ? first_out : job.d_out);
      a.out = (i == 0) ? first_out : job.d_out;
      a.tw = job.inverse ? p->inv.tw : p->fwd.tw;
      a.n = p->n;
      a.logn = p->logn;
      a.K = ps.K;
      a.k = ps.k;
      a.logc = ps.logc;
      a.last = (i + 1 == passes.size()) ? 1u : 0u;
      a.scale = (job.inverse && i + 1 == passes.size()) ? 1u : 0u;
      uint32_t rec = (uint32_t)g.recs.size();
      g.recs.push_back(a);
      size_t off = g.consts.size();
      g.consts.resize(off + cb);
      ntt_fill_consts(f, p->fe->dc, job.inverse ? &p->inv_consts : &none, g.consts.data() + off);
      uint64_t E = 1ull << (ps.k + ps.logc);
      uint64_t cost = E * ps.k;
      auto& v = g.items[(uint32_t)i];
      for (uint64_t t = 0; t < ps.tiles; t++) v.push_back({cost, make_uint2(rec, (uint32_t)t)});
      size_t bytes = (size_t)E * f.L * sizeof(uint32_t);
      g.lds[(uint32_t)i] = std::max(g.lds[(uint32_t)i], bytes);
    }
    if (f.Ls > f.L && job.d_out != job.d_in) b.fills.push_back({job.d_out, p->n, f.L, f.Ls});
  }
  // upload tables and build the launch list, phase by phase
  uint32_t max_phase = 0;
  for (auto& kv : groups)
    for (auto& it : kv.second.items) max_phase = std::max(max_phase, it.first + 1);
  std::map<int, std::pair<void*, void*>> dev_recs;
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
      int L = kv.first;
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
      bl.radix_log = std::min(2u, max_radix_log(L));
      bl.threads = std::min(256u, ntt_max_threads(L, bl.radix_log));
      bl.lds = kv.second.lds[ph];
      bl.nitems = (uint32_t)items.size();
      bl.grid = std::min<uint32_t>(bl.nitems, 4096);
      bl.d_passes = (const NttPassArgs*)dev_recs[L].first;
      bl.d_consts = dev_recs[L].second;
      bl.d_items = (const uint2*)di;
      b.launches.push_back(bl);
      b.items += bl.nitems;
    }
  }
  for (const BatchLaunch& bl : b.launches) ntt_batch_prepare(bl.L, bl.radix_log, bl.lds);
  // capture the launches into one graph
  if (hipStreamCreate(&b.cap)) return hip_fail(1, "batch stream");
  if (hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal)) return hip_fail(1, "begin capture");
  int err = 0;
  for (const BatchLaunch& bl : b.launches) {
    err = launch_ntt_batch(bl.L, bl.radix_log, bl.threads, bl.lds, bl.grid, bl.d_passes, bl.d_consts, bl.d_items,
                           bl.nitems, b.cap);
    if (err) break;
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
  hipError_t e = hipGraphLaunch(b->impl.exec, (hipStream_t)stream);
  if (e) return hip_fail((int)e, "graph launch");
  return MOMA_OK;
}

int moma_batch_info(moma_batch_t b, uint32_t* launches, uint64_t* items) {
  if (!b) return set_error(MOMA_E_ARG, "batch is NULL");
  if (launches) *launches = (uint32_t)(b->impl.launches.size() + b->impl.fills.size());
  if (items) *items = b->impl.items;
  return MOMA_OK;
}

int moma_batch_destroy(moma_batch_t b) {
  delete b;
  return MOMA_OK;
}

}  // extern "C"
