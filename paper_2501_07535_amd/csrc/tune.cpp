// tune.cpp - schedule autotuner and its timing database.
//
// A transform plan can run under many launch shapes (moma_ntt_schedule_t); all
// compute the same result and differ only in speed.  The tuner enumerates the
// feasible shapes for one (n, limbs), times each with HIP events (warm-up, then
// the median of several repetitions, each long enough to dwarf event
// resolution), installs the fastest in the plan and appends every measurement
// to an in-process database.  The database can be saved and loaded as CSV;
// plans created afterwards on the same device start from the best recorded
// shape for their (limbs, log2 n).  When a learned cost model is loaded
// (costmodel.cpp) and top_k > 0, only the model's top_k shapes are timed.
// Ties go to the candidate that comes first in enumeration order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/moma.h"
#include "common.hpp"
#include "plan.hpp"

namespace moma {

struct TuneRow {
  std::string device;
  uint32_t L, logn, tile_log, col_log, threads, radix_log;
  float us;
  uint32_t reps;
  uint32_t kara = 0;  // the butterfly's word products by Karatsuba (Eq. (mulk))
};

static std::mutex g_tune_mu;
static std::vector<TuneRow> g_rows;

static std::string device_name() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string s = p.gcnArchName;
  size_t c = s.find(':');
  if (c != std::string::npos) s = s.substr(0, c);
  return s + "/" + std::to_string(p.multiProcessorCount) + "cu";
}

// every shape the pass kernels can run, in a fixed order: the schoolbook
// butterflies first, then the radix-2 shapes again with the Karatsuba form of
// the twiddle multiply (2 to 24 limbs; not for full-width moduli)
std::vector<NttSchedule> enumerate_schedules(int L, uint32_t logn, bool fw) {
  std::vector<NttSchedule> out;
  std::string keep = g_detail;
  for (uint32_t tl = 5; tl <= 14; tl++) {
    bool single = logn <= tl;
    for (uint32_t cl : {2u, 3u, 4u, 5u}) {
      if (single && cl != 2) continue;  // the column count does not apply to one-pass plans
      for (uint32_t r = 1; r <= max_radix_log(L, fw); r++) {
        for (uint32_t t : {64u, 128u, 256u, 512u, 1024u}) {
          NttSchedule s{single ? logn : tl, single ? 0u : cl, t, r};
          std::vector<NttPass> ps;
          if (plan_passes(L, logn, s, &ps, fw) != MOMA_OK) continue;
          // more threads than units per round would idle whole waves
          uint32_t e = single ? logn : tl;
          uint32_t units = 1u << (e > r ? e - r : 0);
          if (t > 64 && t > units) continue;
          // a radix-16 unit on passes of fewer than 4 stages runs as radix 8
          if (r == 4 && std::max_element(ps.begin(), ps.end(), [](const NttPass& x, const NttPass& y) {
                          return x.k < y.k;
                        })->k < 4)
            continue;
          bool dup = false;
          for (const NttSchedule& o : out)
            dup |= o.tile_log == s.tile_log && o.col_log == s.col_log && o.threads == s.threads &&
                   o.radix_log == s.radix_log;
          if (!dup) out.push_back(s);
        }
      }
    }
  }
  if (!fw && L >= 2 && L <= kMaxLimbsKara) {
    const size_t nschool = out.size();
    for (size_t i = 0; i < nschool; i++)
      if (out[i].radix_log == 1) {
        NttSchedule s = out[i];
        s.kara = 1;
        out.push_back(s);
      }
  }
  g_detail = keep;
  return out;
}

// the best recorded schedule for (device, L, logn), if any
bool tune_db_best(const std::string& dev, int L, uint32_t logn, NttSchedule* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  // keep the latest measurement of each shape, then take the fastest
  std::map<std::tuple<uint32_t, uint32_t, uint32_t, uint32_t, uint32_t>, float> last;
  for (const TuneRow& r : g_rows)
    if (r.device == dev && (int)r.L == L && r.logn == logn)
      last[std::make_tuple(r.tile_log, r.col_log, r.threads, r.radix_log, r.kara)] = r.us;
  if (last.empty()) return false;
  auto best = last.begin();
  for (auto it = last.begin(); it != last.end(); ++it)
    if (it->second < best->second) best = it;
  *out = NttSchedule{std::get<0>(best->first), std::get<1>(best->first), std::get<2>(best->first),
                     std::get<3>(best->first), std::get<4>(best->first)};
  return true;
}

std::string current_device_name() { return device_name(); }

// median time in microseconds of one transform under schedule s
static int time_schedule(NttPlan& p, const NttSchedule& s, const uint32_t* din, uint32_t* dout, uint32_t warmup,
                         uint32_t reps, hipStream_t st, hipEvent_t e0, hipEvent_t e1, float* us) {
  std::vector<NttPass> ps;
  int rc = plan_passes(p.fe->f.L, p.logn, s, &ps, p.fe->f.fw);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(p.mu);
    p.sched = s;
    p.passes = ps;
  }
  for (uint32_t i = 0; i < warmup; i++) {
    rc = run_plan(p, false, din, dout, st);
    if (rc) return rc;
  }
  // size the inner loop so one timed repetition lasts >= ~200 us
  if (hipEventRecord(e0, st) || run_plan(p, false, din, dout, st) || hipEventRecord(e1, st) ||
      hipEventSynchronize(e1))
    return hip_fail(1, "tuner timing");
  float first = 0;
  (void)hipEventElapsedTime(&first, e0, e1);
  uint32_t inner = (uint32_t)std::min(1000.0, std::max(1.0, std::ceil(0.2 / std::max(first, 1e-4f))));
  std::vector<float> v;
  for (uint32_t r = 0; r < reps; r++) {
    if (hipEventRecord(e0, st)) return hip_fail(1, "event record");
    for (uint32_t i = 0; i < inner; i++) {
      rc = run_plan(p, false, din, dout, st);
      if (rc) return rc;
    }
    if (hipEventRecord(e1, st) || hipEventSynchronize(e1)) return hip_fail(1, "event sync");
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    v.push_back(ms * 1000.0f / inner);
  }
  std::sort(v.begin(), v.end());
  *us = v[v.size() / 2];
  return MOMA_OK;
}

static int tune(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, const moma_tune_opts_t* o,
                moma_tune_result_t* res) {
  std::shared_ptr<NttPlan> p;
  int rc = get_plan(q, omega, n, limbs, &p);
  if (rc) return rc;
  moma_tune_opts_t opts = {5, 2, 0, 0};
  if (o) opts = *o;
  if (opts.reps == 0) opts.reps = 1;
  int L = p->fe->f.L;
  const bool fw = p->fe->f.fw != 0;
  std::vector<NttSchedule> cands = enumerate_schedules(L, p->logn, fw);
  uint32_t feasible = (uint32_t)cands.size();
  if (opts.top_k > 0) {
    std::vector<float> sc;
    rc = costmodel_scores(L, p->logn, cands, &sc);
    if (rc) return rc;
    std::vector<size_t> idx(cands.size());
    for (size_t i = 0; i < idx.size(); i++) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return sc[a] < sc[b]; });
    std::vector<NttSchedule> top;
    for (size_t i = 0; i < idx.size() && i < opts.top_k; i++) top.push_back(cands[idx[i]]);
    cands = top;
  }
  if (opts.max_candidates > 0 && cands.size() > opts.max_candidates) cands.resize(opts.max_candidates);
  if (cands.empty()) return set_error(MOMA_E_UNSUPPORTED, "no feasible schedule");
  // the caller's storage planes (a transform writes all of them), at least the compute limbs
  const int planes = std::max(L, p->fe->f.Ls);
  size_t words = (size_t)p->n * planes;
  uint32_t *din = nullptr, *dout = nullptr;
  if (hipMalloc((void**)&din, words * 4) || hipMalloc((void**)&dout, words * 4)) {
    (void)hipFree(din);
    return set_error(MOMA_E_NOMEM, "tuner buffers");
  }
  // random residues: the kernels' power draw, and with it the clock, depends on the data
  rc = fill_random_residues(p->fe->f, din, p->n, 0x5eed1u, nullptr);
  if (rc) {
    (void)hipFree(din);
    (void)hipFree(dout);
    return rc;
  }
  hipStream_t st;
  hipEvent_t e0, e1;
  (void)hipStreamCreate(&st);
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  NttSchedule prev;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    prev = p->sched;
  }
  std::string dev = device_name();
  float best_us = 0;
  int best = -1;
  std::vector<TuneRow> rows;
  for (size_t i = 0; i < cands.size(); i++) {
    float us = 0;
    rc = time_schedule(*p, cands[i], din, dout, opts.warmup, opts.reps, st, e0, e1, &us);
    if (rc) break;
    const NttSchedule& s = cands[i];
    rows.push_back({dev, (uint32_t)L, p->logn, s.tile_log, s.col_log, s.threads, s.radix_log, us, opts.reps, s.kara});
    if (best < 0 || us < best_us) {
      best = (int)i;
      best_us = us;
    }
  }
  (void)hipStreamSynchronize(st);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  (void)hipFree(din);
  (void)hipFree(dout);
  NttSchedule chosen = (rc == MOMA_OK && best >= 0) ? cands[best] : prev;
  std::vector<NttPass> ps;
  (void)plan_passes(L, p->logn, chosen, &ps, fw);
  {
    std::lock_guard<std::mutex> lk(p->mu);
    p->sched = chosen;
    p->passes = ps;
  }
  if (rc) return rc;
  {
    // the database's rows are keyed by compute limbs and describe the
    // headroom kernels; a full-width plan's timings stay out of it
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!fw) g_rows.insert(g_rows.end(), rows.begin(), rows.end());
  }
  if (res) {
    res->best = {chosen.tile_log, chosen.col_log, chosen.threads, chosen.radix_log, chosen.kara};
    res->best_us = best_us;
    res->timed = (uint32_t)rows.size();
    res->feasible = feasible;
  }
  return MOMA_OK;
}

}  // namespace moma

using namespace moma;

extern "C" {

int moma_ntt_tune(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, const moma_tune_opts_t* opts,
                  moma_tune_result_t* result) {
  return tune(q, omega, n, limbs, opts, result);
}

int moma_ntt_candidates(uint32_t limbs_compute, uint32_t log2_n, moma_ntt_schedule_t* out, uint32_t max,
                        uint32_t* count) {
  if (!count) return set_error(MOMA_E_ARG, "count is NULL");
  if (limbs_compute < 1 || limbs_compute > (uint32_t)kMaxLimbs || log2_n < 1 || log2_n > MOMA_MAX_LOG_N)
    return set_error(MOMA_E_ARG, "limbs or log2_n out of range");
  std::vector<NttSchedule> c = enumerate_schedules((int)limbs_compute, log2_n);
  *count = (uint32_t)c.size();
  if (out)
    for (uint32_t i = 0; i < max && i < c.size(); i++)
      out[i] = {c[i].tile_log, c[i].col_log, c[i].threads, c[i].radix_log, c[i].kara};
  return MOMA_OK;
}

uint32_t moma_tune_db_count(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return (uint32_t)g_rows.size();
}

int moma_tune_db_get(uint32_t i, moma_tune_row_t* row) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!row || i >= g_rows.size()) return set_error(MOMA_E_ARG, "row index out of range");
  const TuneRow& r = g_rows[i];
  row->limbs = r.L;
  row->log2_n = r.logn;
  row->sched = {r.tile_log, r.col_log, r.threads, r.radix_log, r.kara};
  row->us = r.us;
  row->reps = r.reps;
  return MOMA_OK;
}

void moma_tune_db_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_rows.clear();
}

int moma_tune_db_save(const char* path) {
  if (!path) return set_error(MOMA_E_ARG, "path is NULL");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = fopen(path, "w");
  if (!f) return set_error(MOMA_E_ARG, std::string("cannot open ") + path);
  fprintf(f, "device,limbs,log2_n,tile_log,col_log,threads,radix_log,us,reps,mul_variant\n");
  for (const TuneRow& r : g_rows)
    fprintf(f, "%s,%u,%u,%u,%u,%u,%u,%.4f,%u,%u\n", r.device.c_str(), r.L, r.logn, r.tile_log, r.col_log,
            r.threads, r.radix_log, r.us, r.reps, r.kara);
  fclose(f);
  return MOMA_OK;
}

int moma_tune_db_load(const char* path) {
  if (!path) return set_error(MOMA_E_ARG, "path is NULL");
  FILE* f = fopen(path, "r");
  if (!f) return set_error(MOMA_E_ARG, std::string("cannot open ") + path);
  char line[512];
  std::vector<TuneRow> rows;
  bool header = true;
  while (fgets(line, sizeof(line), f)) {
    if (header) {
      header = false;
      continue;
    }
    char dev[128];
    TuneRow r;
    // rows written before the mul_variant column read as schoolbook
    int got = sscanf(line, "%127[^,],%u,%u,%u,%u,%u,%u,%f,%u,%u", dev, &r.L, &r.logn, &r.tile_log, &r.col_log,
                     &r.threads, &r.radix_log, &r.us, &r.reps, &r.kara);
    if ((got != 9 && got != 10) || r.kara > 1) {
      fclose(f);
      return set_error(MOMA_E_ARG, std::string("malformed tuning row: ") + line);
    }
    r.device = dev;
    rows.push_back(r);
  }
  fclose(f);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_rows.insert(g_rows.end(), rows.begin(), rows.end());
  return MOMA_OK;
}

}  // extern "C"
