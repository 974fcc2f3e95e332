// costmodel.cpp - learned cost model for transform schedules.
//
// A small FP32 perceptron (mlp.hip) maps the features of a (size, limbs,
// schedule) triple to the natural log of its measured time in microseconds.
// It is trained on the GPU, by the library's own forward/backward/Adam
// kernels, from rows of the tuner's timing database; the tuner then times only
// the model's best-ranked schedules.  Features (each z-scored with the
// training set's mean and standard deviation):
//   log2 n, compute limbs, log2 radix (stages per register unit), stages fused
//   per pass, log2 threads per workgroup, log2 LDS bytes per workgroup.
// The target is z-scored as well; predictions are mapped back to log(us).
// Minibatch order comes from SplitMix64 (Steele, Lea and Flood 2014) seeded by
// the caller; initial weights are He-normal draws from the same generator
// through the Box-Muller transform.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/moma.h"
#include "common.hpp"
#include "plan.hpp"

namespace moma {

int mlp_nparams();
int launch_mlp_forward(const float* params, const float* x, unsigned rows, float* y, float* h1, float* h2,
                       hipStream_t s);
int launch_mlp_grad(const float* params, const float* x, const float* t, unsigned rows, float* grad, float* loss,
                    float* ws, hipStream_t s);
size_t mlp_grad_workspace_floats(unsigned rows);
int launch_mlp_adam(float* p, const float* g, float* m, float* v, unsigned step, float lr, float b1, float b2,
                    float eps, hipStream_t s);

static const int kFeat = MOMA_COSTMODEL_FEATURES;

struct CostModel {
  bool ready = false;
  std::vector<float> params;
  float fmean[kFeat], fstd[kFeat];
  float tmean = 0, tstd = 1;
};

static std::mutex g_cm_mu;
static CostModel g_cm;
static uint64_t g_cm_gen = 0;  // bumped whenever the model changes
// the model's pick per (compute limbs, log2 n), valid for model generation g_pick_gen
static std::map<std::pair<int, uint32_t>, NttSchedule> g_pick;
static uint64_t g_pick_gen = 0;

static uint64_t sm64(uint64_t key, uint64_t i) {
  uint64_t z = key + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void schedule_features(int L, uint32_t logn, const NttSchedule& s, float* f) {
  std::vector<NttPass> ps;
  std::string keep = g_detail;
  uint32_t fused = 0;
  if (plan_passes(L, logn, s, &ps) == MOMA_OK)
    for (const NttPass& p : ps) fused = std::max(fused, p.k);
  g_detail = keep;
  // one-pass plans hold the whole transform in LDS; multi-pass plans hold one tile
  double lds = 4.0 * L * std::ldexp(1.0, (int)(logn <= s.tile_log ? logn : s.tile_log));
  f[0] = (float)logn;
  f[1] = (float)L;
  f[2] = (float)s.radix_log;
  f[3] = (float)fused;
  f[4] = (float)std::log2((double)s.threads);
  f[5] = (float)std::log2(lds);
  f[6] = (float)s.kara;
}

static int predict_locked(const float* feats, uint32_t rows, float* out) {
  if (!g_cm.ready) return set_error(MOMA_E_UNSUPPORTED, "no cost model is loaded or trained");
  if (rows == 0) return MOMA_OK;
  std::vector<float> xn((size_t)rows * kFeat);
  for (uint32_t r = 0; r < rows; r++)
    for (int j = 0; j < kFeat; j++) xn[(size_t)r * kFeat + j] = (feats[(size_t)r * kFeat + j] - g_cm.fmean[j]) / g_cm.fstd[j];
  float *dp = nullptr, *dx = nullptr, *dy = nullptr;
  int np = mlp_nparams();
  if (hipMalloc((void**)&dp, np * 4) || hipMalloc((void**)&dx, xn.size() * 4) || hipMalloc((void**)&dy, rows * 4)) {
    (void)hipFree(dp);
    (void)hipFree(dx);
    return set_error(MOMA_E_NOMEM, "cost model buffers");
  }
  int e = (int)hipMemcpy(dp, g_cm.params.data(), np * 4, hipMemcpyHostToDevice);
  if (!e) e = (int)hipMemcpy(dx, xn.data(), xn.size() * 4, hipMemcpyHostToDevice);
  if (!e) e = launch_mlp_forward(dp, dx, rows, dy, nullptr, nullptr, 0);
  if (!e) e = (int)hipMemcpy(out, dy, rows * 4, hipMemcpyDeviceToHost);
  (void)hipFree(dp);
  (void)hipFree(dx);
  (void)hipFree(dy);
  if (e) return hip_fail(e, "cost model predict");
  for (uint32_t r = 0; r < rows; r++) out[r] = out[r] * g_cm.tstd + g_cm.tmean;
  return MOMA_OK;
}

int costmodel_scores(int L, uint32_t logn, const std::vector<NttSchedule>& cands, std::vector<float>* scores) {
  std::vector<float> f(cands.size() * kFeat);
  for (size_t i = 0; i < cands.size(); i++) schedule_features(L, logn, cands[i], &f[i * kFeat]);
  scores->assign(cands.size(), 0.f);
  std::lock_guard<std::mutex> lk(g_cm_mu);
  return predict_locked(f.data(), (uint32_t)cands.size(), scores->data());
}

bool costmodel_pick(int L, uint32_t logn, NttSchedule* out) {
  const std::pair<int, uint32_t> key(L, logn);
  {
    std::lock_guard<std::mutex> lk(g_cm_mu);
    if (!g_cm.ready) return false;
    if (g_pick_gen != g_cm_gen) {
      g_pick.clear();
      g_pick_gen = g_cm_gen;
    }
    auto it = g_pick.find(key);
    if (it != g_pick.end()) {
      *out = it->second;
      return true;
    }
  }
  std::string keep = g_detail;
  std::vector<NttSchedule> cands = enumerate_schedules(L, logn);
  std::vector<float> sc;
  if (cands.empty() || costmodel_scores(L, logn, cands, &sc) != MOMA_OK) {
    g_detail = keep;
    return false;
  }
  size_t best = 0;
  for (size_t i = 1; i < cands.size(); i++)
    if (sc[i] < sc[best]) best = i;
  *out = cands[best];
  std::lock_guard<std::mutex> lk(g_cm_mu);
  g_pick[key] = *out;
  return true;
}

static void he_init(uint64_t seed, std::vector<float>* p) {
  int np = mlp_nparams();
  p->assign(np, 0.f);
  uint64_t key = sm64(0x6d6f6d61ull, seed);
  uint64_t ctr = 0;
  auto normal = [&]() {
    double u1 = ((double)(sm64(key, ctr++) >> 11) + 1.0) / 9007199254740992.0;
    double u2 = ((double)(sm64(key, ctr++) >> 11) + 1.0) / 9007199254740992.0;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
  };
  const int H = 64, I = kFeat;
  int o = 0;
  for (int i = 0; i < H * I; i++) (*p)[o + i] = (float)(normal() * std::sqrt(2.0 / I));
  o += H * I + H;
  for (int i = 0; i < H * H; i++) (*p)[o + i] = (float)(normal() * std::sqrt(2.0 / H));
  o += H * H + H;
  for (int i = 0; i < H; i++) (*p)[o + i] = (float)(normal() * std::sqrt(2.0 / H));
}

static int train(const float* feats, const float* target, uint32_t rows, const moma_train_opts_t* o, float* final_loss) {
  if (!feats || !target || rows < 2) return set_error(MOMA_E_ARG, "need at least two training rows");
  moma_train_opts_t opts = {200, 256, 3e-3f, 1};
  if (o) opts = *o;
  if (opts.batch == 0 || opts.epochs == 0) return set_error(MOMA_E_ARG, "epochs and batch must be positive");
  CostModel m;
  for (int j = 0; j < kFeat; j++) {
    double s = 0, s2 = 0;
    for (uint32_t r = 0; r < rows; r++) s += feats[(size_t)r * kFeat + j];
    double mu = s / rows;
    for (uint32_t r = 0; r < rows; r++) s2 += std::pow(feats[(size_t)r * kFeat + j] - mu, 2);
    m.fmean[j] = (float)mu;
    m.fstd[j] = (float)std::max(std::sqrt(s2 / rows), 1e-6);
  }
  {
    double s = 0, s2 = 0;
    for (uint32_t r = 0; r < rows; r++) s += target[r];
    double mu = s / rows;
    for (uint32_t r = 0; r < rows; r++) s2 += std::pow(target[r] - mu, 2);
    m.tmean = (float)mu;
    m.tstd = (float)std::max(std::sqrt(s2 / rows), 1e-6);
  }
  he_init(opts.seed, &m.params);
  int np = mlp_nparams();
  std::vector<float> xn((size_t)rows * kFeat), tn(rows);
  for (uint32_t r = 0; r < rows; r++) {
    for (int j = 0; j < kFeat; j++) xn[(size_t)r * kFeat + j] = (feats[(size_t)r * kFeat + j] - m.fmean[j]) / m.fstd[j];
    tn[r] = (target[r] - m.tmean) / m.tstd;
  }
  uint32_t B = std::min(opts.batch, rows);
  float *dp = nullptr, *dg = nullptr, *dm = nullptr, *dv = nullptr, *dx = nullptr, *dt = nullptr, *dl = nullptr,
        *ws = nullptr;
  size_t wsz = mlp_grad_workspace_floats(rows);
  bool ok = !hipMalloc((void**)&dp, np * 4) && !hipMalloc((void**)&dg, np * 4) && !hipMalloc((void**)&dm, np * 4) &&
            !hipMalloc((void**)&dv, np * 4) && !hipMalloc((void**)&dx, xn.size() * 4) &&
            !hipMalloc((void**)&dt, rows * 4) && !hipMalloc((void**)&dl, 4) && !hipMalloc((void**)&ws, wsz * 4);
  auto release = [&]() {
    for (float* q : {dp, dg, dm, dv, dx, dt, dl, ws}) (void)hipFree(q);
  };
  if (!ok) {
    release();
    return set_error(MOMA_E_NOMEM, "cost model training buffers");
  }
  int e = (int)hipMemcpy(dp, m.params.data(), np * 4, hipMemcpyHostToDevice);
  if (!e) e = (int)hipMemset(dm, 0, np * 4);
  if (!e) e = (int)hipMemset(dv, 0, np * 4);
  std::vector<uint32_t> perm(rows);
  std::vector<float> xs(xn.size()), ts(rows);
  uint64_t key = sm64(0x73687566ull, opts.seed);
  uint32_t step = 0;
  for (uint32_t ep = 0; ep < opts.epochs && !e; ep++) {
    for (uint32_t r = 0; r < rows; r++) perm[r] = r;
    for (uint32_t r = rows - 1; r > 0; r--) {  // Fisher-Yates
      uint32_t j = (uint32_t)(sm64(key, (uint64_t)ep * rows + r) % (r + 1));
      std::swap(perm[r], perm[j]);
    }
    for (uint32_t r = 0; r < rows; r++) {
      memcpy(&xs[(size_t)r * kFeat], &xn[(size_t)perm[r] * kFeat], kFeat * 4);
      ts[r] = tn[perm[r]];
    }
    e = (int)hipMemcpy(dx, xs.data(), xs.size() * 4, hipMemcpyHostToDevice);
    if (!e) e = (int)hipMemcpy(dt, ts.data(), rows * 4, hipMemcpyHostToDevice);
    for (uint32_t b0 = 0; b0 + B <= rows && !e; b0 += B) {
      e = launch_mlp_grad(dp, dx + (size_t)b0 * kFeat, dt + b0, B, dg, dl, ws, 0);
      if (!e) e = launch_mlp_adam(dp, dg, dm, dv, ++step, opts.lr, 0.9f, 0.999f, 1e-8f, 0);
    }
  }
  float loss = 0;
  if (!e) e = (int)hipMemcpy(dx, xn.data(), xn.size() * 4, hipMemcpyHostToDevice);
  if (!e) e = (int)hipMemcpy(dt, tn.data(), rows * 4, hipMemcpyHostToDevice);
  if (!e) e = launch_mlp_grad(dp, dx, dt, rows, dg, dl, ws, 0);
  if (!e) e = (int)hipMemcpy(&loss, dl, 4, hipMemcpyDeviceToHost);
  if (!e) e = (int)hipMemcpy(m.params.data(), dp, np * 4, hipMemcpyDeviceToHost);
  release();
  if (e) return hip_fail(e, "cost model training");
  m.ready = true;
  if (final_loss) *final_loss = loss * m.tstd * m.tstd;  // mean squared error in (log us)^2
  std::lock_guard<std::mutex> lk(g_cm_mu);
  g_cm = m;
  return MOMA_OK;
}

}  // namespace moma

using namespace moma;

extern "C" {

uint32_t moma_mlp_nparams(void) { return (uint32_t)mlp_nparams(); }

int moma_mlp_forward(const float* d_params, const float* d_x, uint32_t rows, float* d_y, void* stream) {
  if (!d_params || (rows && (!d_x || !d_y))) return set_error(MOMA_E_ARG, "NULL pointer");
  int e = launch_mlp_forward(d_params, d_x, rows, d_y, nullptr, nullptr, (hipStream_t)stream);
  return e ? hip_fail(e, "mlp forward") : MOMA_OK;
}

int moma_mlp_grad(const float* d_params, const float* d_x, const float* d_t, uint32_t rows, float* d_grad,
                  float* d_loss, void* stream) {
  if (!d_params || !d_x || !d_t || !d_grad || !d_loss || rows == 0) return set_error(MOMA_E_ARG, "bad argument");
  float* ws = nullptr;
  if (hipMalloc((void**)&ws, mlp_grad_workspace_floats(rows) * 4)) return set_error(MOMA_E_NOMEM, "mlp workspace");
  int e = launch_mlp_grad(d_params, d_x, d_t, rows, d_grad, d_loss, ws, (hipStream_t)stream);
  if (!e) e = (int)hipStreamSynchronize((hipStream_t)stream);
  (void)hipFree(ws);
  return e ? hip_fail(e, "mlp grad") : MOMA_OK;
}

int moma_mlp_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t step, float lr, float beta1,
                  float beta2, float eps, void* stream) {
  if (!d_params || !d_grad || !d_m || !d_v || step == 0) return set_error(MOMA_E_ARG, "bad argument");
  int e = launch_mlp_adam(d_params, d_grad, d_m, d_v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
  return e ? hip_fail(e, "mlp adam") : MOMA_OK;
}

int moma_costmodel_features(uint32_t limbs_compute, uint32_t log2_n, const moma_ntt_schedule_t* sched, float* out7) {
  if (!sched || !out7) return set_error(MOMA_E_ARG, "NULL pointer");
  NttSchedule s{sched->tile_log, sched->col_log, sched->threads, sched->radix_log, sched->mul_variant};
  schedule_features((int)limbs_compute, log2_n, s, out7);
  return MOMA_OK;
}

int moma_costmodel_train(const float* features, const float* log_us, uint32_t rows, const moma_train_opts_t* opts,
                         float* final_mse) {
  return train(features, log_us, rows, opts, final_mse);
}

int moma_costmodel_predict(const float* features, uint32_t rows, float* log_us) {
  if (!features || !log_us) return set_error(MOMA_E_ARG, "NULL pointer");
  std::lock_guard<std::mutex> lk(g_cm_mu);
  return predict_locked(features, rows, log_us);
}

int moma_costmodel_save(const char* path) {
  std::lock_guard<std::mutex> lk(g_cm_mu);
  if (!g_cm.ready) return set_error(MOMA_E_UNSUPPORTED, "no cost model to save");
  FILE* f = fopen(path, "w");
  if (!f) return set_error(MOMA_E_ARG, std::string("cannot open ") + path);
  fprintf(f, "moma-costmodel 1 %d\n", (int)g_cm.params.size());
  for (int j = 0; j < kFeat; j++) fprintf(f, "%.9g %.9g\n", g_cm.fmean[j], g_cm.fstd[j]);
  fprintf(f, "%.9g %.9g\n", g_cm.tmean, g_cm.tstd);
  for (float v : g_cm.params) fprintf(f, "%.9g\n", v);
  fclose(f);
  return MOMA_OK;
}

int moma_costmodel_load(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return set_error(MOMA_E_ARG, std::string("cannot open ") + path);
  CostModel m;
  int ver = 0, np = 0;
  bool ok = fscanf(f, "moma-costmodel %d %d", &ver, &np) == 2 && ver == 1 && np == mlp_nparams();
  for (int j = 0; ok && j < kFeat; j++) ok = fscanf(f, "%f %f", &m.fmean[j], &m.fstd[j]) == 2;
  ok = ok && fscanf(f, "%f %f", &m.tmean, &m.tstd) == 2;
  m.params.resize(np > 0 ? np : 0);
  for (int i = 0; ok && i < np; i++) ok = fscanf(f, "%f", &m.params[i]) == 1;
  fclose(f);
  if (!ok) return set_error(MOMA_E_ARG, std::string("malformed cost model file ") + path);
  m.ready = true;
  std::lock_guard<std::mutex> lk(g_cm_mu);
  g_cm = m;
  g_cm_gen++;
  return MOMA_OK;
}

void moma_costmodel_clear(void) {
  std::lock_guard<std::mutex> lk(g_cm_mu);
  g_cm = CostModel();
  g_cm_gen++;
}

}  // extern "C"
