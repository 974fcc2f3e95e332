// capi.cpp - host runtime behind include/moma.h: argument validation, per-modulus
// constants, the transform plan cache (twiddle tables, pass schedule, scratch)
// and the extern "C" entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/moma.h"
#include "common.hpp"
#include "hostbig.hpp"
#include "plan.hpp"

namespace moma {

thread_local std::string g_detail;

int set_error(int code, const std::string& detail) {
  g_detail = detail;
  return code;
}

int hip_fail(int e, const char* what) {
  if (e == 0) return MOMA_OK;
  return set_error(MOMA_E_HIP, std::string(what) + ": " + hipGetErrorString((hipError_t)e));
}

// ------------------------------------------------------------------ fields

std::mutex g_mu;
static std::map<std::vector<uint32_t>, std::shared_ptr<FieldEntry>> g_fields;

// v (< 2^(bD)) as the D b-bit digits of the transform's digit form
static void digits_of(const HBig& v, int L, bool fw, uint32_t* out) {
  int b = digit_bits(L), D = digit_count(L, fw);
  for (int i = 0; i < D; i++) {
    uint32_t w[2] = {0, 0};
    HBig::shr(v, b * i).to_limbs(w, 2);
    out[i] = w[0] & ((1u << b) - 1);
  }
}

int build_field(const uint32_t* q, uint32_t limbs, std::shared_ptr<FieldEntry>* out) {
  if (!q) return set_error(MOMA_E_ARG, "q is NULL");
  if (limbs < MOMA_MIN_LIMBS || limbs > MOMA_MAX_LIMBS)
    return set_error(MOMA_E_ARG, "limbs must be in [2, 32], got " + std::to_string(limbs));
  std::vector<uint32_t> key(q, q + limbs);
  key.push_back(limbs);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_fields.find(key);
    if (it != g_fields.end()) {
      *out = it->second;
      return MOMA_OK;
    }
  }
  auto fe = std::make_shared<FieldEntry>();
  HBig Q = HBig::from_limbs(q, (int)limbs);
  if (!Q.is_odd() || HBig::cmp(Q, HBig(3)) < 0) return set_error(MOMA_E_MODULUS, "q must be odd and >= 3");
  int M = Q.bitlen();
  if (M > 32 * (int)limbs)
    return set_error(MOMA_E_MODULUS, "bitlen(q) = " + std::to_string(M) + " exceeds 32*limbs = " +
                                         std::to_string(32 * limbs));
  FieldRaw& f = fe->f;
  memset(&f, 0, sizeof(f));
  // compute limbs keep 4 bits of headroom for the lazy reductions and
  // Barrett's pre-scaled modulus; a modulus within 4 bits of the storage
  // width (full width) computes in the storage limbs with canonical operands
  // and Montgomery products that carry out of the top limb
  f.L = (M + 4 + 31) / 32;
  f.fw = f.L > (int)limbs ? 1 : 0;
  if (f.fw) f.L = (int)limbs;
  f.Ls = (int)limbs;
  Q.to_limbs(f.q, kMaxLimbs);
  f.qinv = neg_inv32(f.q[0]);
  HBig one_m = HBig::mod(HBig::pow2(32 * f.L), Q);
  one_m.to_limbs(f.one_m, kMaxLimbs);
  HBig::mod(HBig::pow2(64 * f.L), Q).to_limbs(f.r2, kMaxLimbs);
  if (!f.fw) {
    int Mn = 32 * f.L - 4;
    f.d = (uint32_t)(Mn - M);
    HBig qn = HBig::shl(Q, (int)f.d);
    qn.to_limbs(f.qn, kMaxLimbs);
    HBig mu;
    HBig::divmod(HBig::pow2(2 * Mn + 3), qn, &mu, nullptr);
    if (mu.bitlen() > 32 * f.L) return set_error(MOMA_E_MODULUS, "internal: Barrett constant too wide");
    mu.to_limbs(f.mu, kMaxLimbs);
  }
  // digit form of the transform's twiddle multiply
  {
    DigitConsts& dc = fe->dc;
    memset(&dc, 0, sizeof(dc));
    int b = digit_bits(f.L), D = digit_count(f.L, f.fw);
    digits_of(Q, f.L, f.fw, dc.qd);
    dc.qinvd = f.qinv & ((1u << b) - 1);
    fe->adj = HBig::mod(HBig::pow2(b * D), Q);
    fe->adj.to_limbs(dc.adj, kMaxLimbs);
  }
  fe->Q = Q;
  fe->one_m = one_m;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_fields.find(key);
  if (it != g_fields.end()) {
    *out = it->second;
  } else {
    g_fields[key] = fe;
    *out = fe;
  }
  return MOMA_OK;
}

// ------------------------------------------------------------------ transform plans

static std::map<std::vector<uint32_t>, std::shared_ptr<NttPlan>> g_plans;

uint32_t max_radix_log(int L, bool fw) {
  uint32_t r = L <= kMaxLimbsRadix16 ? 4u : (L <= kMaxLimbsRadix8 ? 3u : (L <= kMaxLimbsRadix4 ? 2u : 1u));
  return fw ? std::min(r, L <= kMaxLimbsRadix4Fw ? 2u : 1u) : r;
}

// Split log2 n stages into passes for a schedule; returns MOMA_OK or an error
// code when the schedule cannot run this size.
int plan_passes(int L, uint32_t logn, const NttSchedule& s, std::vector<NttPass>* out, bool fw) {
  if (s.threads < 64 || s.threads > 1024 || s.threads % 64)
    return set_error(MOMA_E_ARG, "threads must be a multiple of 64 in [64, 1024]");
  if (s.radix_log < 1 || s.radix_log > max_radix_log(L, fw))
    return set_error(MOMA_E_UNSUPPORTED, "radix_log out of range for this limb count");
  if (s.kara > 1) return set_error(MOMA_E_ARG, "unknown multiply variant");
  if (s.kara && (fw || s.radix_log != 1 || L < 2 || L > kMaxLimbsKara))
    return set_error(MOMA_E_UNSUPPORTED,
                     "the Karatsuba butterfly runs radix-2 units at 2 to 24 compute limbs (not full width)");
  if (s.threads > ntt_max_threads(L, s.radix_log))
    return set_error(MOMA_E_UNSUPPORTED, "too many threads for this limb count and radix");
  if (s.tile_log < 1 || s.tile_log > 20) return set_error(MOMA_E_ARG, "tile_log out of range");
  if (((uint64_t)L << s.tile_log) * 4 > 160 * 1024)
    return set_error(MOMA_E_UNSUPPORTED, "tile exceeds the 160 KiB LDS of a compute unit");
  std::vector<NttPass> ps;
  uint64_t n = 1ull << logn;
  if (logn <= s.tile_log) {
    ps.push_back({0, logn, 0, 1});
  } else {
    if (s.col_log < 1 || s.col_log + 1 > s.tile_log) return set_error(MOMA_E_ARG, "col_log out of range");
    uint32_t kmax = s.tile_log - s.col_log;
    uint32_t P = (logn + kmax - 1) / kmax;
    uint32_t base = logn / P, extra = logn % P;
    uint32_t K = 0;
    for (uint32_t i = 0; i < P; i++) {
      uint32_t k = base + (i < extra ? 1 : 0);
      // the C groups of a tile need C offsets (first pass) or C blocks (later passes)
      if (K == 0 && logn - k < s.col_log) return set_error(MOMA_E_UNSUPPORTED, "first pass too wide");
      if (K > 0 && K < s.col_log) return set_error(MOMA_E_UNSUPPORTED, "pass needs more blocks than columns");
      ps.push_back({K, k, s.col_log, n >> (k + s.col_log)});
      K += k;
    }
  }
  *out = ps;
  return MOMA_OK;
}

// First feasible of an ordered list of (tile_log, col_log), with the radix
// and thread count filled in by rule: radix 4 up to max_limbs_radix4 limbs,
// and enough threads to give each one or two units per round.  (From 11 limbs
// a radix-4 unit holds the lane at 3 waves per SIMD, 2 from 13.  For a lone
// transform the fixed rule stays at radix 2 there, and the tuner and the cost
// model find where radix 4 pays.  Inside a batch, where other jobs fill the
// chip, 12-limb jobs take radix 4: the 4096-job batch ran 6.78 ms against
// 6.89 ms with radix 2.)
constexpr int kRuleMaxLimbsRadix4 = 10, kBatchMaxLimbsRadix4 = 12;
static NttSchedule first_feasible(int L, uint32_t logn, const std::vector<std::pair<uint32_t, uint32_t>>& shapes,
                                  int max_limbs_radix4 = kRuleMaxLimbsRadix4) {
  uint32_t radix = std::min(L <= max_limbs_radix4 ? 2u : 1u, max_radix_log(L));
  std::string keep = g_detail;
  NttSchedule last{};
  for (auto tc : shapes) {
    NttSchedule s{tc.first, tc.second, 0, radix};
    uint32_t e = std::min(logn, s.tile_log);
    uint32_t units = 1u << (e > s.radix_log ? e - s.radix_log : 0);
    uint32_t t = std::min(units > 256 ? 256u : units, ntt_max_threads(L, s.radix_log));
    s.threads = t < 64 ? 64 : (t + 63) / 64 * 64;
    last = s;
    std::vector<NttPass> ps;
    if (plan_passes(L, logn, s, &ps) == MOMA_OK) {
      g_detail = keep;
      return s;
    }
  }
  g_detail = keep;
  return last;
}

static uint32_t tile_log_for(uint32_t words) {
  uint32_t t = 0;
  while ((2u << t) <= words) t++;
  return t;
}

// Default launch shape, first feasible of: one pass when the whole transform
// fits a 64 KiB tile; otherwise 32 KiB tiles (several workgroups per CU) with
// 16, 8 or 4 coalesced columns, then 64 KiB tiles.
NttSchedule default_schedule(int L, uint32_t logn) {
  uint32_t t64 = tile_log_for(16384u / (uint32_t)L), t32 = tile_log_for(8192u / (uint32_t)L);
  std::vector<std::pair<uint32_t, uint32_t>> shapes;
  if (logn <= t64) shapes.push_back({logn, 0});
  for (uint32_t cl : {4u, 3u, 2u}) shapes.push_back({t32, cl});
  for (uint32_t cl : {4u, 3u, 2u, 1u}) shapes.push_back({t64, cl});
  return first_feasible(L, logn, shapes);
}

// Shape for a small job inside a batch, where other jobs fill the chip: one
// pass when the transform fits a 64 KiB tile, else the largest tiles (fewest
// passes) with 32 or 16 columns.
NttSchedule batch_schedule(int L, uint32_t logn) {
  uint32_t t64 = tile_log_for(16384u / (uint32_t)L), t32 = tile_log_for(8192u / (uint32_t)L);
  std::vector<std::pair<uint32_t, uint32_t>> shapes;
  if (logn <= t64) shapes.push_back({logn, 0});
  for (uint32_t cl : {5u, 4u}) shapes.push_back({t64, cl});
  for (uint32_t cl : {5u, 4u, 3u, 2u}) shapes.push_back({t32, cl});
  for (uint32_t cl : {3u, 2u, 1u}) shapes.push_back({t64, cl});
  return first_feasible(L, logn, shapes, kBatchMaxLimbsRadix4);
}

NttSchedule initial_schedule(int L, uint32_t logn, bool fw) {
  std::string keep = g_detail;
  NttSchedule s;
  std::vector<NttPass> ps;
  bool ok = tune_db_best(current_device_name(), L, logn, &s) && plan_passes(L, logn, s, &ps, fw) == MOMA_OK;
  if (!ok) ok = costmodel_pick(L, logn, &s) && plan_passes(L, logn, s, &ps, fw) == MOMA_OK;
  if (!ok) s = default_schedule(L, logn);
  g_detail = keep;
  return s;
}

static int check_planes(const NttPlan& p) {
  for (const NttPass& s : p.passes) {
    if (s.K == 0 && (p.n >> s.k) < (1ull << s.logc)) return -1;
    if (s.K > 0 && (1ull << s.K) < (1ull << s.logc)) return -1;
  }
  return 0;
}

// device copy of host words; on failure *dptr is left NULL and nothing is held
static int upload(uint32_t** dptr, const std::vector<uint32_t>& host) {
  *dptr = nullptr;
  int e = (int)hipMalloc((void**)dptr, host.size() * sizeof(uint32_t));
  if (e) {
    *dptr = nullptr;
    return e;
  }
  e = (int)hipMemcpy(*dptr, host.data(), host.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e) {
    (void)hipFree(*dptr);
    *dptr = nullptr;
  }
  return e;
}

static void free_tables(DirTables* t) {
  (void)hipFree(t->tw);
  (void)hipFree(t->ladder);
  t->tw = t->ladder = nullptr;
}

// One direction's ladder and twiddle table.  On failure both are freed (and
// NULL), so a failed plan build holds no device memory for this direction.
static int build_tables(NttPlan& p, const HBig& w, DirTables* t) {
  const FieldRaw& f = p.fe->f;
  const HBig& Q = p.fe->Q;
  int L = f.L;
  std::vector<uint32_t> lad((size_t)(p.logn + 2) * L);
  HBig cur = w;
  for (uint32_t b = 0; b < p.logn; b++) {
    HBig m = HBig::mulmod(cur, p.fe->one_m, Q);
    m.to_limbs(&lad[(size_t)b * L], L);
    cur = HBig::mulmod(cur, cur, Q);
  }
  p.fe->one_m.to_limbs(&lad[(size_t)p.logn * L], L);
  for (int j = 0; j < L; j++) lad[(size_t)(p.logn + 1) * L + j] = p.fe->dc.adj[j];
  int e = upload(&t->ladder, lad);
  if (e) return hip_fail(e, "ladder upload");
  e = (int)hipMalloc((void**)&t->tw, (size_t)p.n * digit_stride(L, f.fw) * sizeof(uint32_t));
  if (e) {
    t->tw = nullptr;
    free_tables(t);
    return set_error(MOMA_E_NOMEM, "twiddle table allocation failed");
  }
  e = launch_twiddle_gen(f, p.fe->dc, t->tw, p.n, p.logn, t->ladder, 0);
  if (e) {
    free_tables(t);
    return hip_fail(e, "twiddle generation launch");
  }
  return MOMA_OK;
}

static std::vector<uint32_t> plan_key(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, int dev) {
  std::vector<uint32_t> key(q, q + limbs);
  key.insert(key.end(), omega, omega + limbs);
  key.push_back(limbs);
  key.push_back((uint32_t)n);
  key.push_back((uint32_t)(n >> 32));
  key.push_back((uint32_t)dev);
  return key;
}

int find_plan(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, std::shared_ptr<NttPlan>* out) {
  if (!q || !omega) return set_error(MOMA_E_ARG, "q or omega is NULL");
  if (limbs < MOMA_MIN_LIMBS || limbs > MOMA_MAX_LIMBS)
    return set_error(MOMA_E_ARG, "limbs must be in [2, 32], got " + std::to_string(limbs));
  if (n < 2 || (n & (n - 1)) || n > (1ull << MOMA_MAX_LOG_N))
    return set_error(MOMA_E_ARG, "n must be a power of two in [2, 2^26], got " + std::to_string(n));
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::vector<uint32_t> key = plan_key(q, omega, n, limbs, dev);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_plans.find(key);
  if (it == g_plans.end())
    return set_error(MOMA_E_ARG, "no plan for these arguments on this device: build it first (moma_ntt_prepare)");
  *out = it->second;
  return MOMA_OK;
}

int get_plan(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, std::shared_ptr<NttPlan>* out) {
  if (!omega) return set_error(MOMA_E_ARG, "omega is NULL");
  if (n < 2 || (n & (n - 1)) || n > (1ull << MOMA_MAX_LOG_N))
    return set_error(MOMA_E_ARG, "n must be a power of two in [2, 2^26], got " + std::to_string(n));
  std::shared_ptr<FieldEntry> fe;
  int rc = build_field(q, limbs, &fe);
  if (rc) return rc;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::vector<uint32_t> key = plan_key(q, omega, n, limbs, dev);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
      *out = it->second;
      return MOMA_OK;
    }
  }
  const HBig& Q = fe->Q;
  HBig W = HBig::from_limbs(omega, (int)limbs);
  if (HBig::cmp(W, Q) >= 0) return set_error(MOMA_E_ROOT, "omega must be < q");
  HBig qm1 = HBig::sub(Q, HBig(1));
  HBig nq, nr;
  HBig::divmod(qm1, HBig(n), &nq, &nr);
  if (!nr.is_zero()) return set_error(MOMA_E_ROOT, "n does not divide q - 1");
  // order exactly n  <=>  w^(n/2) == -1 (n a power of two)
  if (HBig::cmp(HBig::powmod(W, HBig(n / 2), Q), qm1) != 0)
    return set_error(MOMA_E_ROOT, "omega^(n/2) != q - 1: omega is not a primitive n-th root of unity");
  auto p = std::make_shared<NttPlan>();
  p->fe = fe;
  p->device = dev;
  p->n = n;
  p->logn = 0;
  while ((1ull << p->logn) < n) p->logn++;
  p->sched = initial_schedule(fe->f.L, p->logn, fe->f.fw);
  rc = plan_passes(fe->f.L, p->logn, p->sched, &p->passes, fe->f.fw);
  if (rc) return rc;
  if (check_planes(*p)) return set_error(MOMA_E_UNSUPPORTED, "no valid pass split for this size");
  HBig Winv = HBig::powmod(W, HBig(n - 1), Q);
  HBig ninv = HBig::sub(Q, nq);  // n * (q - (q-1)/n) == 1 mod q
  // last-pass scales in digit Montgomery form (R = 2^(bD)): n^-1 R for the
  // inverse; n^-1 R^2 after the fused pointwise product of a cyclic product,
  // which leaves a factor R^-1
  const HBig& rd = fe->adj;
  HBig nscale = HBig::mulmod(ninv, rd, Q);
  memset(&p->inv_consts, 0, sizeof(p->inv_consts));
  digits_of(nscale, fe->f.L, fe->f.fw, p->inv_consts.nscale_d);
  memset(&p->mul_consts, 0, sizeof(p->mul_consts));
  digits_of(HBig::mulmod(nscale, rd, Q), fe->f.L, fe->f.fw, p->mul_consts.nscale_d);
  rc = build_tables(*p, W, &p->fwd);
  if (rc) return rc;
  rc = build_tables(*p, Winv, &p->inv);
  if (rc) {
    free_tables(&p->fwd);  // (the plan's destructor would too; freed here so the failure path holds nothing)
    return rc;
  }
  int e = (int)hipDeviceSynchronize();
  if (e) return hip_fail(e, "plan build");
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    *out = it->second;
  } else {
    g_plans[key] = p;
    *out = p;
  }
  return MOMA_OK;
}

// Enqueue the passes of one transform over the compute limbs.  d_in2, when
// set, is multiplied into d_in element by element as the first pass loads
// (a Montgomery product, so c must carry the matching scale).  first_out is
// where the first pass writes when there are several (the later ones work in
// place on d_out).
static int enqueue_passes(NttPlan& p, const std::vector<NttPass>& passes, const NttSchedule& sched,
                          const DirTables& t, const NttConsts& c, bool scale, const uint32_t* d_in,
                          const uint32_t* d_in2, uint32_t* first_out, uint32_t* d_out, hipStream_t s) {
  const FieldRaw& f = p.fe->f;
  size_t P = passes.size();
  for (size_t i = 0; i < P; i++) {
    const NttPass& ps = passes[i];
    NttPassArgs a{};
    a.in = (i == 0) ? d_in : (i == 1 ? first_out : d_out);
    a.in2 = (i == 0) ? d_in2 : nullptr;
    a.out = (i == 0) ? first_out : d_out;
    a.tw = t.tw;
    a.n = p.n;
    a.logn = p.logn;
    a.K = ps.K;
    a.k = ps.k;
    a.logc = ps.logc;
    a.last = (i + 1 == P) ? 1u : 0u;
    a.scale = (scale && i + 1 == P) ? 1u : 0u;
    int e = launch_ntt_pass(f, p.fe->dc, a, c, sched.threads, ps.tiles, sched.radix_log, sched.kara, s);
    if (e) return hip_fail(e, "ntt pass launch");
  }
  return MOMA_OK;
}

int fill_random_residues(const FieldRaw& f, uint32_t* d, uint64_t n, uint32_t seed, hipStream_t s) {
  int top = kMaxLimbs - 1;
  while (top > 0 && f.q[top] == 0) top--;
  uint32_t m = f.q[top];  // q's top limb, >= 1: keep the top word strictly below it
  uint32_t mask = 0;
  while (mask < (m >> 1)) mask = (mask << 1) | 1u;
  if (mask >= m) mask >>= 1;
  int e = launch_fill_residues(d, n, f.Ls, top, mask, seed, s);
  if (!e) e = (int)hipStreamSynchronize(s);
  return e ? hip_fail(e, "random residues") : MOMA_OK;
}

// lazily allocated per-plan buffer of n x L words (under the plan's mutex)
static int plan_buffer(NttPlan& p, uint32_t** slot, size_t copies, const char* what) {
  if (!*slot && hipMalloc((void**)slot, copies * (size_t)p.n * p.fe->f.L * sizeof(uint32_t)))
    return set_error(MOMA_E_NOMEM, std::string(what) + " allocation failed");
  return MOMA_OK;
}

int run_plan(NttPlan& p, bool inverse, const uint32_t* d_in, uint32_t* d_out, hipStream_t s) {
  const FieldRaw& f = p.fe->f;
  std::vector<NttPass> passes;
  NttSchedule sched;
  uint32_t* first_out = d_out;
  {
    std::lock_guard<std::mutex> lk(p.mu);
    passes = p.passes;
    sched = p.sched;
    if (passes.size() > 1 && d_in == d_out) {
      int rc = plan_buffer(p, &p.scratch, 1, "scratch");
      if (rc) return rc;
      first_out = p.scratch;
    }
  }
  NttConsts none;
  memset(&none, 0, sizeof(none));
  const DirTables& t = inverse ? p.inv : p.fwd;
  const NttConsts& nc = inverse ? p.inv_consts : none;
  int rc = enqueue_passes(p, passes, sched, t, nc, inverse, d_in, nullptr, first_out, d_out, s);
  if (rc) return rc;
  if (f.Ls > f.L && d_out != d_in) {
    int e = launch_zero_planes(d_out, p.n, f.L, f.Ls, s);
    if (e) return hip_fail(e, "zero planes launch");
  }
  return MOMA_OK;
}

// Cyclic product a * b mod (x^n - 1): both forward transforms go to the
// plan's spectra buffer, and the inverse transform's first pass multiplies
// them pointwise while loading (digit-form Montgomery, a factor 2^(-bD)); its
// last pass scales by n^-1 2^(bD), which cancels that factor.
uint64_t cyclic_mul_scratch_words(const NttPlan& p) { return 2ull * p.n * (uint64_t)p.fe->f.L; }

int run_cyclic_mul(NttPlan& p, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_out, hipStream_t s,
                   uint32_t* ext) {
  const FieldRaw& f = p.fe->f;
  std::vector<NttPass> passes;
  NttSchedule sched;
  uint32_t* spec = ext;  // caller-provided scratch: [spectrum a | spectrum b]
  {
    std::lock_guard<std::mutex> lk(p.mu);
    passes = p.passes;
    sched = p.sched;
    if (!ext) {
      int rc = plan_buffer(p, &p.spectra, 2, "spectra");
      if (rc) return rc;
      spec = p.spectra;
    }
  }
  uint32_t* sa = spec;
  uint32_t* sb = spec + (size_t)p.n * f.L;
  NttConsts none;
  memset(&none, 0, sizeof(none));
  int rc = enqueue_passes(p, passes, sched, p.fwd, none, false, d_a, nullptr, sa, sa, s);
  if (!rc) rc = enqueue_passes(p, passes, sched, p.fwd, none, false, d_b, nullptr, sb, sb, s);
  if (!rc) rc = enqueue_passes(p, passes, sched, p.inv, p.mul_consts, true, sa, sb, d_out, d_out, s);
  if (rc) return rc;
  if (f.Ls > f.L) {
    int e = launch_zero_planes(d_out, p.n, f.L, f.Ls, s);
    if (e) return hip_fail(e, "zero planes launch");
  }
  return MOMA_OK;
}

// ------------------------------------------------------------------ input check

static int g_check_inputs = -1;  // -1: MOMA_CHECK_INPUTS not read yet

bool input_check_on() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_check_inputs < 0) {
    const char* e = getenv("MOMA_CHECK_INPUTS");
    g_check_inputs = (e && *e && strcmp(e, "0") != 0) ? 1 : 0;
  }
  return g_check_inputs == 1;
}

int count_noncanonical(const FieldRaw& f, const uint32_t* d_x, uint64_t n, hipStream_t s, uint64_t* bad,
                       uint32_t* d_part) {
  *bad = 0;
  if (n == 0) return MOMA_OK;
  const uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (n + 255) / 256);
  const bool own = d_part == nullptr;
  if (own && hipMalloc((void**)&d_part, blocks * sizeof(uint32_t)))
    return set_error(MOMA_E_NOMEM, "input check buffer");
  std::vector<uint32_t> part(blocks, 0);
  int e = launch_count_noncanonical(f.q, f.Ls, d_x, n, d_part, blocks, s);
  if (!e) e = (int)hipMemcpyAsync(part.data(), d_part, blocks * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (!e) e = (int)hipStreamSynchronize(s);
  if (own) (void)hipFree(d_part);
  if (e) return hip_fail(e, "input check");
  for (uint32_t v : part) *bad += v;
  return MOMA_OK;
}

int check_inputs(const FieldRaw& f, const uint32_t* const* d_x, int nx, uint64_t n, hipStream_t s,
                 uint32_t* d_part) {
  for (int i = 0; i < nx; i++) {
    uint64_t bad = 0;
    int rc = count_noncanonical(f, d_x[i], n, s, &bad, d_part);
    if (rc) return rc;
    if (bad)
      return set_error(MOMA_E_ARG, "input " + std::to_string(i) + " holds " + std::to_string(bad) +
                                       " elements >= q (input check on)");
  }
  return MOMA_OK;
}

static int ntt_entry(bool inverse, const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs,
                     const uint32_t* d_in, uint32_t* d_out, void* stream) {
  if (!d_in || !d_out) return set_error(MOMA_E_ARG, "device pointer is NULL");
  std::shared_ptr<NttPlan> p;
  int rc = get_plan(q, omega, n, limbs, &p);
  if (rc) return rc;
  if (input_check_on()) {
    rc = check_inputs(p->fe->f, &d_in, 1, n, (hipStream_t)stream);
    if (rc) return rc;
  }
  return run_plan(*p, inverse, d_in, d_out, (hipStream_t)stream);
}

// ------------------------------------------------------------------ BLAS

// vmul's product variant per compute limb count (MOMA_VMUL_*), set by
// moma_vmul_set_variant or moma_vmul_tune; schoolbook until then
static uint32_t g_vmul_variant[kMaxLimbs + 1];

uint32_t vmul_variant(int L) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_vmul_variant[L];
}

int axpy_alpha(FieldEntry& fe, const uint32_t* alpha, uint32_t limbs, uint32_t* alpha_m) {
  if (!alpha) return set_error(MOMA_E_ARG, "alpha is NULL");
  std::vector<uint32_t> key(alpha, alpha + limbs);
  std::lock_guard<std::mutex> lk(g_mu);
  if (fe.alpha_key != key) {
    HBig A = HBig::from_limbs(alpha, (int)limbs);
    if (HBig::cmp(A, fe.Q) >= 0) return set_error(MOMA_E_ARG, "alpha must be < q");
    HBig am = HBig::mulmod(A, fe.one_m, fe.Q);
    fe.alpha_m.assign(kMaxLimbs, 0);
    am.to_limbs(fe.alpha_m.data(), kMaxLimbs);
    fe.alpha_key = key;
  }
  memcpy(alpha_m, fe.alpha_m.data(), sizeof(uint32_t) * kMaxLimbs);
  return MOMA_OK;
}

static int blas_entry(int op, const uint32_t* q, uint32_t limbs, uint64_t n, const uint32_t* alpha,
                      const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_out, void* stream) {
  std::shared_ptr<FieldEntry> fe;
  int rc = build_field(q, limbs, &fe);
  if (rc) return rc;
  if (n > (1ull << 31)) return set_error(MOMA_E_ARG, "n must be <= 2^31");
  if (n == 0) return MOMA_OK;
  if (!d_a || !d_b || !d_out) return set_error(MOMA_E_ARG, "device pointer is NULL");
  BlasArgs a;
  memset(&a, 0, sizeof(a));
  a.a = d_a;
  a.b = d_b;
  a.out = d_out;
  a.n = n;
  a.ls = (uint32_t)fe->f.Ls;
  if (op == OP_VMUL) a.variant = vmul_variant(fe->f.L);
  if (op == OP_AXPY) {
    int r = axpy_alpha(*fe, alpha, limbs, a.alpha_m);
    if (r) return r;
  }
  hipStream_t s = (hipStream_t)stream;
  if (input_check_on()) {
    const uint32_t* xs[2] = {d_a, d_b};
    rc = check_inputs(fe->f, xs, 2, n, s);
    if (rc) return rc;
  }
  int e = launch_blas(op, fe->f, a, s);
  if (e) return hip_fail(e, "blas launch");
  if (fe->f.Ls > fe->f.L) {
    const uint32_t* ins[2] = {d_a, d_b};
    bool aliased = ins[0] == d_out || ins[1] == d_out;
    if (!aliased) {
      e = launch_zero_planes(d_out, n, fe->f.L, fe->f.Ls, s);
      if (e) return hip_fail(e, "zero planes launch");
    }
  }
  return MOMA_OK;
}

}  // namespace moma

using namespace moma;

extern "C" {

const char* moma_strerror(int code) {
  switch (code) {
    case MOMA_OK: return "MOMA_OK";
    case MOMA_E_ARG: return "MOMA_E_ARG: invalid argument";
    case MOMA_E_MODULUS: return "MOMA_E_MODULUS: invalid modulus";
    case MOMA_E_ROOT: return "MOMA_E_ROOT: omega is not a primitive n-th root of unity";
    case MOMA_E_NOMEM: return "MOMA_E_NOMEM: device allocation failed";
    case MOMA_E_HIP: return "MOMA_E_HIP: HIP runtime error";
    case MOMA_E_UNSUPPORTED: return "MOMA_E_UNSUPPORTED: unsupported request";
  }
  return "unknown error";
}

const char* moma_last_error_detail(void) { return g_detail.c_str(); }

const char* moma_version(void) { return "moma-mi355x 0.1 (gfx950)"; }

int moma_vadd(const uint32_t* q, uint32_t limbs, uint64_t n, const uint32_t* d_a, const uint32_t* d_b,
              uint32_t* d_out, void* stream) {
  return blas_entry(OP_VADD, q, limbs, n, nullptr, d_a, d_b, d_out, stream);
}

int moma_vsub(const uint32_t* q, uint32_t limbs, uint64_t n, const uint32_t* d_a, const uint32_t* d_b,
              uint32_t* d_out, void* stream) {
  return blas_entry(OP_VSUB, q, limbs, n, nullptr, d_a, d_b, d_out, stream);
}

int moma_vmul(const uint32_t* q, uint32_t limbs, uint64_t n, const uint32_t* d_a, const uint32_t* d_b,
              uint32_t* d_out, void* stream) {
  return blas_entry(OP_VMUL, q, limbs, n, nullptr, d_a, d_b, d_out, stream);
}

int moma_vmul_set_variant(const uint32_t* q, uint32_t limbs, uint32_t variant) {
  std::shared_ptr<FieldEntry> fe;
  int rc = build_field(q, limbs, &fe);
  if (rc) return rc;
  if (variant > MOMA_VMUL_KARATSUBA) return set_error(MOMA_E_ARG, "unknown vmul variant");
  if (variant == MOMA_VMUL_KARATSUBA && fe->f.L < 2)
    return set_error(MOMA_E_UNSUPPORTED, "Karatsuba needs at least 2 compute limbs");
  std::lock_guard<std::mutex> lk(g_mu);
  g_vmul_variant[fe->f.L] = variant;
  return MOMA_OK;
}

int moma_vmul_get_variant(const uint32_t* q, uint32_t limbs, uint32_t* variant) {
  if (!variant) return set_error(MOMA_E_ARG, "variant is NULL");
  std::shared_ptr<FieldEntry> fe;
  int rc = build_field(q, limbs, &fe);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  *variant = g_vmul_variant[fe->f.L];
  return MOMA_OK;
}

int moma_vmul_tune(const uint32_t* q, uint32_t limbs, uint64_t n, uint32_t reps, float* us_out, uint32_t* chosen) {
  if (!us_out) return set_error(MOMA_E_ARG, "us_out is NULL");
  std::shared_ptr<FieldEntry> fe;
  int rc = build_field(q, limbs, &fe);
  if (rc) return rc;
  if (n == 0 || n > (1ull << 31)) return set_error(MOMA_E_ARG, "n must be in [1, 2^31]");
  if (reps == 0) reps = 5;
  const int L = fe->f.L;
  const uint32_t nvar = L >= 2 ? 2 : 1;
  // random residues in the caller's storage planes: the kernels' power draw,
  // and with it the clock, depends on the data
  const int planes = std::max(L, fe->f.Ls);
  uint32_t* buf = nullptr;
  const size_t words = (size_t)n * planes;
  if (hipMalloc((void**)&buf, 3 * words * sizeof(uint32_t))) return set_error(MOMA_E_NOMEM, "tune buffers");
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int err = fill_random_residues(fe->f, buf, n, 0x5eed2u, nullptr);
  if (!err) err = fill_random_residues(fe->f, buf + words, n, 0x5eed3u, nullptr);
  if (!err) err = (int)hipStreamCreate(&st);
  if (!err) err = (int)hipEventCreate(&e0);
  if (!err) err = (int)hipEventCreate(&e1);
  float best = 0;
  uint32_t pick = 0;
  for (uint32_t v = 0; v < nvar && !err; v++) {
    BlasArgs a;
    memset(&a, 0, sizeof(a));
    a.a = buf;
    a.b = buf + words;
    a.out = buf + 2 * words;
    a.n = n;
    a.ls = (uint32_t)fe->f.Ls;
    a.variant = v;
    std::vector<float> t;
    for (uint32_t r = 0; r < reps + 1 && !err; r++) {
      err = (int)hipEventRecord(e0, st);
      if (!err) err = launch_blas(OP_VMUL, fe->f, a, st);
      if (!err) err = (int)hipEventRecord(e1, st);
      if (!err) err = (int)hipEventSynchronize(e1);
      float ms = 0;
      if (!err) (void)hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) t.push_back(ms * 1e3f);  // the first run warms up
    }
    if (err) break;
    std::sort(t.begin(), t.end());
    us_out[v] = t[t.size() / 2];
    if (v == 0 || us_out[v] < best) {
      best = us_out[v];
      pick = v;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  (void)hipFree(buf);
  if (err) return hip_fail(err, "vmul tuning");
  if (nvar == 1) us_out[1] = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_vmul_variant[L] = pick;
  }
  if (chosen) *chosen = pick;
  return MOMA_OK;
}

int moma_axpy(const uint32_t* q, uint32_t limbs, uint64_t n, const uint32_t* alpha, const uint32_t* d_x,
              const uint32_t* d_y, uint32_t* d_out, void* stream) {
  return blas_entry(OP_AXPY, q, limbs, n, alpha, d_x, d_y, d_out, stream);
}

int moma_ntt_fwd(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, const uint32_t* d_in,
                 uint32_t* d_out, void* stream) {
  return ntt_entry(false, q, omega, n, limbs, d_in, d_out, stream);
}

int moma_ntt_inv(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, const uint32_t* d_in,
                 uint32_t* d_out, void* stream) {
  return ntt_entry(true, q, omega, n, limbs, d_in, d_out, stream);
}

int moma_ntt_cyclic_mul(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, const uint32_t* d_a,
                        const uint32_t* d_b, uint32_t* d_out, void* stream) {
  if (!d_a || !d_b || !d_out) return set_error(MOMA_E_ARG, "device pointer is NULL");
  std::shared_ptr<NttPlan> p;
  int rc = get_plan(q, omega, n, limbs, &p);
  if (rc) return rc;
  if (input_check_on()) {
    const uint32_t* xs[2] = {d_a, d_b};
    rc = check_inputs(p->fe->f, xs, 2, n, (hipStream_t)stream);
    if (rc) return rc;
  }
  return run_cyclic_mul(*p, d_a, d_b, d_out, (hipStream_t)stream);
}

int moma_check_canonical(const uint32_t* q, uint32_t limbs, uint64_t n, const uint32_t* d_x, uint64_t* bad_out,
                         void* stream) {
  if (!bad_out) return set_error(MOMA_E_ARG, "bad_out is NULL");
  std::shared_ptr<FieldEntry> fe;
  int rc = build_field(q, limbs, &fe);
  if (rc) return rc;
  if (n > (1ull << 31)) return set_error(MOMA_E_ARG, "n must be <= 2^31");
  if (n && !d_x) return set_error(MOMA_E_ARG, "device pointer is NULL");
  return count_noncanonical(fe->f, d_x, n, (hipStream_t)stream, bad_out);
}

static int layout_entry(uint32_t limbs, uint64_t n, const uint32_t* d_src, uint32_t* d_dst, bool to_planar,
                        void* stream) {
  if (limbs < MOMA_MIN_LIMBS || limbs > MOMA_MAX_LIMBS) return set_error(MOMA_E_ARG, "limbs must be in [2, 32]");
  if (n > (1ull << 31)) return set_error(MOMA_E_ARG, "n must be <= 2^31");
  if (n == 0) return MOMA_OK;
  if (!d_src || !d_dst) return set_error(MOMA_E_ARG, "device pointer is NULL");
  if (d_src == d_dst) return set_error(MOMA_E_ARG, "layout conversion cannot run in place");
  int e = launch_layout(d_src, d_dst, n, limbs, to_planar, (hipStream_t)stream);
  if (e) return hip_fail(e, "layout launch");
  return MOMA_OK;
}

int moma_pack_planar(uint32_t limbs, uint64_t n, const uint32_t* d_elems, uint32_t* d_planar, void* stream) {
  return layout_entry(limbs, n, d_elems, d_planar, true, stream);
}

int moma_unpack_planar(uint32_t limbs, uint64_t n, const uint32_t* d_planar, uint32_t* d_elems, void* stream) {
  return layout_entry(limbs, n, d_planar, d_elems, false, stream);
}

int moma_set_input_check(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_check_inputs = on ? 1 : 0;
  return MOMA_OK;
}

int moma_ntt_prepare(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs) {
  std::shared_ptr<NttPlan> p;
  return get_plan(q, omega, n, limbs, &p);
}

int moma_ntt_describe(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, uint32_t* npasses,
                      uint32_t* pass_stages, uint32_t max_passes, uint32_t* compute_limbs) {
  if (!npasses) return set_error(MOMA_E_ARG, "npasses is NULL");
  std::shared_ptr<NttPlan> p;
  int rc = get_plan(q, omega, n, limbs, &p);
  if (rc) return rc;
  *npasses = (uint32_t)p->passes.size();
  if (pass_stages)
    for (uint32_t i = 0; i < max_passes && i < p->passes.size(); i++) pass_stages[i] = p->passes[i].k;
  if (compute_limbs) *compute_limbs = (uint32_t)p->fe->f.L;
  return MOMA_OK;
}

int moma_ntt_set_schedule(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs,
                          const moma_ntt_schedule_t* sched) {
  std::shared_ptr<NttPlan> p;
  int rc = get_plan(q, omega, n, limbs, &p);
  if (rc) return rc;
  NttSchedule s = sched ? NttSchedule{sched->tile_log, sched->col_log, sched->threads, sched->radix_log,
                                      sched->mul_variant}
                        : initial_schedule(p->fe->f.L, p->logn, p->fe->f.fw);
  std::vector<NttPass> ps;
  rc = plan_passes(p->fe->f.L, p->logn, s, &ps, p->fe->f.fw);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(p->mu);
  p->sched = s;
  p->passes = ps;
  return MOMA_OK;
}

int moma_ntt_get_schedule(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs,
                          moma_ntt_schedule_t* sched) {
  if (!sched) return set_error(MOMA_E_ARG, "sched is NULL");
  std::shared_ptr<NttPlan> p;
  int rc = get_plan(q, omega, n, limbs, &p);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(p->mu);
  sched->tile_log = p->sched.tile_log;
  sched->col_log = p->sched.col_log;
  sched->threads = p->sched.threads;
  sched->radix_log = p->sched.radix_log;
  sched->mul_variant = p->sched.kara;
  return MOMA_OK;
}

int moma_ntt_default_schedule(uint32_t limbs_compute, uint32_t log2_n, moma_ntt_schedule_t* sched) {
  if (!sched) return set_error(MOMA_E_ARG, "sched is NULL");
  if (limbs_compute < 1 || limbs_compute > (uint32_t)kMaxLimbs || log2_n < 1 || log2_n > MOMA_MAX_LOG_N)
    return set_error(MOMA_E_ARG, "limbs or log2_n out of range");
  NttSchedule s = default_schedule((int)limbs_compute, log2_n);
  *sched = {s.tile_log, s.col_log, s.threads, s.radix_log, s.kara};
  return MOMA_OK;
}

void moma_shutdown(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_plans.clear();
  g_fields.clear();
}

}  // extern "C"
