/*
 * moma.h - C ABI of the MI355X (gfx950) multi-word modular arithmetic library.
 *
 * The library computes, exactly, over a prime field Z_q whose elements are
 * split into 32-bit machine words ("limbs"):
 *   - the ring operations of the paper's Section 2.1 applied elementwise to
 *     vectors (vadd, vsub, vmul) and axpy y = a*x + y (Section 2.3);
 *   - the forward number theoretic transform of Eq. (ntt),
 *     y(k) = sum_j x(j) w^{jk} mod q, and its inverse
 *     x(j) = n^{-1} sum_k y(k) w^{-jk} mod q.
 * Every output is the unique canonical residue in [0, q).
 *
 * Data layout
 *   Scalars (q, omega, alpha) are HOST pointers to `limbs` little-endian
 *   32-bit words (word 0 least significant).  The paper writes digits most
 *   significant first (Eq. (def_mp)); only the storage order differs.
 *   Vectors are DEVICE pointers in limb-planar layout: word j of element i is
 *   at index j*n + i (so a wavefront reads 64 consecutive words per limb).
 *   Inputs must be canonical (each element < q); words of limbs above the
 *   top limb of q must therefore be zero.  Non-canonical inputs give
 *   undefined (but memory-safe) results; the paper assumes reduced operands
 *   throughout (Section 2.1).  The input check below finds them.
 *
 * Preconditions checked on the host before anything is enqueued
 *   2 <= limbs <= 32; q odd, q >= 3, bitlen(q) <= 32*limbs.  The paper's
 *   moduli are four bits short of the class width (Section 5.2), which
 *   leaves headroom for lazy reduction and Barrett's pre-scaled modulus; a
 *   modulus within 4 bits of the storage width ("full width", up to 1024
 *   bits in 32 limbs) computes in the same limbs with canonical operands and
 *   Montgomery products that carry out of the top limb (Section 5.2 names
 *   Montgomery multiplication for such moduli): vmul then takes two
 *   Montgomery products (the product variant does not apply), and the
 *   transforms use radix-2 and radix-4 units only;
 *   n a power of two, 2 <= n <= 2^26 (BLAS: any n >= 0);
 *   omega of multiplicative order exactly n (omega^{n/2} == q - 1), which
 *   also implies n | q - 1 for prime q.  Primality of q is the caller's
 *   contract.
 *
 * Ownership and concurrency
 *   The caller owns device buffers and streams.  The library owns cached
 *   plans (twiddle tables, constants, scratch) until moma_shutdown().
 *   In-place operation is allowed (d_out == d_in, d_out == d_a/d_b,
 *   d_out == d_y); partial overlap is undefined.  Work is enqueued on
 *   `stream` (a hipStream_t passed as void*; NULL is the default stream) and
 *   returns without synchronising.  Plan creation may allocate device memory
 *   and synchronise once.  The plan cache is thread safe.  A plan's scratch
 *   (used by in-place multi-pass transforms and by the cyclic product) is one
 *   buffer per plan: such calls for the same plan on different streams must
 *   not run at the same time.
 *
 * Errors
 *   Functions return MOMA_OK (0) or a negative code; moma_strerror() names
 *   it and moma_last_error_detail() gives the last failure's text.
 */
#ifndef MOMA_H
#define MOMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MOMA_OK = 0,
  MOMA_E_ARG = -1,         /* null pointer, bad size, bad limb count      */
  MOMA_E_MODULUS = -2,     /* q even, too small, or too wide for `limbs`  */
  MOMA_E_ROOT = -3,        /* omega does not have order exactly n         */
  MOMA_E_NOMEM = -4,       /* device allocation failed                    */
  MOMA_E_HIP = -5,         /* a HIP runtime call failed                   */
  MOMA_E_UNSUPPORTED = -6  /* valid request the library cannot run         */
};

#define MOMA_MIN_LIMBS 2
#define MOMA_MAX_LIMBS 32
#define MOMA_MAX_LOG_N 26

/* Name of an error code (static string). */
const char* moma_strerror(int code);
/* Text describing the most recent failure on the calling thread. */
const char* moma_last_error_detail(void);
/* Library version string. */
const char* moma_version(void);

/*
 * Input check (the canonical-input precondition of Section 2.1: every operand
 * is already reduced mod q).
 *   moma_check_canonical: *bad_out = the number of elements of the
 *     limb-planar vector d_x (`limbs` planes of n words, n <= 2^31) whose
 *     value is >= q.  Runs a counting kernel on `stream`, then waits for that
 *     stream; allocates and frees a small device buffer per call.  Errors:
 *     MOMA_E_ARG (NULL pointer, n too large), the modulus errors of the other
 *     calls, MOMA_E_NOMEM, MOMA_E_HIP.
 *   moma_set_input_check: on != 0 makes every BLAS, transform, cyclic product
 *     and batch run count its inputs first and fail with MOMA_E_ARG, before
 *     enqueueing anything, when an input holds a non-canonical element.  Each
 *     checked call then waits for its stream, so this is a debugging mode.
 *     The environment variable MOMA_CHECK_INPUTS=1 turns it on at start-up;
 *     the default is off.
 */
int moma_check_canonical(const uint32_t* q, uint32_t limbs, uint64_t n, const uint32_t* d_x, uint64_t* bad_out,
                         void* stream);
int moma_set_input_check(int on);


/*
 * Layout conversion on the device, for data held as an array of multi-word
 * integers (element i's limb j at d_elems[i * limbs + j], little-endian limbs).
 *   moma_pack_planar:   d_planar[j * n + i] = d_elems[i * limbs + j]
 *   moma_unpack_planar: d_elems[i * limbs + j] = d_planar[j * n + i]
 * 2 <= limbs <= 32, n <= 2^31 (0 is a no-op).  Asynchronous on `stream`.  The
 * two buffers must not overlap (the same pointer is MOMA_E_ARG).  Values are
 * copied as words; no reduction mod q happens.
 */
int moma_pack_planar(uint32_t limbs, uint64_t n, const uint32_t* d_elems, uint32_t* d_planar, void* stream);
int moma_unpack_planar(uint32_t limbs, uint64_t n, const uint32_t* d_planar, uint32_t* d_elems, void* stream);

/*
 * Elementwise modular BLAS (paper Section 2.3; ring operations of Section 2.1).
 *   moma_vadd: out_i = (a_i + b_i) mod q
 *   moma_vsub: out_i = (a_i - b_i) mod q
 *   moma_vmul: out_i = (a_i * b_i) mod q      (Barrett reduction, Eq. (barrett))
 *   moma_axpy: out_i = (alpha * x_i + y_i) mod q   (Montgomery multiply by alpha)
 * n is the element count (0 is a no-op).  Device arrays are limb-planar with
 * `limbs` planes of n words.  alpha is a host scalar in [0, q).
 */
int moma_vadd(const uint32_t* q, uint32_t limbs, uint64_t n, const uint32_t* d_a, const uint32_t* d_b,
              uint32_t* d_out, void* stream);
int moma_vsub(const uint32_t* q, uint32_t limbs, uint64_t n, const uint32_t* d_a, const uint32_t* d_b,
              uint32_t* d_out, void* stream);
int moma_vmul(const uint32_t* q, uint32_t limbs, uint64_t n, const uint32_t* d_a, const uint32_t* d_b,
              uint32_t* d_out, void* stream);
int moma_axpy(const uint32_t* q, uint32_t limbs, uint64_t n, const uint32_t* alpha, const uint32_t* d_x,
              const uint32_t* d_y, uint32_t* d_out, void* stream);

/*
 * vmul's word-product variant, per compute limb count (Eq. (mulk)): the two
 * full L x L products of the Barrett multiply by schoolbook product scanning
 * (L^2 word products each) or by one level of Karatsuba (3 ceil(L/2)^2 plus
 * the additions).  Both give the same result, bit for bit; which is faster
 * depends on the width, so it is an autotuner choice.
 *   moma_vmul_set_variant / moma_vmul_get_variant: the variant used by later
 *     moma_vmul calls whose modulus has the same compute limb count
 *     (MOMA_E_UNSUPPORTED for Karatsuba below 2 compute limbs);
 *   moma_vmul_tune: times each variant on n pseudo-random residues (median
 *     of reps runs after one warm-up; reps 0 means 5), installs the faster, writes the
 *     two times in microseconds to us_out[2] (us_out[1] = 0 when only
 *     schoolbook applies) and the choice to *chosen (may be NULL).  Allocates
 *     3 n L words for the duration of the call and synchronises.
 * The setting is process-wide and survives moma_shutdown.
 */
enum moma_vmul_variant { MOMA_VMUL_SCHOOLBOOK = 0, MOMA_VMUL_KARATSUBA = 1 };
int moma_vmul_set_variant(const uint32_t* q, uint32_t limbs, uint32_t variant);
int moma_vmul_get_variant(const uint32_t* q, uint32_t limbs, uint32_t* variant);
int moma_vmul_tune(const uint32_t* q, uint32_t limbs, uint64_t n, uint32_t reps, float* us_out, uint32_t* chosen);

/*
 * Number theoretic transform, Eq. (ntt): natural order in, natural order out.
 *   moma_ntt_fwd: d_out[k] = sum_j d_in[j] * omega^{jk} mod q
 *   moma_ntt_inv: d_out[j] = n^{-1} sum_k d_in[k] * omega^{-jk} mod q
 * `omega` is the FORWARD primitive n-th root in both calls; the inverse uses
 * omega^{-1} and n^{-1} itself.  A butterfly is one modular add, one modular
 * subtract and one modular multiply (Section 5.3); a transform performs
 * (n/2) log2 n of them.  The first call for a given (q, omega, n, limbs)
 * builds a plan (twiddle tables on the device) and synchronises once.
 */
int moma_ntt_fwd(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, const uint32_t* d_in,
                 uint32_t* d_out, void* stream);
int moma_ntt_inv(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, const uint32_t* d_in,
                 uint32_t* d_out, void* stream);

/*
 * Cyclic product of two polynomials of n coefficients (the use of the NTT in
 * Section 2.3, via the convolution theorem):
 *   d_out[k] = sum over i + j == k (mod n) of d_a[i] * d_b[j]  mod q,
 * that is a * b mod (x^n - 1).  The full product of two polynomials of
 * degree < n/2 (Section 2.3) is this product of their zero-padded
 * coefficient vectors.  Same arguments and preconditions as
 * moma_ntt_fwd; omega is a primitive n-th root (any one gives the same
 * result).  Runs fwd(a), fwd(b) and the inverse transform, whose first pass
 * multiplies the two spectra pointwise as it loads them: no separate
 * pointwise kernel and no extra pass over memory.  d_out may equal d_a or
 * d_b.  The first call for a plan allocates 2 * n * L words of spectra
 * scratch (L = compute limbs), kept with the plan.
 */
int moma_ntt_cyclic_mul(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, const uint32_t* d_a,
                        const uint32_t* d_b, uint32_t* d_out, void* stream);

/*
 * The cyclic product above for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result (bit for bit) and preconditions as
 * moma_ntt_cyclic_mul, and the same kernels; it calls no hipMalloc, hipFree or
 * other allocating routine.  Differences:
 *   - the plan for (q, omega, n, limbs) on the current device must already
 *     exist (moma_ntt_prepare, or any earlier call that built it); otherwise
 *     MOMA_E_ARG and nothing is enqueued;
 *   - the two spectra, 2 * n * L words (L = compute limbs), live in a fixed
 *     library-wide device array of MOMA_NOALLOC_SCRATCH_WORDS 32-bit words
 *     (64 MiB) that each GPU holds until the process ends; a request needing
 *     more is MOMA_E_ARG (at 256 bits, L = 8, n may be up to 2^20).
 * Every call on one GPU shares that array and leaves its contents behind:
 * calls that overlap on one GPU (other streams, other host threads) race and
 * give undefined results.  With the input check on, the per-workgroup counts
 * also use the array, and the call waits for its stream before enqueueing.
 */
#define MOMA_NOALLOC_SCRATCH_WORDS (1u << 24)
int moma_ntt_cyclic_mul_noalloc(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs,
                                const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_out, void* stream);

/*
 * Build (or look up) the plan for (q, omega, n, limbs) without running a
 * transform, so timed loops exclude plan creation.  Returns MOMA_OK or an
 * error code for invalid parameters.
 */
int moma_ntt_prepare(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs);

/*
 * Describe the schedule of the plan for (q, omega, n, limbs): the number of
 * kernel launches (passes) per transform, the stages each pass runs, and the
 * compute limb count.  pass_stages must hold max_passes entries; entries past
 * *npasses are left untouched.  Builds the plan if needed.
 */
int moma_ntt_describe(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, uint32_t* npasses,
                      uint32_t* pass_stages, uint32_t max_passes, uint32_t* compute_limbs);

/*
 * Launch shape of a transform plan (the knobs the autotuner searches):
 *   tile_log  - log2 of the elements one workgroup keeps in LDS (LDS bytes =
 *               4 * compute_limbs * 2^tile_log, at most 160 KiB);
 *   col_log   - log2 of the coalesced groups per tile in multi-pass plans;
 *               passes run tile_log - col_log stages each;
 *   threads   - threads per workgroup, a multiple of 64 in [64, 1024];
 *   radix_log - stages each thread runs in registers per LDS round trip
 *               (radix 2, 4, 8 or 16; radix 16 up to 2 limbs, radix 8 up to 5,
 *               radix 4 up to 16, also for a full-width modulus);
 *   mul_variant - how the butterfly's twiddle multiply forms its word
 *               products (Eq. (mulk)): MOMA_NTT_MUL_SCHOOLBOOK, or
 *               MOMA_NTT_MUL_KARATSUBA (one level of Karatsuba on the
 *               multiply's digits; radix 2 only, 2 to 24 compute limbs, not
 *               for full-width moduli; batches run the schoolbook form).
 * Every schedule computes the same result; only speed differs.
 */
enum moma_ntt_mul_variant { MOMA_NTT_MUL_SCHOOLBOOK = 0, MOMA_NTT_MUL_KARATSUBA = 1 };
typedef struct moma_ntt_schedule {
  uint32_t tile_log;
  uint32_t col_log;
  uint32_t threads;
  uint32_t radix_log;
  uint32_t mul_variant;
} moma_ntt_schedule_t;

/* Set the schedule of the plan for (q, omega, n, limbs); NULL restores the
 * plan's initial choice: the timing database's fastest schedule for this
 * (compute limbs, n) if it has one, else the loaded cost model's top-ranked
 * schedule, else the fixed rule of moma_ntt_default_schedule.  New plans
 * start with that same choice.  MOMA_E_UNSUPPORTED if the shape cannot run
 * this size, MOMA_E_ARG for malformed values.  Affects calls enqueued
 * afterwards. */
int moma_ntt_set_schedule(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs,
                          const moma_ntt_schedule_t* sched);
/* The fixed rule a new plan falls back to when neither the timing database
 * nor a loaded cost model gives it a schedule. */
int moma_ntt_default_schedule(uint32_t limbs_compute, uint32_t log2_n, moma_ntt_schedule_t* sched);
/* Read the schedule the plan currently uses. */
int moma_ntt_get_schedule(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs,
                          moma_ntt_schedule_t* sched);

/*
 * Autotuner.  For one (q, omega, n, limbs) plan: enumerate every launch shape
 * the kernels can run (moma_ntt_candidates), time each with HIP events
 * (`warmup` untimed runs, then the median of `reps` repetitions, each long
 * enough to dwarf event resolution), install the fastest in the plan and
 * append every measurement to the process's timing database.  With top_k > 0
 * and a cost model loaded, only the model's top_k shapes are timed (without a
 * model that returns MOMA_E_UNSUPPORTED).  max_candidates > 0 truncates the
 * enumeration.  Ties go to the earlier candidate.  The timed input is n
 * pseudo-random residues (the clock under load depends on the data, so zeros
 * would time optimistically).  Allocates two scratch transforms and
 * synchronises.
 */
typedef struct moma_tune_opts {
  uint32_t reps;            /* timed repetitions per shape (median), default 5 */
  uint32_t warmup;          /* untimed runs per shape, default 2 */
  uint32_t top_k;           /* 0: exhaustive; else time the cost model's top_k */
  uint32_t max_candidates;  /* 0: no limit */
} moma_tune_opts_t;

typedef struct moma_tune_result {
  moma_ntt_schedule_t best;
  float best_us;            /* median microseconds of one forward transform */
  uint32_t timed;           /* shapes timed */
  uint32_t feasible;        /* shapes enumerated */
} moma_tune_result_t;

int moma_ntt_tune(const uint32_t* q, const uint32_t* omega, uint64_t n, uint32_t limbs, const moma_tune_opts_t* opts,
                  moma_tune_result_t* result);
/* The feasible shapes for a compute limb count and size, in the tuner's order
 * (the schoolbook shapes, then the radix-2 ones again with the Karatsuba
 * multiply where it applies).  Writes at most `max` entries to out (may be
 * NULL) and the total to *count. */
int moma_ntt_candidates(uint32_t limbs_compute, uint32_t log2_n, moma_ntt_schedule_t* out, uint32_t max,
                        uint32_t* count);

/* Timing database: one row per timed shape.  Plans created after a load start
 * from the fastest recorded shape for their (compute limbs, log2 n) on the
 * same device name.  CSV: device,limbs,log2_n,tile_log,col_log,threads,
 * radix_log,us,reps,mul_variant (rows without the last column load as
 * schoolbook).  Tuning a full-width plan records nothing. */
typedef struct moma_tune_row {
  uint32_t limbs;           /* compute limbs */
  uint32_t log2_n;
  moma_ntt_schedule_t sched;
  float us;
  uint32_t reps;
} moma_tune_row_t;
uint32_t moma_tune_db_count(void);
int moma_tune_db_get(uint32_t index, moma_tune_row_t* row);
void moma_tune_db_clear(void);
int moma_tune_db_save(const char* path);
int moma_tune_db_load(const char* path);

/*
 * Learned cost model: an FP32 perceptron 7 -> 64 -> 64 -> 1 (ReLU) predicting
 * log(microseconds) of a schedule from seven features (moma_costmodel_features:
 * log2 n, compute limbs, log2 radix, stages fused per pass, log2 threads,
 * log2 LDS bytes, Karatsuba multiply 0/1), trained on the GPU by the library's own kernels with Adam
 * on mean squared error.  Features and targets are z-scored with the training
 * set's statistics, which are saved with the weights.  While a model is
 * loaded (or trained), new plans whose shape the timing database does not
 * cover start from the model's top-ranked schedule (one prediction per
 * (compute limbs, log2 n), cached until the model changes).
 */
typedef struct moma_train_opts {
  uint32_t epochs;          /* default 200 */
  uint32_t batch;           /* minibatch rows, default 256 */
  float lr;                 /* Adam step size, default 3e-3 */
  uint64_t seed;            /* initial weights and minibatch order (SplitMix64) */
} moma_train_opts_t;

#define MOMA_COSTMODEL_FEATURES 7
int moma_costmodel_features(uint32_t limbs_compute, uint32_t log2_n, const moma_ntt_schedule_t* sched, float* out7);
/* Train from host arrays features[rows][7] and targets log_us[rows]; replaces the
 * current model.  *final_mse (may be NULL) is the training-set mean squared
 * error in (log us)^2. */
int moma_costmodel_train(const float* features, const float* log_us, uint32_t rows, const moma_train_opts_t* opts,
                         float* final_mse);
/* Predict log(us) for host features[rows][7]. */
int moma_costmodel_predict(const float* features, uint32_t rows, float* log_us);
int moma_costmodel_save(const char* path);
int moma_costmodel_load(const char* path);
void moma_costmodel_clear(void);

/* The network's kernels on raw device arrays (features already normalised),
 * for checking them against a reference: parameters are W1[64][7], b1[64],
 * W2[64][64], b2[64], W3[64], b3 (moma_mlp_nparams() floats).
 *   forward: y[r] for rows x[r][7];
 *   grad:    gradient of mean((y - t)^2) into grad[nparams] and the loss into
 *            *d_loss; allocates a workspace and synchronises `stream`;
 *   adam:    one bias-corrected Adam step (step >= 1) on params, m, v. */
uint32_t moma_mlp_nparams(void);
int moma_mlp_forward(const float* d_params, const float* d_x, uint32_t rows, float* d_y, void* stream);
int moma_mlp_grad(const float* d_params, const float* d_x, const float* d_t, uint32_t rows, float* d_grad,
                  float* d_loss, void* stream);
int moma_mlp_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t step, float lr, float beta1,
                  float beta2, float eps, void* stream);

/*
 * Batched transforms and BLAS calls (the paper batches kernels to fill the
 * GPU, Section 5.1): many NTTs and vector operations of different sizes,
 * limb counts and moduli run as one hipGraph launch.  A job is one call of
 * the kind moma_ntt_fwd, moma_ntt_inv, moma_ntt_cyclic_mul, moma_vadd,
 * moma_vsub, moma_vmul or moma_axpy runs, with the same argument meanings and
 * preconditions; transform plans are built (and shared with identical jobs)
 * by moma_batch_create, and a cyclic product gets 2 * n * L words of spectra
 * scratch of its own, owned by the batch.  The batch keeps the job buffers'
 * addresses: they must stay allocated, and are read and written by every
 * moma_batch_run.  Each job's output equals what the plain call with the same
 * arguments produces, bit for bit.  Jobs must not overlap one another's
 * output buffers, and no job may read another job's output.
 * Field use by kind:
 *   transforms: omega, n (a power of two), d_in (cyclic product: a), d_in2
 *     (cyclic product: b), d_out;
 *   BLAS: n (any, 0 is a no-op), d_in = a (axpy: x), d_in2 = b (axpy: y),
 *     d_out, and for axpy the host scalar alpha; omega is ignored.  vmul
 *     uses the product variant set for its compute limb count at creation.
 */
enum moma_job_kind {
  MOMA_JOB_FORWARD = 0,
  MOMA_JOB_INVERSE = 1,
  MOMA_JOB_CYCLIC_MUL = 2,
  MOMA_JOB_VADD = 3,
  MOMA_JOB_VSUB = 4,
  MOMA_JOB_VMUL = 5,
  MOMA_JOB_AXPY = 6
};

typedef struct moma_ntt_job {
  const uint32_t* q;      /* host, limbs words */
  const uint32_t* omega;  /* host, limbs words: forward primitive n-th root (transforms) */
  uint64_t n;
  uint32_t limbs;
  uint32_t kind;          /* enum moma_job_kind */
  const uint32_t* d_in;   /* device, limb-planar (cyclic product: a; BLAS: a or x) */
  uint32_t* d_out;        /* device, limb-planar; may equal d_in (or d_in2) */
  const uint32_t* d_in2;  /* device, limb-planar: b of a cyclic product or BLAS op (axpy: y) */
  const uint32_t* alpha;  /* host, limbs words: axpy's scalar; ignored otherwise */
} moma_ntt_job_t;

typedef struct moma_batch* moma_batch_t;

/* Validate the jobs, build their plans and capture the batch into a graph.
 * Synchronises the device.  *out is NULL on failure. */
int moma_batch_create(const moma_ntt_job_t* jobs, uint32_t njobs, moma_batch_t* out);
/* Enqueue the whole batch on `stream` as one graph launch. */
int moma_batch_run(moma_batch_t batch, void* stream);
/* Kernel launches inside the graph and work items (tiles) they cover. */
int moma_batch_info(moma_batch_t batch, uint32_t* launches, uint64_t* items);
/* Release the graph and the batch's tables (plans stay cached). */
int moma_batch_destroy(moma_batch_t batch);

/*
 * Measured issue rates and bandwidths (measurement support, not a step of the
 * method).  The roofline of the integer kernels prices a modular multiply as
 * its word products and carry steps (Section 2.2: a 2w-bit product from
 * w-bit products, additions with carry); on gfx950 a word product with its
 * 64-bit accumulation is one v_mad_u64_u32 and a carry step one
 * v_addc_co_u32.  moma_measure_peaks times long runs of independent chains of
 * each instruction over every SIMD of the device (latency hidden, only issue
 * throughput counts) and two streaming kernels over buffers of hbm_bytes
 * each (0 means 1 GiB; at most 16 GiB): rates in lane operations per second
 * (for add_co_addc_u32 and mad_addc_u32 both instructions of a pair count)
 * and bytes per second (read plus written).  Allocates three buffers of
 * hbm_bytes for the duration of the call and synchronises `stream`.  Errors:
 * MOMA_E_ARG (NULL out, hbm_bytes out of range), MOMA_E_NOMEM, MOMA_E_HIP.
 */
typedef struct moma_peak_rates {
  double add_u32;          /* v_add_u32: the full-rate reference */
  double add_co_addc_u32;  /* v_add_co_u32 followed by v_addc_co_u32 */
  double mad_u64_u32;      /* v_mad_u64_u32: 32x32-bit product plus 64-bit addend */
  double mad_addc_u32;     /* v_mad_u64_u32 whose carry-out feeds a v_addc_co_u32 */
  double mul_lo_u32;       /* v_mul_lo_u32 */
  double mul_hi_u32;       /* v_mul_hi_u32 */
  double hbm_copy;         /* one read per write, bytes/s */
  double hbm_triad;        /* two reads per write, bytes/s */
  uint32_t compute_units;
} moma_peak_rates_t;
int moma_measure_peaks(moma_peak_rates_t* out, uint64_t hbm_bytes, void* stream);

/* Free every cached plan and device table.  Safe to call more than once. */
void moma_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* MOMA_H */
