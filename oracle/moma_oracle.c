/*
 * Plain CPU oracle for multi-word modular arithmetic (MoMA), the modular BLAS
 * operations and the number theoretic transform.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU library.
 *
 * Every result here is computed from its plain definition:
 *   - ring operations in Z_q (paper Section 2.1, first displayed equation):
 *     c = a + b mod q, c = a - b mod q, c = a*b mod q, each reduced by a true
 *     long division (Knuth, TAOCP vol. 2, Section 4.3.1, Algorithm D), i.e.
 *     the floor definition of Eq. (barrett) c = ab - floor(ab/q) q, with no
 *     Barrett or Montgomery shortcut;
 *   - schoolbook multi-digit add / sub / multiply (paper Section 2.2);
 *   - the NTT y(k) = sum_j x(j) w^{jk} mod q (paper Eq. (ntt)), evaluated
 *     directly, O(n^2) for whole vectors or O(n) per sampled output;
 *   - the inverse x(j) = n^{-1} sum_k y(k) w^{-jk} mod q (the paper does not
 *     state the inverse; this is the standard inverse of Eq. (ntt));
 *   - a textbook iterative radix-2 Cooley-Tukey transform (CLRS ch. 30) as a
 *     faster whole-vector oracle, itself pinned against the direct sum;
 *   - axpy y = a x + y (paper Section 2.3) elementwise mod q.
 *
 * Numbers are little-endian arrays of 32-bit limbs (limb 0 least significant);
 * vectors are element-major: limb j of element i at x[i*L + j].  The paper
 * writes digits most-significant first; only the storage order differs.
 * Parallelism: OpenMP over independent outputs only.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef uint32_t limb_t;
typedef uint64_t dlimb_t;

#define MAXL 64           /* max limbs of a residue handled by the oracle   */
#define WORK (4 * MAXL + 4)

/* how often the add-back branch of Algorithm D ran (lets tests show that the
   rare branch is exercised by their inputs) */
static int64_t g_addbacks = 0;

/* ------------------------------------------------------------ bigint basics */

/* number of significant limbs (0 for zero) */
static int big_len(const limb_t *a, int n) {
  while (n > 0 && a[n - 1] == 0) n--;
  return n;
}

/* compare a and b of n limbs: -1, 0, 1 */
static int big_cmp(const limb_t *a, const limb_t *b, int n) {
  for (int i = n - 1; i >= 0; i--) {
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  }
  return 0;
}

/* r = a + b over n limbs, returns the carry out (Section 2.2 addition) */
static limb_t big_add(limb_t *r, const limb_t *a, const limb_t *b, int n) {
  dlimb_t c = 0;
  for (int i = 0; i < n; i++) {
    c += (dlimb_t)a[i] + b[i];
    r[i] = (limb_t)c;
    c >>= 32;
  }
  return (limb_t)c;
}

/* r = a - b over n limbs, returns the borrow out (Section 2.2 subtraction) */
static limb_t big_sub(limb_t *r, const limb_t *a, const limb_t *b, int n) {
  limb_t br = 0;
  for (int i = 0; i < n; i++) {
    dlimb_t d = (dlimb_t)a[i] - b[i] - br;
    r[i] = (limb_t)d;
    br = (limb_t)((d >> 32) & 1);
  }
  return br;
}

/* r[0..na+nb) = a * b, schoolbook (Eq. (muls) applied digit by digit) */
static void big_mul(limb_t *r, const limb_t *a, int na, const limb_t *b, int nb) {
  memset(r, 0, sizeof(limb_t) * (size_t)(na + nb));
  for (int i = 0; i < na; i++) {
    dlimb_t c = 0;
    for (int j = 0; j < nb; j++) {
      c += (dlimb_t)a[i] * b[j] + r[i + j];
      r[i + j] = (limb_t)c;
      c >>= 32;
    }
    r[i + nb] = (limb_t)c;
  }
}

/*
 * rem[0..n) = u mod v, u of m limbs, v of n limbs with v[n-1] != 0, m >= n.
 * Knuth Algorithm D: normalise so the divisor's top bit is set, then produce
 * one quotient digit per step from the top two remainder limbs over the top
 * divisor limb (an estimate that is never too small and at most two too
 * large), multiply-subtract, and add the divisor back while the partial
 * remainder is negative.
 */
static void big_rem(limb_t *rem, const limb_t *u, int m, const limb_t *v, int n) {
  limb_t un[WORK], vn[MAXL + 1];
  if (n == 1) {
    dlimb_t r = 0;
    for (int i = m - 1; i >= 0; i--) r = ((r << 32) | u[i]) % v[0];
    rem[0] = (limb_t)r;
    return;
  }
  /* D1: normalise, shifting divisor and dividend left by s bits */
  int s = __builtin_clz(v[n - 1]);
  for (int i = n - 1; i > 0; i--) vn[i] = (v[i] << s) | (s ? (v[i - 1] >> (32 - s)) : 0);
  vn[0] = v[0] << s;
  un[m] = s ? (u[m - 1] >> (32 - s)) : 0;
  for (int i = m - 1; i > 0; i--) un[i] = (u[i] << s) | (s ? (u[i - 1] >> (32 - s)) : 0);
  un[0] = u[0] << s;
  for (int j = m - n; j >= 0; j--) {
    /* D3: estimate; with vn[n-1] >= 2^31 it is never below the true digit
       and at most two above it (TAOCP 4.3.1, Theorems A and B) */
    dlimb_t num = ((dlimb_t)un[j + n] << 32) | un[j + n - 1];
    dlimb_t qhat = num / vn[n - 1];
    if (qhat > 0xFFFFFFFFull) qhat = 0xFFFFFFFFull;
    /* D4: un[j..j+n] -= qhat * vn, tracking the signed top word */
    int64_t k = 0;
    for (int i = 0; i < n; i++) {
      dlimb_t p = qhat * vn[i];
      int64_t t = (int64_t)un[i + j] - k - (int64_t)(p & 0xFFFFFFFFull);
      un[i + j] = (limb_t)t;
      k = (int64_t)(p >> 32) - (t >> 32);
    }
    int64_t top = (int64_t)un[j + n] - k;
    /* D6: add the divisor back while the partial remainder is negative */
    while (top < 0) {
      __atomic_fetch_add(&g_addbacks, 1, __ATOMIC_RELAXED);
      dlimb_t c = 0;
      for (int i = 0; i < n; i++) {
        c += (dlimb_t)un[i + j] + vn[i];
        un[i + j] = (limb_t)c;
        c >>= 32;
      }
      top += (int64_t)c;
    }
    un[j + n] = (limb_t)top; /* the partial remainder is below vn: this is 0 */
  }
  /* D8: unnormalise the remainder */
  for (int i = 0; i < n; i++) {
    limb_t hi = un[i + 1];
    rem[i] = s ? ((un[i] >> s) | (hi << (32 - s))) : un[i];
  }
}

/* out[0..L) = x mod q, x of m limbs, q of L limbs (q != 0) */
static void reduce(limb_t *out, const limb_t *x, int m, const limb_t *q, int L) {
  int nq = big_len(q, L);
  int nx = big_len(x, m);
  memset(out, 0, sizeof(limb_t) * (size_t)L);
  if (nx < nq || (nx == nq && big_cmp(x, q, nq) < 0)) {
    memcpy(out, x, sizeof(limb_t) * (size_t)nx);
    return;
  }
  big_rem(out, x, nx, q, nq);
}

/* ----------------------------------------------------- Z_q ring operations */

/* c = a + b mod q: full (L+1)-limb sum, then reduction by division */
static void mod_add(limb_t *c, const limb_t *a, const limb_t *b, const limb_t *q, int L) {
  limb_t s[MAXL + 1];
  s[L] = big_add(s, a, b, L);
  reduce(c, s, L + 1, q, L);
}

/* c = a - b mod q: a + (q - b) is non-negative for a, b in [0, q); reduce it */
static void mod_sub(limb_t *c, const limb_t *a, const limb_t *b, const limb_t *q, int L) {
  limb_t t[MAXL + 1], s[MAXL + 1];
  big_sub(t, q, b, L);
  s[L] = big_add(s, a, t, L);
  reduce(c, s, L + 1, q, L);
}

/* c = a * b mod q: 2L-limb schoolbook product, then reduction by division */
static void mod_mul(limb_t *c, const limb_t *a, const limb_t *b, const limb_t *q, int L) {
  limb_t p[2 * MAXL];
  big_mul(p, a, L, b, L);
  reduce(c, p, 2 * L, q, L);
}

/* c = a^e mod q, e of ne limbs, left-to-right square and multiply */
static void mod_pow(limb_t *c, const limb_t *a, const limb_t *e, int ne, const limb_t *q, int L) {
  limb_t r[MAXL], t[MAXL];
  memset(r, 0, sizeof(limb_t) * (size_t)L);
  r[0] = 1;
  reduce(t, r, L, q, L); /* 1 mod q (q could be 1 in a degenerate test) */
  memcpy(r, t, sizeof(limb_t) * (size_t)L);
  for (int i = ne - 1; i >= 0; i--) {
    for (int bit = 31; bit >= 0; bit--) {
      mod_mul(t, r, r, q, L);
      memcpy(r, t, sizeof(limb_t) * (size_t)L);
      if ((e[i] >> bit) & 1) {
        mod_mul(t, r, a, q, L);
        memcpy(r, t, sizeof(limb_t) * (size_t)L);
      }
    }
  }
  memcpy(c, r, sizeof(limb_t) * (size_t)L);
}

/* c = a^{-1} mod q for prime q (Fermat: a^{q-2}) */
static void mod_inv(limb_t *c, const limb_t *a, const limb_t *q, int L) {
  limb_t e[MAXL], two[MAXL];
  memset(two, 0, sizeof(limb_t) * (size_t)L);
  two[0] = 2;
  big_sub(e, q, two, L);
  mod_pow(c, a, e, L, q, L);
}

static void small_to_limbs(limb_t *r, uint64_t v, int L) {
  memset(r, 0, sizeof(limb_t) * (size_t)L);
  r[0] = (limb_t)v;
  if (L > 1) r[1] = (limb_t)(v >> 32);
}

static int check_L(int L) { return L >= 1 && L <= MAXL; }

/* ---------------------------------------------------------- exported: words */

int oracle_max_limbs(void) { return MAXL; }

int64_t oracle_addback_count(void) { return __atomic_load_n(&g_addbacks, __ATOMIC_RELAXED); }

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int oracle_big_mul(limb_t *r, const limb_t *a, int na, const limb_t *b, int nb) {
  if (na < 1 || nb < 1 || na > 2 * MAXL || nb > 2 * MAXL) return -1;
  big_mul(r, a, na, b, nb);
  return 0;
}

/* rem = u mod v with u of m limbs and v of n limbs */
int oracle_big_rem(limb_t *rem, const limb_t *u, int m, const limb_t *v, int n) {
  if (m < 1 || n < 1 || m > 4 * MAXL || n > MAXL) return -1;
  if (big_len(v, n) == 0) return -2;
  limb_t tmp[MAXL];
  int nv = big_len(v, n);
  int nu = big_len(u, m);
  memset(tmp, 0, sizeof(tmp));
  if (nu < nv || (nu == nv && big_cmp(u, v, nv) < 0)) {
    memcpy(tmp, u, sizeof(limb_t) * (size_t)nu);
  } else {
    big_rem(tmp, u, nu, v, nv);
  }
  memcpy(rem, tmp, sizeof(limb_t) * (size_t)n);
  return 0;
}

int oracle_big_add(limb_t *r, const limb_t *a, const limb_t *b, int n) {
  if (n < 1 || n > 4 * MAXL) return -1;
  return (int)big_add(r, a, b, n);
}

int oracle_big_sub(limb_t *r, const limb_t *a, const limb_t *b, int n) {
  if (n < 1 || n > 4 * MAXL) return -1;
  return (int)big_sub(r, a, b, n);
}

int oracle_mod_pow(limb_t *c, const limb_t *a, const limb_t *e, int ne, const limb_t *q, int L) {
  if (!check_L(L) || ne < 1) return -1;
  mod_pow(c, a, e, ne, q, L);
  return 0;
}

int oracle_mod_inv(limb_t *c, const limb_t *a, const limb_t *q, int L) {
  if (!check_L(L)) return -1;
  mod_inv(c, a, q, L);
  return 0;
}

/* ----------------------------------------------------------- exported: BLAS */

int oracle_vadd(const limb_t *q, int L, int64_t n, const limb_t *a, const limb_t *b, limb_t *out) {
  if (!check_L(L) || n < 0) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) mod_add(out + i * L, a + i * L, b + i * L, q, L);
  return 0;
}

int oracle_vsub(const limb_t *q, int L, int64_t n, const limb_t *a, const limb_t *b, limb_t *out) {
  if (!check_L(L) || n < 0) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) mod_sub(out + i * L, a + i * L, b + i * L, q, L);
  return 0;
}

int oracle_vmul(const limb_t *q, int L, int64_t n, const limb_t *a, const limb_t *b, limb_t *out) {
  if (!check_L(L) || n < 0) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) mod_mul(out + i * L, a + i * L, b + i * L, q, L);
  return 0;
}

/* out_i = alpha * x_i + y_i mod q: the (2L+1)-limb value alpha*x_i + y_i reduced by division */
int oracle_axpy(const limb_t *q, int L, int64_t n, const limb_t *alpha, const limb_t *x, const limb_t *y,
                limb_t *out) {
  if (!check_L(L) || n < 0) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    limb_t p[2 * MAXL + 1], yy[2 * MAXL + 1];
    big_mul(p, alpha, L, x + i * L, L);
    memset(yy, 0, sizeof(yy));
    memcpy(yy, y + i * L, sizeof(limb_t) * (size_t)L);
    p[2 * L] = big_add(p, p, yy, 2 * L);
    reduce(out + i * L, p, 2 * L + 1, q, L);
  }
  return 0;
}

/* ------------------------------------------------------------ exported: NTT */

/* y_k = sum_j x_j w^{jk} for the listed k (Eq. (ntt)); w^k, then running powers (w^k)^j */
static void dft_at(const limb_t *q, int L, int64_t n, const limb_t *w, const limb_t *x, const int64_t *ks,
                   int64_t nk, limb_t *out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < nk; t++) {
    limb_t wk[MAXL], p[MAXL], acc[MAXL], term[MAXL], tmp[MAXL], e[2];
    int64_t k = ks[t] % n;
    e[0] = (limb_t)k;
    e[1] = (limb_t)((uint64_t)k >> 32);
    mod_pow(wk, w, e, 2, q, L);
    small_to_limbs(p, 1, L);
    memset(acc, 0, sizeof(acc));
    for (int64_t j = 0; j < n; j++) {
      mod_mul(term, x + j * L, p, q, L);
      mod_add(tmp, acc, term, q, L);
      memcpy(acc, tmp, sizeof(limb_t) * (size_t)L);
      mod_mul(tmp, p, wk, q, L);
      memcpy(p, tmp, sizeof(limb_t) * (size_t)L);
    }
    memcpy(out + t * L, acc, sizeof(limb_t) * (size_t)L);
  }
}

static int check_ntt_args(int L, int64_t n) {
  if (!check_L(L) || n < 1 || (n & (n - 1))) return -1;
  return 0;
}

/* forward NTT by the definition, for the outputs k in ks (all k when ks == NULL and nk == n) */
int oracle_ntt_direct(const limb_t *q, int L, int64_t n, const limb_t *omega, const limb_t *x, const int64_t *ks,
                      int64_t nk, limb_t *out) {
  if (check_ntt_args(L, n)) return -1;
  int64_t *all = NULL;
  if (!ks) {
    all = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t k = 0; k < n; k++) all[k] = k;
    ks = all;
    nk = n;
  }
  dft_at(q, L, n, omega, x, ks, nk, out);
  free(all);
  return 0;
}

/* inverse NTT by the definition: x_j = n^{-1} sum_k y_k w^{-jk} */
int oracle_intt_direct(const limb_t *q, int L, int64_t n, const limb_t *omega, const limb_t *y, const int64_t *js,
                       int64_t nj, limb_t *out) {
  if (check_ntt_args(L, n)) return -1;
  limb_t winv[MAXL], ninv[MAXL], nn[MAXL];
  mod_inv(winv, omega, q, L);
  small_to_limbs(nn, (uint64_t)n, L);
  mod_inv(ninv, nn, q, L);
  int64_t *all = NULL;
  if (!js) {
    all = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t k = 0; k < n; k++) all[k] = k;
    js = all;
    nj = n;
  }
  dft_at(q, L, n, winv, y, js, nj, out);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nj; t++) {
    limb_t tmp[MAXL];
    mod_mul(tmp, out + t * L, ninv, q, L);
    memcpy(out + t * L, tmp, sizeof(limb_t) * (size_t)L);
  }
  free(all);
  return 0;
}

static int64_t bit_reverse(int64_t i, int bits) {
  int64_t r = 0;
  for (int b = 0; b < bits; b++) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

/*
 * Textbook iterative radix-2 transform (CLRS, Section 30.3, ITERATIVE-FFT):
 * bit-reversal copy, then for block lengths m = 2, 4, ..., n combine halves
 * with powers of w_m = w^{n/m}.  Natural order in and out.
 */
static void ntt_radix2(const limb_t *q, int L, int64_t n, const limb_t *w, const limb_t *x, limb_t *a) {
  int lg = 0;
  while (((int64_t)1 << lg) < n) lg++;
  for (int64_t i = 0; i < n; i++) memcpy(a + bit_reverse(i, lg) * L, x + i * L, sizeof(limb_t) * (size_t)L);
  /* powers w^0 .. w^{n/2-1} once, by repeated multiplication */
  int64_t half = n / 2 > 0 ? n / 2 : 1;
  limb_t *pw = (limb_t *)malloc(sizeof(limb_t) * (size_t)(half * L));
  small_to_limbs(pw, 1, L);
  for (int64_t i = 1; i < half; i++) mod_mul(pw + i * L, pw + (i - 1) * L, w, q, L);
  for (int s = 1; s <= lg; s++) {
    int64_t m = (int64_t)1 << s, h = m / 2, step = n / m;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < n / 2; b++) { /* butterfly b: block b / h, position b % h */
      limb_t u[MAXL], t[MAXL];
      int64_t k = (b / h) * m, j = b % h;
      limb_t *lo = a + (k + j) * L, *hi = a + (k + j + h) * L;
      mod_mul(t, pw + (j * step) * L, hi, q, L);
      memcpy(u, lo, sizeof(limb_t) * (size_t)L);
      mod_add(lo, u, t, q, L);
      mod_sub(hi, u, t, q, L);
    }
  }
  free(pw);
}

int oracle_ntt_radix2(const limb_t *q, int L, int64_t n, const limb_t *omega, const limb_t *x, limb_t *out) {
  if (check_ntt_args(L, n)) return -1;
  ntt_radix2(q, L, n, omega, x, out);
  return 0;
}

int oracle_intt_radix2(const limb_t *q, int L, int64_t n, const limb_t *omega, const limb_t *y, limb_t *out) {
  if (check_ntt_args(L, n)) return -1;
  limb_t winv[MAXL], ninv[MAXL], nn[MAXL];
  mod_inv(winv, omega, q, L);
  small_to_limbs(nn, (uint64_t)n, L);
  mod_inv(ninv, nn, q, L);
  ntt_radix2(q, L, n, winv, y, out);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    limb_t tmp[MAXL];
    mod_mul(tmp, out + i * L, ninv, q, L);
    memcpy(out + i * L, tmp, sizeof(limb_t) * (size_t)L);
  }
  return 0;
}

/* cyclic convolution by its definition: c_k = sum_{i + j == k mod n} a_i b_j */
int oracle_cyclic_conv(const limb_t *q, int L, int64_t n, const limb_t *a, const limb_t *b, limb_t *out) {
  if (!check_L(L) || n < 1) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; k++) {
    limb_t acc[MAXL], t[MAXL], s[MAXL];
    memset(acc, 0, sizeof(acc));
    for (int64_t i = 0; i < n; i++) {
      int64_t j = ((k - i) % n + n) % n;
      mod_mul(t, a + i * L, b + j * L, q, L);
      mod_add(s, acc, t, q, L);
      memcpy(acc, s, sizeof(limb_t) * (size_t)L);
    }
    memcpy(out + k * L, acc, sizeof(limb_t) * (size_t)L);
  }
  return 0;
}

/* ================================================================== MLP
 * FP64 reference for the learned schedule cost model: a multilayer perceptron
 * 7 -> 64 -> 64 -> 1 with ReLU after the two hidden layers, mean squared error
 * loss, and Adam (Kingma and Ba, ICLR 2015) with bias correction.  The seven
 * inputs are the schedule features (the six launch-shape features and the
 * butterfly's word-product form, schoolbook or Karatsuba, Eq. (mulk)).
 * Parameters are one flat array:
 *   W1[64][7], b1[64], W2[64][64], b2[64], W3[64], b3   (4737 values)
 * with W[o][i] the weight from input i to output o.
 */
#define MLP_IN 7
#define MLP_H 64
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1)

int oracle_mlp_nparams(void) { return MLP_NPARAM; }

static void mlp_views(const double *p, const double **W1, const double **b1, const double **W2, const double **b2,
                      const double **W3, const double **b3) {
  *W1 = p;
  *b1 = *W1 + MLP_H * MLP_IN;
  *W2 = *b1 + MLP_H;
  *b2 = *W2 + MLP_H * MLP_H;
  *W3 = *b2 + MLP_H;
  *b3 = *W3 + MLP_H;
}

/* one sample: hidden activations (after ReLU) and output */
static double mlp_one(const double *p, const double *x, double *h1, double *h2) {
  const double *W1, *b1, *W2, *b2, *W3, *b3;
  mlp_views(p, &W1, &b1, &W2, &b2, &W3, &b3);
  for (int o = 0; o < MLP_H; o++) {
    double s = b1[o];
    for (int i = 0; i < MLP_IN; i++) s += W1[o * MLP_IN + i] * x[i];
    h1[o] = s > 0 ? s : 0;
  }
  for (int o = 0; o < MLP_H; o++) {
    double s = b2[o];
    for (int i = 0; i < MLP_H; i++) s += W2[o * MLP_H + i] * h1[i];
    h2[o] = s > 0 ? s : 0;
  }
  double y = b3[0];
  for (int i = 0; i < MLP_H; i++) y += W3[i] * h2[i];
  return y;
}

int oracle_mlp_forward(const double *params, const double *x, int64_t rows, double *y) {
  if (rows < 0) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; r++) {
    double h1[MLP_H], h2[MLP_H];
    y[r] = mlp_one(params, x + r * MLP_IN, h1, h2);
  }
  return 0;
}

/* loss = (1/rows) sum (y - t)^2 and its gradient with respect to every parameter
 * (chain rule through the output layer, the second ReLU layer, the first) */
int oracle_mlp_grad(const double *params, const double *x, const double *t, int64_t rows, double *grad,
                    double *loss) {
  if (rows <= 0) return -1;
  const double *W1, *b1, *W2, *b2, *W3, *b3;
  mlp_views(params, &W1, &b1, &W2, &b2, &W3, &b3);
  memset(grad, 0, sizeof(double) * MLP_NPARAM);
  double *gW1 = grad, *gb1 = gW1 + MLP_H * MLP_IN, *gW2 = gb1 + MLP_H, *gb2 = gW2 + MLP_H * MLP_H,
         *gW3 = gb2 + MLP_H, *gb3 = gW3 + MLP_H;
  double L = 0;
  for (int64_t r = 0; r < rows; r++) {
    double h1[MLP_H], h2[MLP_H], d2[MLP_H], d1[MLP_H];
    const double *xr = x + r * MLP_IN;
    double y = mlp_one(params, xr, h1, h2);
    double e = y - t[r];
    L += e * e;
    double dy = 2.0 * e / (double)rows;
    gb3[0] += dy;
    for (int i = 0; i < MLP_H; i++) {
      gW3[i] += dy * h2[i];
      d2[i] = h2[i] > 0 ? dy * W3[i] : 0;
    }
    for (int o = 0; o < MLP_H; o++) {
      gb2[o] += d2[o];
      for (int i = 0; i < MLP_H; i++) gW2[o * MLP_H + i] += d2[o] * h1[i];
    }
    for (int i = 0; i < MLP_H; i++) {
      double s = 0;
      for (int o = 0; o < MLP_H; o++) s += W2[o * MLP_H + i] * d2[o];
      d1[i] = h1[i] > 0 ? s : 0;
    }
    for (int o = 0; o < MLP_H; o++) {
      gb1[o] += d1[o];
      for (int i = 0; i < MLP_IN; i++) gW1[o * MLP_IN + i] += d1[o] * xr[i];
    }
  }
  *loss = L / (double)rows;
  return 0;
}

/* one Adam step, step counter t >= 1:
 * m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;  p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps) */
int oracle_mlp_adam(double *params, const double *grad, double *m, double *v, int64_t t, double lr, double beta1,
                    double beta2, double eps) {
  if (t < 1) return -1;
  double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
  for (int i = 0; i < MLP_NPARAM; i++) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
    params[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
  return 0;
}
