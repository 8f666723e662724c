/*
 * Seeded synthetic-input generators shared by the tests, the oracle's callers
 * and the benchmark.  This file holds random-number generation only: nothing
 * here packs, decodes, filters or aggregates a column.
 *
 *   PCG32 (XSH-RR output on a 64-bit LCG state), written from M. E. O'Neill,
 *   "PCG: A Family of Simple Fast Space-Efficient Statistically Good Algorithms
 *   for Random Number Generation" (2014): state' = state * 6364136223846793005
 *   + inc, output = rotr32(((old >> 18) ^ old) >> 27, old >> 59), with the
 *   two-step seeding of the reference "srandom" procedure.
 *
 *   Jump-ahead: F. B. Brown, "Random number generation with arbitrary strides"
 *   (1994): advancing an LCG by d steps composes the affine map by squaring.
 *   It lets every thread start at its own offset, so a fill is a pure function
 *   of (seed, stream, index) and does not depend on the thread count.
 *
 *   Bounded draws: D. Lemire, "Fast random integer generation in an interval"
 *   (2019), multiply-shift form (x * range) >> 32 WITHOUT the rejection step,
 *   so each output consumes exactly one draw (bias at most range / 2^32).
 *
 *   Gaussian: Box and Muller (1958) from two uniform draws u1, u2 in (0,1):
 *   z = sqrt(-2 ln u1) * cos(2 pi u2); draw i uses PCG outputs 2i and 2i+1.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PCG_MULT 6364136223846793005ULL

typedef struct {
  uint64_t state;
  uint64_t inc;
} pcg32_t;

static inline uint32_t pcg32_next(pcg32_t* r) {
  uint64_t old = r->state;
  r->state = old * PCG_MULT + r->inc;
  uint32_t xs = (uint32_t)(((old >> 18u) ^ old) >> 27u);
  uint32_t rot = (uint32_t)(old >> 59u);
  return (xs >> rot) | (xs << ((32u - rot) & 31u));
}

static void pcg32_seed(pcg32_t* r, uint64_t initstate, uint64_t initseq) {
  r->state = 0u;
  r->inc = (initseq << 1u) | 1u;
  pcg32_next(r);
  r->state += initstate;
  pcg32_next(r);
}

static void pcg32_advance(pcg32_t* r, uint64_t delta) {
  uint64_t cur_mult = PCG_MULT, cur_plus = r->inc;
  uint64_t acc_mult = 1u, acc_plus = 0u;
  while (delta > 0) {
    if (delta & 1u) {
      acc_mult *= cur_mult;
      acc_plus = acc_plus * cur_mult + cur_plus;
    }
    cur_plus = (cur_mult + 1u) * cur_plus;
    cur_mult *= cur_mult;
    delta >>= 1u;
  }
  r->state = acc_mult * r->state + acc_plus;
}

/* ---- threaded fill driver ------------------------------------------------ */

enum { KIND_U32 = 0, KIND_BOUNDED = 1, KIND_GAUSS = 2, KIND_UNIT = 3 };

typedef struct {
  int kind;
  uint64_t seed, stream, first, count;
  uint32_t range;
  double clip;
  void* out;
} fill_job;

static void* fill_worker(void* p) {
  fill_job* j = (fill_job*)p;
  pcg32_t r;
  pcg32_seed(&r, j->seed, j->stream);
  uint64_t draws_per = (j->kind == KIND_GAUSS) ? 2u : 1u;
  pcg32_advance(&r, j->first * draws_per);
  if (j->kind == KIND_U32) {
    uint32_t* o = (uint32_t*)j->out;
    for (uint64_t i = 0; i < j->count; i++) o[i] = pcg32_next(&r);
  } else if (j->kind == KIND_BOUNDED) {
    uint32_t* o = (uint32_t*)j->out;
    for (uint64_t i = 0; i < j->count; i++)
      o[i] = (uint32_t)(((uint64_t)pcg32_next(&r) * (uint64_t)j->range) >> 32);
  } else if (j->kind == KIND_UNIT) {
    double* o = (double*)j->out;
    for (uint64_t i = 0; i < j->count; i++)
      o[i] = ((double)pcg32_next(&r) + 0.5) * (1.0 / 4294967296.0);
  } else {
    double* o = (double*)j->out;
    const double two_pi = 6.283185307179586476925286766559;
    for (uint64_t i = 0; i < j->count; i++) {
      double u1 = ((double)pcg32_next(&r) + 0.5) * (1.0 / 4294967296.0);
      double u2 = ((double)pcg32_next(&r) + 0.5) * (1.0 / 4294967296.0);
      double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
      if (j->clip > 0.0) {
        if (z > j->clip) z = j->clip;
        if (z < -j->clip) z = -j->clip;
      }
      o[i] = z;
    }
  }
  return NULL;
}

static int run_fill(int kind, uint64_t seed, uint64_t stream, uint64_t offset, uint64_t n,
                    uint32_t range, double clip, void* out, size_t elem, int nthreads) {
  if (n == 0) return 0;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  if ((uint64_t)nthreads > n / 65536u + 1u) nthreads = (int)(n / 65536u + 1u);
  pthread_t th[64];
  fill_job jobs[64];
  uint64_t chunk = (n + (uint64_t)nthreads - 1u) / (uint64_t)nthreads;
  int started = 0;
  for (int t = 0; t < nthreads; t++) {
    uint64_t a = (uint64_t)t * chunk;
    if (a >= n) break;
    uint64_t c = (n - a < chunk) ? n - a : chunk;
    jobs[t].kind = kind;
    jobs[t].seed = seed;
    jobs[t].stream = stream;
    jobs[t].first = offset + a;
    jobs[t].count = c;
    jobs[t].range = range;
    jobs[t].clip = clip;
    jobs[t].out = (char*)out + a * elem;
    if (pthread_create(&th[t], NULL, fill_worker, &jobs[t]) != 0) {
      fill_worker(&jobs[t]);
      th[t] = 0;
    }
    started = t + 1;
  }
  for (int t = 0; t < started; t++)
    if (th[t]) pthread_join(th[t], NULL);
  return 0;
}

/* Raw 32-bit outputs number offset .. offset+n-1 of PCG32(seed, stream). */
int synth_pcg32_fill(uint64_t seed, uint64_t stream, uint64_t offset, uint64_t n, uint32_t* out,
                     int nthreads) {
  return run_fill(KIND_U32, seed, stream, offset, n, 0, 0.0, out, sizeof(uint32_t), nthreads);
}

/* Lemire multiply-shift bounded draws in [0, range), one draw each. */
int synth_pcg32_bounded_fill(uint64_t seed, uint64_t stream, uint64_t offset, uint64_t n,
                             uint32_t range, uint32_t* out, int nthreads) {
  if (range == 0) return -1;
  return run_fill(KIND_BOUNDED, seed, stream, offset, n, range, 0.0, out, sizeof(uint32_t),
                  nthreads);
}

/* Uniform doubles in (0,1): (draw + 0.5) / 2^32. */
int synth_unit_fill(uint64_t seed, uint64_t stream, uint64_t offset, uint64_t n, double* out,
                    int nthreads) {
  return run_fill(KIND_UNIT, seed, stream, offset, n, 0, 0.0, out, sizeof(double), nthreads);
}

/* Box-Muller standard normals, optionally clipped to [-clip, clip] (clip <= 0: none). */
int synth_gauss_fill(uint64_t seed, uint64_t stream, uint64_t offset, uint64_t n, double clip,
                     double* out, int nthreads) {
  return run_fill(KIND_GAUSS, seed, stream, offset, n, 0, clip, out, sizeof(double), nthreads);
}

/* Fisher-Yates (Durstenfeld) shuffle of perm[0..n) in place; swap partner for
 * position i (counting down from n-1) is a bounded draw in [0, i+1). */
int synth_fisher_yates(uint64_t seed, uint64_t stream, uint32_t* perm, uint64_t n) {
  if (n < 2) return 0;
  if (n > 0xFFFFFFFFull) return -1;
  pcg32_t r;
  pcg32_seed(&r, seed, stream);
  for (uint64_t i = n - 1; i > 0; i--) {
    uint32_t j = (uint32_t)(((uint64_t)pcg32_next(&r) * (uint64_t)(i + 1u)) >> 32);
    uint32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
  return 0;
}
