/*
 * Seeded synthetic packet-window generator.
 *
 * This module produces the inputs that both the HIP path and the CPU oracle
 * consume.  It holds none of the window-statistics arithmetic: it only draws
 * (src, dst) address pairs and window sizes.  Everything is a pure function
 * of (seed, stream, window, packet chunk), so the output does not depend on
 * the number of threads.
 *
 * Building blocks, each from its published definition:
 *   - SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
 *     generators", OOPSLA 2014) as the counter-based source of 64-bit words.
 *   - Rejection-inversion sampling of a truncated Zipf law (Hoermann and
 *     Derflinger, "Rejection-inversion to generate variates from monotone
 *     discrete distributions", ACM TOMACS 6(3), 1996), O(1) memory, valid for
 *     any exponent > 0 including 1.
 *   - A keyed bijection on 32-bit words (xor-key, odd multiply and xorshift
 *     rounds, each invertible) that maps a popularity rank to an address, so
 *     the addresses of one pool are pairwise distinct by construction.
 *
 * The paper's workload is a single anonymized 2^30-packet capture cut into
 * windows of 2^17 packets (Section III "Inputs", Section IV "GraphBLAS
 * format"); the capture is not available, so heavy-tailed seeded traffic of
 * the same shape stands in for it.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYNTH_CHUNK 65536

typedef struct synth_dist {
  int32_t kind;          /* 0: uniform over the pool, 1: truncated Zipf */
  int32_t pad0;
  double alpha;          /* Zipf exponent (kind 1) */
  uint64_t pool_size;    /* number of addresses in the pool, >= 1 */
  uint32_t pool_key;     /* key of the rank -> address bijection */
  uint32_t super_rank;   /* rank of the super address (outside the pool) */
  double p_super;        /* probability that a draw is the super address */
} synth_dist;

/* ---- SplitMix64 -------------------------------------------------------- */

static inline uint64_t sm64_next(uint64_t* state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline double u01(uint64_t* state) {
  /* 53 random bits -> [0, 1) */
  return (double)(sm64_next(state) >> 11) * (1.0 / 9007199254740992.0);
}

/* Seed of one (seed, stream, window, chunk) sub-stream: a few SplitMix64
 * steps over a state built from the four coordinates. */
static uint64_t substream_seed(uint64_t seed, uint64_t stream, uint64_t window,
                               uint64_t chunk) {
  uint64_t s = seed;
  uint64_t a = sm64_next(&s);
  s ^= stream * 0xD1B54A32D192ED03ull;
  uint64_t b = sm64_next(&s);
  s ^= window * 0x8CB92BA72F3D8DD7ull + a;
  uint64_t c = sm64_next(&s);
  s ^= chunk * 0xABC98388FB8FAC03ull + b;
  return sm64_next(&s) ^ c;
}

/* ---- keyed bijection rank -> address ----------------------------------- */

uint32_t synth_pool_address(uint32_t rank, uint32_t key) {
  uint32_t x = rank ^ key;
  x *= 0x1D637A39u;
  x ^= x >> 15;
  x += key * 0x47759F21u;
  x *= 0xC435E48Bu;
  x ^= x >> 13;
  x *= 0x886C82E7u;
  x ^= x >> 16;
  return x;
}

/* ---- truncated Zipf by rejection-inversion ----------------------------- */

typedef struct zipf_state {
  double q;       /* exponent */
  double n;       /* number of ranks */
  double hx1;     /* H(1.5) - h(1) */
  double hn;      /* H(n + 0.5) */
  double s;       /* squeeze constant */
} zipf_state;

/* log1p(t)/t, continuous at 0 */
static double log1p_over(double t) {
  if (fabs(t) > 1e-8) return log1p(t) / t;
  return 1.0 - t * (0.5 - t * (1.0 / 3.0 - 0.25 * t));
}

/* expm1(t)/t, continuous at 0 */
static double expm1_over(double t) {
  if (fabs(t) > 1e-8) return expm1(t) / t;
  return 1.0 + t * 0.5 * (1.0 + t * (1.0 / 3.0) * (1.0 + 0.25 * t));
}

/* h(x) = x^-q, the (unnormalised) density */
static double zh(const zipf_state* z, double x) { return exp(-z->q * log(x)); }

/* H(x) = integral of h from 1 to x: (x^(1-q) - 1)/(1-q), log x when q = 1 */
static double zH(const zipf_state* z, double x) {
  double lx = log(x);
  return expm1_over((1.0 - z->q) * lx) * lx;
}

/* inverse of H */
static double zHinv(const zipf_state* z, double y) {
  double t = y * (1.0 - z->q);
  if (t < -1.0) t = -1.0;
  return exp(log1p_over(t) * y);
}

static void zipf_init(zipf_state* z, double q, uint64_t n) {
  z->q = q;
  z->n = (double)n;
  z->hx1 = zH(z, 1.5) - 1.0;
  z->hn = zH(z, z->n + 0.5);
  z->s = 2.0 - zHinv(z, zH(z, 2.5) - zh(z, 2.0));
}

/* returns a rank in [1, n] */
static uint64_t zipf_draw(const zipf_state* z, uint64_t* rng) {
  for (;;) {
    double u = z->hn + u01(rng) * (z->hx1 - z->hn);
    double x = zHinv(z, u);
    double kf = floor(x + 0.5);
    if (kf < 1.0) kf = 1.0;
    if (kf > z->n) kf = z->n;
    if (kf - x <= z->s || u >= zH(z, kf + 0.5) - zh(z, kf)) return (uint64_t)kf;
  }
}

/* ---- one address draw -------------------------------------------------- */

typedef struct dist_rt {
  synth_dist d;
  zipf_state z;
} dist_rt;

static void dist_prepare(dist_rt* r, const synth_dist* d) {
  r->d = *d;
  if (d->kind == 1) zipf_init(&r->z, d->alpha, d->pool_size);
}

static inline uint32_t dist_draw(const dist_rt* r, uint64_t* rng) {
  if (r->d.p_super > 0.0 && u01(rng) < r->d.p_super)
    return synth_pool_address(r->d.super_rank, r->d.pool_key);
  uint64_t rank;
  if (r->d.kind == 1) {
    rank = zipf_draw(&r->z, rng) - 1;
  } else {
    rank = (uint64_t)(u01(rng) * (double)r->d.pool_size);
    if (rank >= r->d.pool_size) rank = r->d.pool_size - 1;
  }
  return synth_pool_address((uint32_t)rank, r->d.pool_key);
}

/* ---- batch fill, parallel over (window, chunk) items ------------------- */

typedef struct fill_job {
  uint32_t* src;
  uint32_t* dst;
  const int64_t* offsets;
  int64_t num_windows;
  int64_t first_window;   /* window index of offsets[0]'s window in the stream */
  uint64_t seed;
  dist_rt s, d;
  int64_t* item_prefix;   /* chunks before window w */
  int64_t total_items;
  int64_t next;           /* shared work counter */
  pthread_mutex_t mu;
} fill_job;

static void fill_item(fill_job* j, int64_t item) {
  /* find the window of this item */
  int64_t lo = 0, hi = j->num_windows - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) / 2;
    if (j->item_prefix[mid] <= item) lo = mid; else hi = mid - 1;
  }
  int64_t w = lo;
  int64_t chunk = item - j->item_prefix[w];
  int64_t wbeg = j->offsets[w], wend = j->offsets[w + 1];
  int64_t beg = wbeg + chunk * SYNTH_CHUNK;
  int64_t end = beg + SYNTH_CHUNK;
  if (end > wend) end = wend;
  uint64_t gw = (uint64_t)(j->first_window + w);
  uint64_t rs = substream_seed(j->seed, 1, gw, (uint64_t)chunk);
  uint64_t rd = substream_seed(j->seed, 2, gw, (uint64_t)chunk);
  for (int64_t i = beg; i < end; ++i) {
    j->src[i] = dist_draw(&j->s, &rs);
    j->dst[i] = dist_draw(&j->d, &rd);
  }
}

static void* fill_worker(void* arg) {
  fill_job* j = (fill_job*)arg;
  for (;;) {
    int64_t item;
    pthread_mutex_lock(&j->mu);
    item = j->next;
    j->next += 1;
    pthread_mutex_unlock(&j->mu);
    if (item >= j->total_items) break;
    fill_item(j, item);
  }
  return NULL;
}

/*
 * Fill src/dst for the windows [offsets[w], offsets[w+1]), w < num_windows.
 * Window w draws from the sub-streams of global window index first_window+w.
 * Returns 0, or -1 on bad arguments.
 */
int synth_fill(uint32_t* src, uint32_t* dst, const int64_t* offsets,
               int64_t num_windows, int64_t first_window, uint64_t seed,
               const synth_dist* sd, const synth_dist* dd, int threads) {
  if (num_windows < 0 || (num_windows > 0 && (!src || !dst || !offsets)) || !sd || !dd)
    return -1;
  if (sd->pool_size == 0 || dd->pool_size == 0) return -1;
  if (sd->pool_size > 0x100000000ull || dd->pool_size > 0x100000000ull) return -1;
  if (num_windows == 0) return 0;
  fill_job j;
  memset(&j, 0, sizeof j);
  j.src = src; j.dst = dst; j.offsets = offsets; j.num_windows = num_windows;
  j.first_window = first_window; j.seed = seed;
  dist_prepare(&j.s, sd);
  dist_prepare(&j.d, dd);
  j.item_prefix = (int64_t*)malloc(sizeof(int64_t) * (size_t)(num_windows + 1));
  if (!j.item_prefix) return -1;
  int64_t acc = 0;
  for (int64_t w = 0; w < num_windows; ++w) {
    int64_t n = offsets[w + 1] - offsets[w];
    if (n < 0) { free(j.item_prefix); return -1; }
    j.item_prefix[w] = acc;
    acc += (n + SYNTH_CHUNK - 1) / SYNTH_CHUNK;
  }
  j.item_prefix[num_windows] = acc;
  j.total_items = acc;
  pthread_mutex_init(&j.mu, NULL);
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  if (threads == 1 || acc <= 1) {
    fill_worker(&j);
  } else {
    pthread_t tid[256];
    int started = 0;
    for (int t = 0; t < threads; ++t)
      if (pthread_create(&tid[t], NULL, fill_worker, &j) == 0) ++started;
    if (started == 0) fill_worker(&j);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
  }
  pthread_mutex_destroy(&j.mu);
  free(j.item_prefix);
  return 0;
}

/* Window sizes n = floor(2^U), U ~ Uniform[lo_log2, hi_log2), clamped to
 * [2^lo_log2, 2^hi_log2]. */
void synth_log_uniform_sizes(int64_t* out, int64_t count, uint64_t seed,
                             double lo_log2, double hi_log2) {
  uint64_t rng = substream_seed(seed, 3, 0, 0);
  double lo = ldexp(1.0, (int)lo_log2), hi = ldexp(1.0, (int)hi_log2);
  for (int64_t i = 0; i < count; ++i) {
    double u = lo_log2 + u01(&rng) * (hi_log2 - lo_log2);
    double n = floor(exp2(u));
    if (n < lo) n = lo;
    if (n > hi) n = hi;
    out[i] = (int64_t)n;
  }
}

/* Exponential inter-arrival gaps with the given mean (Poisson arrivals). */
void synth_exponential_gaps(double* out, int64_t count, uint64_t seed, double mean) {
  uint64_t rng = substream_seed(seed, 4, 0, 0);
  for (int64_t i = 0; i < count; ++i) {
    double u = u01(&rng);
    out[i] = -mean * log1p(-u);
  }
}

/* Raw uniform draws in [0, 1) for tests of the generator itself. */
void synth_uniform(double* out, int64_t count, uint64_t seed) {
  uint64_t rng = substream_seed(seed, 5, 0, 0);
  for (int64_t i = 0; i < count; ++i) out[i] = u01(&rng);
}

/* Raw Zipf ranks in [1, n] for tests of the sampler itself. */
void synth_zipf_ranks(uint64_t* out, int64_t count, uint64_t seed, double alpha,
                      uint64_t n) {
  zipf_state z;
  zipf_init(&z, alpha, n);
  uint64_t rng = substream_seed(seed, 6, 0, 0);
  for (int64_t i = 0; i < count; ++i) out[i] = zipf_draw(&z, &rng);
}
