/* Seeded synthetic text generators (input side only: no suffix-sorting
 * arithmetic lives here). Shared by the tests and the benchmark, which feed the
 * same bytes to the CPU oracle and to the HIP library.
 *
 * Random numbers: xoshiro256** (Blackman and Vigna, 2018) seeded through
 * SplitMix64 (Steele, Lea and Flood, 2014), both written from their published
 * definitions. A uniform double in [0, 1) is the top 53 bits times 2^-53.
 */
#include <stdint.h>
#include <stddef.h>
#include <math.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t* x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static void rng_seed(rng_t* r, uint64_t seed) {
  uint64_t x = seed;
  for (int k = 0; k < 4; ++k) r->s[k] = splitmix64(&x);
}

static inline uint64_t rotl(uint64_t v, int k) { return (v << k) | (v >> (64 - k)); }

static inline uint64_t rng_next(rng_t* r) {
  uint64_t* s = r->s;
  uint64_t result = rotl(s[1] * 5, 7) * 9;
  uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl(s[3], 45);
  return result;
}

static inline double rng_uniform(rng_t* r) {
  return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0);
}

/* Standard normal by the Box-Muller transform. */
static double rng_normal(rng_t* r) {
  double u1 = 1.0 - rng_uniform(r); /* (0, 1] */
  double u2 = rng_uniform(r);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* Gamma(a, 1). Marsaglia and Tsang (2000) for a >= 1; for a < 1 the boost
 * Gamma(a) = Gamma(a + 1) * U^(1/a). */
static double rng_gamma(rng_t* r, double a) {
  if (a < 1.0) {
    double u = rng_uniform(r);
    return rng_gamma(r, a + 1.0) * pow(u, 1.0 / a);
  }
  double d = a - 1.0 / 3.0, c = 1.0 / sqrt(9.0 * d);
  for (;;) {
    double x = rng_normal(r), v = 1.0 + c * x;
    if (v <= 0.0) continue;
    v = v * v * v;
    double u = rng_uniform(r);
    if (u < 1.0 - 0.0331 * x * x * x * x) return d * v;
    if (log(u) < 0.5 * x * x + d * (1.0 - v + log(v))) return d * v;
  }
}

/* Transition table of an order-`order` Markov chain over k symbols: k^order
 * rows, each ~ Dirichlet(alpha * 1_k), stored as 16-bit cumulative thresholds:
 * cdf16[row * (k - 1) + j] = min(65535, floor(65536 * (p_0 + ... + p_j))) for
 * j < k - 1. Row r is drawn from its own stream seeded with seed * 2^32 + r, so
 * the table does not depend on the thread count. */
void gen_markov_table(uint64_t seed, int k, int order, double alpha, uint16_t* cdf16) {
  int64_t rows = 1;
  for (int q = 0; q < order; ++q) rows *= k;
#pragma omp parallel
  {
    double g[256];
#pragma omp for schedule(static)
    for (int64_t row = 0; row < rows; ++row) {
      rng_t r;
      rng_seed(&r, (seed << 32) + (uint64_t)row);
      double sum = 0.0;
      for (int j = 0; j < k; ++j) {
        g[j] = rng_gamma(&r, alpha);
        sum += g[j];
      }
      if (sum <= 0.0) { g[0] = 1.0; sum = 1.0; }
      double acc = 0.0;
      for (int j = 0; j < k - 1; ++j) {
        acc += g[j] / sum;
        double t = floor(acc * 65536.0);
        cdf16[row * (k - 1) + j] = (uint16_t)(t > 65535.0 ? 65535.0 : t);
      }
    }
  }
}

/* Order-3 Markov chain over k symbols with the table above. The chain starts
 * from the context (0, 0, 0) (oldest first; row = (s0 * k + s1) * k + s2).
 * Each step draws v = the top 16 bits of the next random word and emits the
 * symbol index #{ j < k - 1 : cdf16[row][j] <= v }, mapped to its byte by
 * `symbols`. Job j first runs `burn_in` steps whose output is dropped, then
 * writes lengths[j] bytes at out + offsets[j]; it draws from seed seeds[j].
 * Every job is its own chain, so the bytes do not depend on scheduling: jobs
 * run in parallel under OpenMP, and each thread steps kLanes jobs in turn so
 * that the table-row reads of different chains overlap. */
enum { kLanes = 8 };

typedef struct {
  rng_t r;
  uint8_t* o;
  uint64_t p, end;
  const uint16_t* row;  /* thresholds of the current context (s0, s1, s2) */
  uint32_t last2, last; /* s1 * k + s2 and s2 */
} chain_t;

void gen_markov3(const uint16_t* cdf16, int k, const uint8_t* symbols, uint8_t* out,
                 const uint64_t* offsets, const uint64_t* lengths, const uint64_t* seeds,
                 int64_t njobs, uint64_t burn_in) {
  const int64_t groups = (njobs + kLanes - 1) / kLanes;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t g = 0; g < groups; ++g) {
    chain_t ch[kLanes];
    int live = 0;
    for (int64_t j = g * kLanes; j < njobs && j < (g + 1) * kLanes; ++j) {
      chain_t* c = &ch[live++];
      rng_seed(&c->r, seeds[j]);
      c->o = out + offsets[j];
      c->p = 0;
      c->end = burn_in + lengths[j];
      c->row = cdf16; /* context (0, 0, 0) */
      c->last2 = 0;
      c->last = 0;
    }
    const uint64_t kk = (uint64_t)k;
    const int m = k - 1; /* thresholds per row */
    while (live > 0) {
      for (int q = 0; q < live;) {
        chain_t* c = &ch[q];
        if (c->p >= c->end) {
          ch[q] = ch[--live];
          continue;
        }
        uint32_t v = (uint32_t)(rng_next(&c->r) >> 48);
        const uint16_t* b = c->row;
        /* The thresholds of a row never decrease, so the number of them <= v
         * is found by halving (branch-free upper bound). */
        int len = m;
        while (len > 1) {
          const int half = len >> 1;
          b = (b[half] <= v) ? b + half : b;
          len -= half;
        }
        const uint32_t idx = (uint32_t)(b - c->row) + (m > 0 && *b <= v);
        if (c->p >= burn_in) c->o[c->p - burn_in] = symbols[idx];
        /* Next context (s1, s2, idx): row (s1 * k + s2) * k + idx. */
        c->row = cdf16 + ((uint64_t)c->last2 * kk + idx) * (uint64_t)m;
        c->last2 = c->last * (uint32_t)k + idx;
        c->last = idx;
        c->p += 1;
        ++q;
      }
    }
  }
}
