/*
 * netgen.c - seeded synthetic network generator (inputs only).
 *
 * Fills the in-edge CSR of a region-structured random network: for each
 * post-synaptic neuron i of target region t, k_in sources drawn uniformly
 * (with replacement, no autapse) from region t and k_cross sources drawn by
 * first picking a source region s != t with probability proportional to the
 * region-connection weight M[s -> t] and then a neuron uniformly in s.
 * Integer delays are uniform on [1, max_delay] and weights log-normal.
 * Each row is returned with its own-region sources first, then its
 * cross-region ones, each part sorted by (source id, delay, draw index): the
 * own-region part is the row's J_intra share when a partition holds whole
 * regions, the cross-region part what other partitions would send.
 *
 * The random numbers come from a counter-based hash (SplitMix64 finaliser,
 * Steele, Lea & Flood, OOPSLA 2014) keyed by (seed, stream, neuron, draw), so
 * the output does not depend on the thread count.  This file holds none of
 * the simulation arithmetic: it only produces the inputs that both the
 * simulator and the reference consume.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define STREAM_SRC 0x5352434bull  /* source choice */
#define STREAM_DLY 0x444c594bull  /* delay */
#define STREAM_WGT 0x5747544bull  /* weight */
#define STREAM_REG 0x5245474bull  /* cross-region choice */

static inline uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

static inline uint64_t hash4(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  return mix64(mix64(mix64(mix64(seed) ^ stream) ^ a) ^ b);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double unif(uint64_t h) { return (double)(h >> 11) * (1.0 / 9007199254740992.0); }

/* uniform integer in [0, n) by 64x64 multiply-high (bias < 2^-32 for n < 2^32) */
static inline uint64_t below(uint64_t h, uint64_t n) {
  return (uint64_t)(((unsigned __int128)h * n) >> 64);
}

static void sort_keys(uint64_t* k, float* w, int n) {
  /* insertion sort on (key, weight) pairs; rows are short (tens to hundreds) */
  for (int a = 1; a < n; a++) {
    uint64_t kk = k[a];
    float ww = w[a];
    int b = a - 1;
    while (b >= 0 && k[b] > kk) {
      k[b + 1] = k[b];
      w[b + 1] = w[b];
      b--;
    }
    k[b + 1] = kk;
    w[b + 1] = ww;
  }
}

/*
 * region_start : [n_regions + 1] first neuron of each region (regions are
 *                contiguous id ranges, region r = [start[r], start[r+1]))
 * cross_cdf    : [n_regions][n_regions] row t = cumulative distribution over
 *                source regions s for the cross-region draws of target t
 *                (entry t itself carries zero mass); a row whose last entry
 *                is 0 means "no cross-region sources": those draws fall back
 *                to the own region.
 * Outputs col/delay/w are [n * (k_in + k_cross)] in row order.
 * Returns 0 on success, -1 on bad arguments.
 */
int netgen_fill(int64_t n, int32_t n_regions, const int64_t* region_start,
                int32_t k_in, int32_t k_cross, const double* cross_cdf,
                int32_t max_delay, double w_mu, double w_sigma, uint64_t seed,
                int32_t* col, uint8_t* delay, float* w) {
  if (n <= 0 || n_regions <= 0 || k_in < 0 || k_cross < 0 || max_delay < 1 || max_delay > 255)
    return -1;
  const int K = k_in + k_cross;
  if (K <= 0 || K > 65535) return -1;
  if (region_start[0] != 0 || region_start[n_regions] != n) return -1;

  int bad = 0;
#pragma omp parallel
  {
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)K);
    float* ws = (float*)malloc(sizeof(float) * (size_t)K);
#pragma omp for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; i++) {
      /* target region of i (binary search over region starts) */
      int lo = 0, hi = n_regions - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (region_start[mid] <= i) lo = mid; else hi = mid - 1;
      }
      const int t = lo;
      const int64_t t0 = region_start[t], tn = region_start[t + 1] - t0;
      const double* cdf = cross_cdf + (size_t)t * n_regions;
      const double total = cdf[n_regions - 1];
      for (int k = 0; k < K; k++) {
        int64_t s0 = t0, sn = tn;
        if (k >= k_in && total > 0.0) {
          double u = unif(hash4(seed, STREAM_REG, (uint64_t)i, (uint64_t)k)) * total;
          int a = 0, b = n_regions - 1;
          while (a < b) {
            int m = (a + b) >> 1;
            if (cdf[m] > u) b = m; else a = m + 1;
          }
          s0 = region_start[a];
          sn = region_start[a + 1] - s0;
        }
        int64_t src = -1;
        for (uint64_t attempt = 0; attempt < 1024; attempt++) {
          uint64_t h = hash4(seed, STREAM_SRC, (uint64_t)i, (uint64_t)k | (attempt << 32));
          int64_t c = s0 + (int64_t)below(h, (uint64_t)sn);
          if (c != i) { src = c; break; }
        }
        if (src < 0) {
#pragma omp atomic write
          bad = 1;
          src = 0;
        }
        uint64_t d = 1 + below(hash4(seed, STREAM_DLY, (uint64_t)i, (uint64_t)k), (uint64_t)max_delay);
        /* log-normal weight: Box-Muller normal from two hashed uniforms */
        uint64_t hw = hash4(seed, STREAM_WGT, (uint64_t)i, (uint64_t)k);
        double u1 = ((double)(hw >> 40) + 0.5) * (1.0 / 16777216.0);
        double u2 = (double)((hw >> 16) & 0xFFFFFF) * (1.0 / 16777216.0);
        double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        ws[k] = (float)exp(w_mu + w_sigma * z);
        const uint64_t cross = (src < t0 || src >= t0 + tn) ? 1ull : 0ull;
        keys[k] = (cross << 62) | ((uint64_t)src << 24) | (d << 16) | (uint64_t)k;
      }
      sort_keys(keys, ws, K);
      const int64_t base = i * (int64_t)K;
      for (int k = 0; k < K; k++) {
        col[base + k] = (int32_t)((keys[k] & ~(1ull << 62)) >> 24);
        delay[base + k] = (uint8_t)((keys[k] >> 16) & 0xFF);
        w[base + k] = ws[k];
      }
    }
    free(keys);
    free(ws);
  }
  return bad ? -1 : 0;
}

/* uniform floats in [lo, hi) for per-neuron initial values, keyed like the rest */
int netgen_uniform(int64_t n, double lo, double hi, uint64_t seed, uint64_t stream, float* out) {
  if (n < 0 || !(hi >= lo)) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double u = unif(hash4(seed, stream, (uint64_t)i, 0));
    float v = (float)(lo + (hi - lo) * u);
    if (v >= (float)hi) v = nextafterf((float)hi, -INFINITY);
    out[i] = v;
  }
  return 0;
}
