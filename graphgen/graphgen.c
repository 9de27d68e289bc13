/*
 * graphgen.c -- seeded synthetic inputs for correlation clustering.
 *
 * This module only produces inputs: random permutations (the order pi) and
 * positive-edge graphs in symmetric CSR form.  It holds none of the
 * clustering method's arithmetic, and both the CPU oracle and the GPU
 * library consume what it writes.
 *
 * Random numbers (all published generators, restated here):
 *   - SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the i-th output of a
 *     stream with key k is mix(k + (i+1) * 0x9E3779B97F4A7C15), so it doubles
 *     as a counter-based generator (used for R-MAT samples).
 *   - xoshiro256** (Blackman & Vigna, 2018) for sequential streams, seeded
 *     from SplitMix64.
 *   - Lemire's nearly-divisionless bounded integers (ACM TOMACS 2019).
 *   - Durstenfeld's in-place Fisher-Yates shuffle.
 *   - Box-Muller for normal variates.
 *
 * Graphs (vertex ids are int32, offsets int64, rows sorted ascending, no
 * self-loops, no duplicate entries, every edge stored in both rows):
 *   - Erdos-Renyi G(n,p) by Batagelj-Brandes geometric skipping (2005).
 *   - Chung-Lu with power-law weights, sampled by the Miller-Hagberg
 *     skipping method (2011), p_uv = min(1, w_u w_v / S).
 *   - R-MAT (Chakrabarti, Zhan & Faloutsos 2004) with quadrant
 *     probabilities (a,b,c,d), no per-level noise, seeded vertex relabel,
 *     self-loops dropped, symmetrised and deduplicated.
 *   - Batches of stochastic-block-model graphs (local vertex ids per graph).
 *
 * Every generator is deterministic for a given seed, independent of the
 * number of OpenMP threads: per-item streams are keyed by (seed, item), and
 * rows are sorted after the (unordered) parallel scatter.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GG_GOLDEN 0x9E3779B97F4A7C15ULL

/* ---------------------------------------------------------------- RNG --- */

static inline uint64_t gg_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* i-th output (i >= 0) of the SplitMix64 stream whose state starts at key. */
static inline uint64_t gg_splitmix_at(uint64_t key, uint64_t i) {
  return gg_mix64(key + (i + 1) * GG_GOLDEN);
}

uint64_t gg_splitmix64_at(uint64_t key, uint64_t i) { return gg_splitmix_at(key, i); }

typedef struct { uint64_t s[4]; } gg_xoshiro;

static inline uint64_t gg_rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t gg_next(gg_xoshiro *r) {
  uint64_t *s = r->s;
  const uint64_t result = gg_rotl(s[1] * 5, 7) * 9;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = gg_rotl(s[3], 45);
  return result;
}

/* Stream `id` of generator `seed`: xoshiro256** state filled by SplitMix64
 * from a key that mixes both numbers. */
static void gg_stream(gg_xoshiro *r, uint64_t seed, uint64_t id) {
  uint64_t key = gg_mix64(seed * GG_GOLDEN + 0x632BE59BD9B4E019ULL) ^ gg_mix64(id + 0xD1B54A32D192ED03ULL);
  for (int i = 0; i < 4; i++) r->s[i] = gg_splitmix_at(key, (uint64_t)i);
}

/* Uniform integer in [0, range), range >= 1 (Lemire). */
static inline uint64_t gg_bounded(gg_xoshiro *r, uint64_t range) {
  uint64_t x = gg_next(r);
  __uint128_t m = (__uint128_t)x * range;
  uint64_t l = (uint64_t)m;
  if (l < range) {
    uint64_t t = (0 - range) % range;
    while (l < t) {
      x = gg_next(r);
      m = (__uint128_t)x * range;
      l = (uint64_t)m;
    }
  }
  return (uint64_t)(m >> 64);
}

/* Uniform double in [0, 1) with 53 random bits. */
static inline double gg_uniform(gg_xoshiro *r) { return (double)(gg_next(r) >> 11) * 0x1.0p-53; }

/* Uniform double in (0, 1]. */
static inline double gg_uniform_pos(gg_xoshiro *r) { return ((double)(gg_next(r) >> 11) + 1.0) * 0x1.0p-53; }

/* First few xoshiro256** outputs of stream (seed,id): used by golden tests. */
void gg_stream_outputs(uint64_t seed, uint64_t id, int64_t count, uint64_t *out) {
  gg_xoshiro r;
  gg_stream(&r, seed, id);
  for (int64_t i = 0; i < count; i++) out[i] = gg_next(&r);
}

void gg_bounded_outputs(uint64_t seed, uint64_t id, uint64_t range, int64_t count, uint64_t *out) {
  gg_xoshiro r;
  gg_stream(&r, seed, id);
  for (int64_t i = 0; i < count; i++) out[i] = gg_bounded(&r, range);
}

/* ------------------------------------------------------- permutations --- */

/* order[k] = vertex at rank k: a uniform random permutation of 0..n-1
 * (Durstenfeld's shuffle of the identity), stream (seed, 0). */
void gg_permutation(uint64_t seed, int64_t n, int32_t *order) {
  gg_xoshiro r;
  gg_stream(&r, seed, 0);
  for (int64_t i = 0; i < n; i++) order[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; i--) {
    int64_t j = (int64_t)gg_bounded(&r, (uint64_t)(i + 1));
    int32_t t = order[i];
    order[i] = order[j];
    order[j] = t;
  }
}

/* --------------------------------------------------------- CSR buffers --- */

typedef struct {
  int64_t n;     /* vertices */
  int64_t nnz;   /* stored entries (= 2 * undirected edges) */
  int64_t *off;  /* [n+1] */
  int32_t *col;  /* [nnz] */
  int64_t ngraphs;   /* 1 for a single graph */
  int64_t *vtx_ptr;  /* [ngraphs+1] first vertex of each graph, or NULL */
} gg_csr;

void gg_free(gg_csr *g) {
  if (!g) return;
  free(g->off);
  free(g->col);
  free(g->vtx_ptr);
  free(g);
}

/* Sorts a[0..len) ascending: insertion sort for short rows, else an LSD
 * radix sort on `bits`-bit keys (non-negative values) using tmp[len]. */
static void gg_sort_row(int32_t *a, int64_t len, int bits, int32_t *tmp) {
  if (len <= 48) {
    for (int64_t i = 1; i < len; i++) {
      int32_t x = a[i];
      int64_t j = i - 1;
      while (j >= 0 && a[j] > x) {
        a[j + 1] = a[j];
        j--;
      }
      a[j + 1] = x;
    }
    return;
  }
  const int passes = (bits + 10) / 11;
  int32_t *src = a, *dst = tmp;
  for (int p = 0; p < passes; p++) {
    const int shift = 11 * p;
    int64_t cnt[2049];
    memset(cnt, 0, sizeof(cnt));
    for (int64_t i = 0; i < len; i++) cnt[(((uint32_t)src[i] >> shift) & 2047u) + 1]++;
    for (int d = 0; d < 2048; d++) cnt[d + 1] += cnt[d];
    for (int64_t i = 0; i < len; i++) dst[cnt[((uint32_t)src[i] >> shift) & 2047u]++] = src[i];
    int32_t *t = src;
    src = dst;
    dst = t;
  }
  if (src != a) memcpy(a, src, sizeof(int32_t) * (size_t)len);
}

/* Sort every row, drop duplicate entries, then compact rows to the left.
 * `off` holds the scatter layout on entry and the final layout on exit. */
static void gg_sort_dedup_compact(gg_csr *g) {
  const int64_t n = g->n;
  int64_t *newdeg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < n) bits++;
  int64_t maxlen = 0;
  for (int64_t v = 0; v < n; v++)
    if (g->off[v + 1] - g->off[v] > maxlen) maxlen = g->off[v + 1] - g->off[v];
#pragma omp parallel
  {
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxlen > 0 ? maxlen : 1));
#pragma omp for schedule(dynamic, 4096)
    for (int64_t v = 0; v < n; v++) {
      int32_t *row = g->col + g->off[v];
      int64_t len = g->off[v + 1] - g->off[v];
      gg_sort_row(row, len, bits, tmp);
      int64_t k = 0;
      for (int64_t i = 0; i < len; i++)
        if (k == 0 || row[i] != row[k - 1]) row[k++] = row[i];
      newdeg[v] = k;
    }
    free(tmp);
  }
  /* rows only move left, so a forward serial pass can compact in place */
  int64_t pos = 0;
  for (int64_t v = 0; v < n; v++) {
    int64_t start = g->off[v];
    if (pos != start && newdeg[v] > 0)
      memmove(g->col + pos, g->col + start, sizeof(int32_t) * (size_t)newdeg[v]);
    g->off[v] = pos;
    pos += newdeg[v];
  }
  g->off[n] = pos;
  g->nnz = pos;
  free(newdeg);
  if (pos > 0) {
    int32_t *shrunk = (int32_t *)realloc(g->col, sizeof(int32_t) * (size_t)pos);
    if (shrunk) g->col = shrunk;
  }
}

static gg_csr *gg_alloc(int64_t n) {
  gg_csr *g = (gg_csr *)calloc(1, sizeof(gg_csr));
  g->n = n;
  g->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  g->ngraphs = 1;
  return g;
}

/* deg[] (in g->off[1..n]) -> exclusive offsets; allocates col. */
static int gg_offsets_from_counts(gg_csr *g) {
  int64_t acc = 0;
  for (int64_t v = 0; v < g->n; v++) {
    int64_t d = g->off[v + 1];
    g->off[v] = acc;
    acc += d;
  }
  g->off[g->n] = acc;
  g->nnz = acc;
  g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(acc > 0 ? acc : 1));
  return g->col != NULL;
}

/* ------------------------------------------------------- Erdos-Renyi --- */

/* G(n, p), undirected.  Batagelj-Brandes: walk the lower-triangle pair
 * sequence (v, w), w < v, jumping by geometric gaps of parameter p. */
gg_csr *gg_erdos_renyi(int64_t n, double p, uint64_t seed) {
  gg_csr *g = gg_alloc(n);
  if (n < 2 || p <= 0.0) return g;
  /* edge list first (serial, small graphs), then CSR */
  int64_t cap = 1024, ne = 0;
  int32_t *eu = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
  int32_t *ev = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
  gg_xoshiro r;
  gg_stream(&r, seed, 0);
  const double lq = (p < 1.0) ? log(1.0 - p) : 0.0;
  int64_t v = 1, w = -1;
  while (v < n) {
    if (p < 1.0) {
      double u = gg_uniform(&r);
      w += 1 + (int64_t)floor(log(1.0 - u) / lq);
    } else {
      w += 1;
    }
    while (w >= v && v < n) {
      w -= v;
      v++;
    }
    if (v < n) {
      if (ne == cap) {
        cap *= 2;
        eu = (int32_t *)realloc(eu, sizeof(int32_t) * (size_t)cap);
        ev = (int32_t *)realloc(ev, sizeof(int32_t) * (size_t)cap);
      }
      eu[ne] = (int32_t)v;
      ev[ne] = (int32_t)w;
      ne++;
    }
  }
  for (int64_t e = 0; e < ne; e++) {
    g->off[eu[e] + 1]++;
    g->off[ev[e] + 1]++;
  }
  gg_offsets_from_counts(g);
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  for (int64_t x = 0; x < n; x++) cur[x] = g->off[x];
  for (int64_t e = 0; e < ne; e++) {
    g->col[cur[eu[e]]++] = ev[e];
    g->col[cur[ev[e]]++] = eu[e];
  }
  free(cur);
  free(eu);
  free(ev);
  gg_sort_dedup_compact(g);
  return g;
}

/* ---------------------------------------------------------- Chung-Lu --- */

/* Power-law weights w_i = c (i + i0)^(-1/(gamma-1)), i = 0..n-1 (sorted
 * descending), with sum S and w_0 = sqrt(S) (the largest weight that keeps
 * every w_u w_v / S <= 1).  Solves i0 by bisection. */
/* sum_i (i0/(i+i0))^alpha over i = 0..n-1, in fixed 65536-wide chunks
 * summed in order, so the result does not depend on the thread count. */
static double gg_cl_sum(int64_t n, double i0, double alpha) {
  const int64_t chunk = 65536, nchunks = (n + chunk - 1) / chunk;
  double *part = (double *)calloc((size_t)(nchunks > 0 ? nchunks : 1), sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < nchunks; q++) {
    double s = 0.0;
    const int64_t end = (q + 1) * chunk < n ? (q + 1) * chunk : n;
    for (int64_t i = q * chunk; i < end; i++) s += pow(i0 / ((double)i + i0), alpha);
    part[q] = s;
  }
  double s = 0.0;
  for (int64_t q = 0; q < nchunks; q++) s += part[q];
  free(part);
  return s;
}

/* Power-law weights w_i = c (i + i0)^(-1/(gamma-1)), i = 0..n-1 (sorted
 * descending), with sum S and w_0 = sqrt(S) (the largest weight that keeps
 * every w_u w_v / S <= 1).  Solves i0 by bisection on a log scale. */
void gg_chung_lu_weights(int64_t n, double gamma, double total, double *w) {
  const double alpha = 1.0 / (gamma - 1.0);
  const double target = sqrt(total);
  /* f(i0) = sum_i (i0/(i+i0))^alpha increases with i0; solve f = sqrt(S) */
  double lo = 1e-9, hi = 1.0;
  while (gg_cl_sum(n, hi, alpha) < target && hi < 1e15) hi *= 2.0;
  for (int it = 0; it < 80; it++) {
    double mid = sqrt(lo * hi);
    if (gg_cl_sum(n, mid, alpha) < target) lo = mid; else hi = mid;
  }
  const double i0 = sqrt(lo * hi);
  const double c = total / gg_cl_sum(n, i0, alpha);
  for (int64_t i = 0; i < n; i++) w[i] = c * pow(i0 / ((double)i + i0), alpha);
}

/* Miller-Hagberg walk for row u (weights sorted descending): calls emit for
 * every sampled neighbour v > u.  Stream (seed, 1 + u). */
#define GG_CL_WALK(...)                                                     \
  do {                                                                       \
    gg_xoshiro r;                                                            \
    gg_stream(&r, seed, 1 + (uint64_t)u);                                    \
    int64_t v = u + 1;                                                       \
    if (v < n) {                                                             \
      double p = w[u] * w[v] / S;                                            \
      if (p > 1.0) p = 1.0;                                                  \
      while (v < n && p > 0.0) {                                             \
        if (p != 1.0) {                                                      \
          double rr = gg_uniform_pos(&r);                                    \
          double skip = floor(log(rr) / log1p(-p));                          \
          v = (skip > (double)n) ? n : v + (int64_t)skip;                    \
        }                                                                    \
        if (v < n) {                                                         \
          double q = w[u] * w[v] / S;                                        \
          if (q > 1.0) q = 1.0;                                              \
          double rr = gg_uniform(&r);                                        \
          if (rr < q / p) { __VA_ARGS__; }                                          \
          p = q;                                                             \
          v++;                                                               \
        }                                                                    \
      }                                                                      \
    }                                                                        \
  } while (0)

gg_csr *gg_chung_lu(int64_t n, double gamma, double total, uint64_t seed) {
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  gg_chung_lu_weights(n, gamma, total, w);
  double S = 0.0;
  for (int64_t i = 0; i < n; i++) S += w[i];
  /* seeded relabel so that weight rank does not reveal the vertex id */
  int32_t *relabel = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  gg_permutation(seed ^ 0xC3A5C85C97CB3127ULL, n, relabel);
  gg_csr *g = gg_alloc(n);
  int64_t *deg = g->off + 1;
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t u = 0; u < n; u++) {
    GG_CL_WALK({
      __atomic_fetch_add(&deg[relabel[u]], 1, __ATOMIC_RELAXED);
      __atomic_fetch_add(&deg[relabel[v]], 1, __ATOMIC_RELAXED);
    });
  }
  gg_offsets_from_counts(g);
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  memcpy(cur, g->off, sizeof(int64_t) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t u = 0; u < n; u++) {
    GG_CL_WALK({
      int32_t a = relabel[u], b = relabel[v];
      g->col[__atomic_fetch_add(&cur[a], 1, __ATOMIC_RELAXED)] = b;
      g->col[__atomic_fetch_add(&cur[b], 1, __ATOMIC_RELAXED)] = a;
    });
  }
  free(cur);
  free(relabel);
  free(w);
  gg_sort_dedup_compact(g);
  return g;
}

/* -------------------------------------------------------------- R-MAT --- */

/* Sample e of an R-MAT(scale; a, b, c) stream: two 32-bit uniforms per
 * SplitMix64 output, one per level, most significant bit first. */
static inline void gg_rmat_sample(uint64_t key, uint64_t e, int scale, uint32_t ta, uint32_t tab,
                                  uint32_t tabc, uint32_t *pu, uint32_t *pv) {
  uint32_t u = 0, v = 0;
  const int draws = (scale + 1) / 2;
  for (int k = 0; k < draws; k++) {
    uint64_t x = gg_splitmix_at(key, e * (uint64_t)draws + (uint64_t)k);
    for (int h = 0; h < 2; h++) {
      int level = 2 * k + h;
      if (level >= scale) break;
      uint32_t r = (uint32_t)(h ? (x >> 32) : x);
      /* quadrant 0..3 = a, b, c, d; row bit = q >> 1, column bit = q & 1 */
      const uint32_t q = (uint32_t)(r >= ta) + (uint32_t)(r >= tab) + (uint32_t)(r >= tabc);
      const uint32_t bu = q >> 1, bv = q & 1u;
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
  }
  *pu = u;
  *pv = v;
}

static inline uint32_t gg_prob32(double p) {
  double t = p * 4294967296.0;
  if (t >= 4294967295.0) return 0xFFFFFFFFu;
  if (t <= 0.0) return 0;
  return (uint32_t)t;
}

/* R-MAT with 2^scale vertices and edge_factor * 2^scale samples.
 * Two passes over the counter-based sample stream: count row lengths, then
 * place entries.  Each thread owns a fixed slice of the samples and private
 * per-row counters (no atomics), and samples are handled in blocks so the
 * cache misses of one block overlap. */
#define GG_BLK 64
gg_csr *gg_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed) {
  const int64_t n = (int64_t)1 << scale;
  const uint64_t samples = (uint64_t)edge_factor << scale;
  const uint32_t ta = gg_prob32(a), tab = gg_prob32(a + b), tabc = gg_prob32(a + b + c);
  const uint64_t key = gg_mix64(seed * GG_GOLDEN + 0x2545F4914F6CDD1DULL);
  int32_t *relabel = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!relabel) return NULL;
  gg_permutation(seed ^ 0x9FB21C651E98DF25ULL, n, relabel);
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  /* cnt[t*n + x]: entries of row x produced by thread t; later its cursor */
  int32_t *cnt = (int32_t *)calloc((size_t)nt * (size_t)n, sizeof(int32_t));
  gg_csr *g = gg_alloc(n);
  if (!cnt || !g || !g->off) {
    free(relabel);
    free(cnt);
    gg_free(g);
    return NULL;
  }
  const uint64_t per = (samples + (uint64_t)nt - 1) / (uint64_t)nt;
#pragma omp parallel num_threads(nt)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    int32_t *mine = cnt + (size_t)t * (size_t)n;
    const uint64_t e0 = (uint64_t)t * per, e1 = (e0 + per < samples) ? e0 + per : samples;
    uint32_t bu[GG_BLK], bv[GG_BLK];
    int32_t bx[GG_BLK], by[GG_BLK];
    for (uint64_t eb = e0; eb < e1; eb += GG_BLK) {
      const int m = (int)((e1 - eb) < GG_BLK ? (e1 - eb) : GG_BLK);
      for (int i = 0; i < m; i++) gg_rmat_sample(key, eb + (uint64_t)i, scale, ta, tab, tabc, &bu[i], &bv[i]);
      for (int i = 0; i < m; i++) {
        bx[i] = relabel[bu[i]];
        by[i] = relabel[bv[i]];
      }
      for (int i = 0; i < m; i++)
        if (bu[i] != bv[i]) {
          mine[bx[i]]++;
          mine[by[i]]++;
        }
    }
  }
  /* row lengths, offsets, and per-thread cursors (exclusive within a row) */
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < n; x++) {
    int64_t acc = 0;
    for (int t = 0; t < nt; t++) {
      int32_t c0 = cnt[(size_t)t * (size_t)n + (size_t)x];
      cnt[(size_t)t * (size_t)n + (size_t)x] = (int32_t)acc;
      acc += c0;
    }
    g->off[x + 1] = acc;
  }
  if (!gg_offsets_from_counts(g)) {
    free(relabel);
    free(cnt);
    gg_free(g);
    return NULL;
  }
#pragma omp parallel num_threads(nt)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    int32_t *mine = cnt + (size_t)t * (size_t)n;
    const uint64_t e0 = (uint64_t)t * per, e1 = (e0 + per < samples) ? e0 + per : samples;
    uint32_t bu[GG_BLK], bv[GG_BLK];
    int32_t bx[GG_BLK], by[GG_BLK];
    for (uint64_t eb = e0; eb < e1; eb += GG_BLK) {
      const int m = (int)((e1 - eb) < GG_BLK ? (e1 - eb) : GG_BLK);
      for (int i = 0; i < m; i++) gg_rmat_sample(key, eb + (uint64_t)i, scale, ta, tab, tabc, &bu[i], &bv[i]);
      for (int i = 0; i < m; i++) {
        bx[i] = relabel[bu[i]];
        by[i] = relabel[bv[i]];
      }
      for (int i = 0; i < m; i++)
        if (bu[i] != bv[i]) {
          g->col[g->off[bx[i]] + mine[bx[i]]++] = by[i];
          g->col[g->off[by[i]] + mine[by[i]]++] = bx[i];
        }
    }
  }
  free(cnt);
  free(relabel);
  gg_sort_dedup_compact(g);
  return g;
}

/* ----------------------------------------------- stochastic block model --- */

/* Standard normal by Box-Muller (one of the pair). */
static double gg_normal(gg_xoshiro *r) {
  double u1 = gg_uniform_pos(r), u2 = gg_uniform(r);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* Sizes and block counts of a batch of SBM graphs: n_g = round(exp(N(mu,
 * sigma^2))) redrawn until it lies in [nmin, nmax]; k_g uniform in
 * [kmin, kmax] (capped at n_g).  Stream (seed, 0). */
void gg_sbm_shapes(int64_t ngraphs, double mu, double sigma, int64_t nmin, int64_t nmax,
                   int64_t kmin, int64_t kmax, uint64_t seed, int64_t *sizes, int64_t *blocks) {
  gg_xoshiro r;
  gg_stream(&r, seed, 0);
  for (int64_t gi = 0; gi < ngraphs; gi++) {
    int64_t ng;
    do {
      ng = (int64_t)llround(exp(mu + sigma * gg_normal(&r)));
    } while (ng < nmin || ng > nmax);
    int64_t k = kmin + (int64_t)gg_bounded(&r, (uint64_t)(kmax - kmin + 1));
    if (k > ng) k = ng;
    sizes[gi] = ng;
    blocks[gi] = k;
  }
}

/* Runs the given statement for every sampled pair (uu, vv) of one SBM graph (local ids,
 * u != v, each unordered pair at most once).  Blocks are contiguous and
 * near-equal: the first (n mod k) blocks get one extra vertex. */
#define GG_SBM_WALK(...)                                                              \
  do {                                                                                 \
    gg_xoshiro r;                                                                      \
    gg_stream(&r, seed, 1 + (uint64_t)gi);                                             \
    const int64_t base = ng / k, extra = ng % k;                                       \
    for (int64_t bi = 0; bi < k; bi++) {                                               \
      const int64_t si = base + (bi < extra), oi = bi * base + (bi < extra ? bi : extra); \
      for (int64_t bj = bi; bj < k; bj++) {                                            \
        const int64_t sj = base + (bj < extra), oj = bj * base + (bj < extra ? bj : extra); \
        const double p = (bi == bj) ? p_in : p_out;                                    \
        const int64_t pairs = (bi == bj) ? si * (si - 1) / 2 : si * sj;                \
        if (p <= 0.0 || pairs <= 0) continue;                                          \
        const double lq = (p < 1.0) ? log1p(-p) : 0.0;                                 \
        int64_t idx = -1;                                                              \
        for (;;) {                                                                     \
          if (p < 1.0) {                                                               \
            double skip = floor(log(gg_uniform_pos(&r)) / lq);                         \
            if (skip >= (double)pairs) break;                                          \
            idx += 1 + (int64_t)skip;                                                  \
          } else {                                                                     \
            idx += 1;                                                                  \
          }                                                                            \
          if (idx >= pairs) break;                                                     \
          int64_t uu, vv;                                                              \
          if (bi == bj) { /* idx -> (row x > col y) in the strict lower triangle */    \
            int64_t x = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)idx)) / 2.0);        \
            while (x * (x - 1) / 2 > idx) x--;                                         \
            while ((x + 1) * x / 2 <= idx) x++;                                        \
            uu = oi + x;                                                               \
            vv = oi + (idx - x * (x - 1) / 2);                                         \
          } else {                                                                     \
            uu = oi + idx / sj;                                                        \
            vv = oj + idx % sj;                                                        \
          }                                                                            \
          __VA_ARGS__;                                                                 \
        }                                                                              \
      }                                                                                \
    }                                                                                  \
  } while (0)

/* A batch of SBM graphs in one CSR: vtx_ptr[g] is the first (global) row of
 * graph g, offsets are global positions in col, and col holds LOCAL ids
 * (0 .. n_g - 1) of the same graph. */
gg_csr *gg_sbm_batch(int64_t ngraphs, const int64_t *sizes, const int64_t *blocks, double p_in,
                     double p_out, uint64_t seed) {
  int64_t ntot = 0;
  for (int64_t gi = 0; gi < ngraphs; gi++) ntot += sizes[gi];
  gg_csr *g = gg_alloc(ntot);
  g->ngraphs = ngraphs;
  g->vtx_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ngraphs + 1));
  g->vtx_ptr[0] = 0;
  for (int64_t gi = 0; gi < ngraphs; gi++) g->vtx_ptr[gi + 1] = g->vtx_ptr[gi] + sizes[gi];
  int64_t *deg = g->off + 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t gi = 0; gi < ngraphs; gi++) {
    const int64_t ng = sizes[gi], k = blocks[gi], v0 = g->vtx_ptr[gi];
    GG_SBM_WALK({
      deg[v0 + uu]++;
      deg[v0 + vv]++;
    });
  }
  gg_offsets_from_counts(g);
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ntot > 0 ? ntot : 1));
  memcpy(cur, g->off, sizeof(int64_t) * (size_t)ntot);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t gi = 0; gi < ngraphs; gi++) {
    const int64_t ng = sizes[gi], k = blocks[gi], v0 = g->vtx_ptr[gi];
    GG_SBM_WALK({
      g->col[cur[v0 + uu]++] = (int32_t)vv;
      g->col[cur[v0 + vv]++] = (int32_t)uu;
    });
  }
  free(cur);
  gg_sort_dedup_compact(g);
  return g;
}

/* ---------------------------------------------------------- utilities --- */

/* Build a symmetric CSR from an undirected edge list (u[e], v[e]); drops
 * self-loops and duplicates.  For hand-written test graphs. */
gg_csr *gg_from_edges(int64_t n, int64_t ne, const int32_t *u, const int32_t *v) {
  gg_csr *g = gg_alloc(n);
  for (int64_t e = 0; e < ne; e++) {
    if (u[e] == v[e]) continue;
    g->off[u[e] + 1]++;
    g->off[v[e] + 1]++;
  }
  gg_offsets_from_counts(g);
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t x = 0; x < n; x++) cur[x] = g->off[x];
  for (int64_t e = 0; e < ne; e++) {
    if (u[e] == v[e]) continue;
    g->col[cur[u[e]]++] = v[e];
    g->col[cur[v[e]]++] = u[e];
  }
  free(cur);
  gg_sort_dedup_compact(g);
  return g;
}

int gg_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
