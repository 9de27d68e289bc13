/*
 * cc_oracle.c -- CPU oracle for parallel correlation clustering
 * (Pan, Papailiopoulos, Oymak, Recht, Ramchandran, Jordan: "Parallel
 * Correlation Clustering on Big Graphs", arXiv 1507.05086).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the GPU library.
 *
 * Plain, serial, single-threaded code, written for clarity rather than speed.
 * Inputs are a positive-edge graph in symmetric CSR (off[n+1] int64,
 * col[off[n]] int32; row v lists N(v)) and the order pi given as
 * order[k] = vertex of rank k (so rank = order^-1).
 *
 * Readings of the paper taken here (where it is silent or ambiguous):
 *  - "n" in the active-set size eps*n/Delta is n_i, the number of vertices
 *    still unclustered when the round starts (the running-time proof and the
 *    Binomial-sampling section use n_i).
 *  - The size is rounded up and kept in [1, n_i]; eps is read in millionths,
 *    eps_q = round(eps * 1e6), and B_i = ceil(eps_q * n_i / (1e6 * Delta_i)),
 *    all in 64-bit integers.  When Delta_i = 0 (only isolated vertices
 *    remain) the round takes all of them: B_i = n_i.
 *  - Delta_i is the largest number of still-unclustered positive neighbours
 *    of a still-unclustered vertex (the maximum degree of G restricted to V).
 *  - clusterID holds the rank of the center while running; the output label
 *    is the center's vertex id.
 *  - A C4 active vertex that is not a center takes the lowest-rank adjacent
 *    center (the serial-equivalence argument of Section 3); createCluster's
 *    target set Gamma(v)\A is read as N(v) minus the active CENTERS for C4,
 *    and as N(v) minus all active vertices for ClusterWild! (where every
 *    active vertex is a center).
 *  - A "blocked" (conflict) vertex is an active vertex with at least one
 *    earlier-ranked active neighbour: the vertices that would wait inside
 *    isCenter (Algorithm 2), counted the same way for both algorithms.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NONE (-1)
#define ORC_INF INT32_MAX

typedef struct {
  int64_t n_i;       /* unclustered vertices at round start */
  int64_t delta_i;   /* max remaining degree at round start */
  int64_t b_i;       /* active-set size */
  int64_t r_i;       /* rank of the last active vertex */
  int64_t centers;   /* centers elected this round */
  int64_t claimed;   /* non-center vertices clustered this round */
  int64_t conflicts; /* active vertices with an earlier active neighbour */
} orc_round;

enum { ORC_C4 = 0, ORC_CW = 1 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ETRACE = -3 };

/* rank[order[k]] = k.  Returns ORC_EINVAL if order is not a permutation. */
static int orc_invert(int64_t n, const int32_t *order, int32_t *rank) {
  for (int64_t v = 0; v < n; v++) rank[v] = -1;
  for (int64_t k = 0; k < n; k++) {
    int32_t v = order[k];
    if (v < 0 || v >= n || rank[v] != -1) return ORC_EINVAL;
    rank[v] = (int32_t)k;
  }
  return ORC_OK;
}

/*
 * KwikCluster with a preassigned order (Algorithm 1, Section 2): take the
 * unclustered vertex of lowest rank, cluster it with its still-unclustered
 * positive neighbours, remove them, repeat.  labels[v] = center vertex id.
 * By the serializability result of Section 3 this is also C4's output for
 * every eps.
 */
int orc_kwikcluster(int64_t n, const int64_t *off, const int32_t *col, const int32_t *order,
                    int32_t *labels) {
  for (int64_t v = 0; v < n; v++) labels[v] = ORC_NONE;
  for (int64_t k = 0; k < n; k++) {
    int32_t v = order[k];
    if (v < 0 || v >= n) return ORC_EINVAL;
    if (labels[v] != ORC_NONE) continue;
    labels[v] = v; /* v is a center */
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
      int32_t u = col[e];
      if (labels[u] == ORC_NONE) labels[u] = v;
    }
  }
  return ORC_OK;
}

static int64_t orc_batch_size(int64_t eps_q, int64_t n_rem, int64_t delta) {
  if (delta == 0) return n_rem;
  const int64_t q = 1000000;
  int64_t num = eps_q * n_rem, den = q * delta;
  int64_t b = (num + den - 1) / den;
  if (b < 1) b = 1;
  if (b > n_rem) b = n_rem;
  return b;
}

/* eps in millionths, round half away from zero (eps > 0). */
int64_t orc_quantize_eps(double eps) { return (int64_t)(eps * 1e6 + 0.5); }

/*
 * Bulk-synchronous C4 / ClusterWild! (Algorithm 2), simulated serially one
 * round at a time.  Each round:
 *   1. Delta_i = max remaining degree; B_i from eps (or sched[i] if given);
 *   2. A = the next B_i unclustered vertices of pi (lazy deletion: a cursor
 *      walks pi once and skips clustered vertices);
 *   3. centers: C4 keeps a in A iff no earlier-ranked active neighbour is a
 *      center (concurrency rule 1, the greedy MIS of G[A] in pi order);
 *      ClusterWild! takes every a in A;
 *   4. every eligible unclustered neighbour of a center joins the adjacent
 *      center of lowest rank (concurrency rule 2, createCluster);
 *   5. clustered vertices leave the graph (remaining degrees drop).
 * sched (optional, sched_len entries, each >= 1) replaces step 1's rule for
 * the first sched_len rounds with B_i = min(sched[i], n_i).
 * Writes labels (center vertex ids), up to trace_cap round records and, if
 * round_of is given, the round in which each vertex was clustered.
 * Returns the number of rounds, or a negative ORC_E* code.
 */
int64_t orc_bsp(int algo, int64_t n, const int64_t *off, const int32_t *col, const int32_t *order,
                int64_t eps_q, const int64_t *sched, int64_t sched_len, int32_t *labels,
                orc_round *trace, int64_t trace_cap, int32_t *round_of) {
  if ((algo != ORC_C4 && algo != ORC_CW) || n < 0 || eps_q <= 0) return ORC_EINVAL;
  for (int64_t i = 0; i < sched_len; i++)
    if (!sched || sched[i] < 1) return ORC_ETRACE;
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; v++)
    if (off[v + 1] - off[v] > maxdeg) maxdeg = off[v + 1] - off[v];

  int32_t *rank = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *resdeg = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *best = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *active_list = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *touched = malloc(sizeof(int32_t) * (size_t)(n + 1));
  uint8_t *active = calloc((size_t)(n + 1), 1);
  uint8_t *center = calloc((size_t)(n + 1), 1);
  int64_t *cnt = calloc((size_t)(maxdeg + 1), sizeof(int64_t));
  int64_t rounds = ORC_ENOMEM;
  if (!rank || !resdeg || !best || !active_list || !touched || !active || !center || !cnt) goto done;
  if (orc_invert(n, order, rank) != ORC_OK) {
    rounds = ORC_EINVAL;
    goto done;
  }
  for (int64_t v = 0; v < n; v++) {
    labels[v] = ORC_NONE;
    resdeg[v] = (int32_t)(off[v + 1] - off[v]);
    best[v] = ORC_INF;
    cnt[resdeg[v]]++; /* histogram of remaining degrees of unclustered vertices */
  }
  int64_t n_rem = n, cursor = 0, delta = maxdeg;
  rounds = 0;
  while (n_rem > 0) {
    /* 1. Delta_i: the largest remaining degree still present */
    while (delta > 0 && cnt[delta] == 0) delta--;
    int64_t b;
    if (rounds < sched_len) b = sched[rounds] < n_rem ? sched[rounds] : n_rem;
    else b = orc_batch_size(eps_q, n_rem, delta);

    /* 2. active set: next b unclustered vertices of pi */
    int64_t na = 0;
    while (na < b) {
      int32_t v = order[cursor++];
      if (labels[v] == ORC_NONE) active_list[na++] = v;
    }
    for (int64_t i = 0; i < na; i++) active[active_list[i]] = 1;

    /* blocked vertices: an earlier-ranked active neighbour exists */
    int64_t conflicts = 0;
    for (int64_t i = 0; i < na; i++) {
      int32_t a = active_list[i];
      for (int64_t e = off[a]; e < off[a + 1]; e++)
        if (active[col[e]] && rank[col[e]] < rank[a]) {
          conflicts++;
          break;
        }
    }

    /* 3. centers (active_list is in rank order) */
    int64_t ncenters = 0;
    for (int64_t i = 0; i < na; i++) {
      int32_t a = active_list[i];
      int ok = 1;
      if (algo == ORC_C4) {
        for (int64_t e = off[a]; e < off[a + 1]; e++)
          if (center[col[e]]) { /* only earlier actives are marked so far */
            ok = 0;
            break;
          }
      }
      center[a] = (uint8_t)ok;
      ncenters += ok;
    }

    /* 4. claims: lowest-rank adjacent center wins */
    int64_t ntouched = 0;
    for (int64_t i = 0; i < na; i++) {
      int32_t c = active_list[i];
      if (!center[c]) continue;
      for (int64_t e = off[c]; e < off[c + 1]; e++) {
        int32_t u = col[e];
        if (labels[u] != ORC_NONE || center[u]) continue;
        if (algo == ORC_CW && active[u]) continue;
        if (best[u] == ORC_INF) touched[ntouched++] = u;
        if (rank[c] < best[u]) best[u] = rank[c];
      }
    }
    for (int64_t i = 0; i < na; i++)
      if (center[active_list[i]]) labels[active_list[i]] = active_list[i];
    for (int64_t i = 0; i < ntouched; i++) labels[touched[i]] = order[best[touched[i]]];
    if (round_of) {
      for (int64_t i = 0; i < na; i++)
        if (center[active_list[i]]) round_of[active_list[i]] = (int32_t)rounds;
      for (int64_t i = 0; i < ntouched; i++) round_of[touched[i]] = (int32_t)rounds;
    }

    /* 5. peel: clustered vertices leave; neighbours lose one degree each */
    for (int64_t i = 0; i < na; i++)
      if (center[active_list[i]]) cnt[resdeg[active_list[i]]]--;
    for (int64_t i = 0; i < ntouched; i++) cnt[resdeg[touched[i]]]--;
    for (int pass = 0; pass < 2; pass++) {
      int64_t len = pass == 0 ? na : ntouched;
      for (int64_t i = 0; i < len; i++) {
        int32_t x = pass == 0 ? active_list[i] : touched[i];
        if (pass == 0 && !center[x]) continue;
        for (int64_t e = off[x]; e < off[x + 1]; e++) {
          int32_t w = col[e];
          if (labels[w] != ORC_NONE) continue;
          cnt[resdeg[w]]--;
          resdeg[w]--;
          cnt[resdeg[w]]++;
        }
      }
    }

    if (rounds < trace_cap && trace) {
      orc_round *r = &trace[rounds];
      r->n_i = n_rem;
      r->delta_i = delta;
      r->b_i = b;
      r->r_i = cursor - 1;
      r->centers = ncenters;
      r->claimed = ntouched;
      r->conflicts = conflicts;
    }
    n_rem -= ncenters + ntouched;
    for (int64_t i = 0; i < na; i++) active[active_list[i]] = center[active_list[i]] = 0;
    for (int64_t i = 0; i < ntouched; i++) best[touched[i]] = ORC_INF;
    rounds++;
  }
done:
  free(rank);
  free(resdeg);
  free(best);
  free(active_list);
  free(touched);
  free(active);
  free(center);
  free(cnt);
  return rounds;
}

/*
 * Disagreements of a clustering on the complete signed graph whose positive
 * edges are G (Section 2, the correlation clustering objective): negative
 * pairs inside clusters plus positive edges across clusters,
 *   cost = sum_k C(s_k, 2) - m_in  +  (m - m_in).
 * labels must lie in [0, n).  Returns -1 on a bad label.
 */
int64_t orc_cost(int64_t n, const int64_t *off, const int32_t *col, const int32_t *labels) {
  int64_t *size = calloc((size_t)(n + 1), sizeof(int64_t));
  if (!size) return -2;
  for (int64_t v = 0; v < n; v++) {
    if (labels[v] < 0 || labels[v] >= n) {
      free(size);
      return -1;
    }
    size[labels[v]]++;
  }
  int64_t pairs_inside = 0;
  for (int64_t v = 0; v < n; v++) pairs_inside += size[v] * (size[v] - 1) / 2;
  free(size);
  int64_t twice_m_in = 0;
  for (int64_t v = 0; v < n; v++)
    for (int64_t e = off[v]; e < off[v + 1]; e++)
      if (labels[col[e]] == labels[v]) twice_m_in++;
  const int64_t m = off[n] / 2, m_in = twice_m_in / 2;
  return pairs_inside - m_in + (m - m_in);
}

/* The same objective counted pair by pair over all C(n,2) pairs (small n).
 * Adjacency is read by binary search in the sorted rows. */
static int orc_adjacent(const int64_t *off, const int32_t *col, int32_t u, int32_t w) {
  int64_t lo = off[u], hi = off[u + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] < w) lo = mid + 1;
    else hi = mid;
  }
  return lo < off[u + 1] && col[lo] == w;
}

int64_t orc_cost_pairs(int64_t n, const int64_t *off, const int32_t *col, const int32_t *labels) {
  int64_t cost = 0;
  for (int32_t u = 0; u < n; u++)
    for (int32_t w = u + 1; w < n; w++) {
      int same = labels[u] == labels[w], pos = orc_adjacent(off, col, u, w);
      if (same != pos) cost++;
    }
  return cost;
}

/*
 * KwikCluster's cost accumulated step by step, as in the bad-triangle lemma
 * (Lemma "algocost", Section 3.2 and its proof): when center v forms
 * C_v = {v} u (unclustered N(v)), it pays T_in = non-adjacent pairs inside
 * C_v plus T_out = positive edges from C_v to vertices still unclustered
 * outside it.  Returns the sum over all steps.
 */
int64_t orc_kc_stepwise_cost(int64_t n, const int64_t *off, const int32_t *col, const int32_t *order) {
  int32_t *lab = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *members = malloc(sizeof(int32_t) * (size_t)(n + 1));
  uint8_t *in_c = calloc((size_t)(n + 1), 1);
  if (!lab || !members || !in_c) return -2;
  for (int64_t v = 0; v < n; v++) lab[v] = ORC_NONE;
  int64_t total = 0;
  for (int64_t k = 0; k < n; k++) {
    int32_t v = order[k];
    if (lab[v] != ORC_NONE) continue;
    int64_t s = 0;
    members[s++] = v;
    for (int64_t e = off[v]; e < off[v + 1]; e++)
      if (lab[col[e]] == ORC_NONE) members[s++] = col[e];
    for (int64_t i = 0; i < s; i++) in_c[members[i]] = 1;
    int64_t twice_inside = 0, out = 0;
    for (int64_t i = 0; i < s; i++) {
      int32_t x = members[i];
      for (int64_t e = off[x]; e < off[x + 1]; e++) {
        int32_t y = col[e];
        if (in_c[y]) twice_inside++;
        else if (lab[y] == ORC_NONE) out++;
      }
    }
    total += s * (s - 1) / 2 - twice_inside / 2 + out;
    for (int64_t i = 0; i < s; i++) {
      lab[members[i]] = v;
      in_c[members[i]] = 0;
    }
  }
  free(lab);
  free(members);
  free(in_c);
  return total;
}

/*
 * Checks, at any size, that labels equal KwikCluster(G, pi) without running
 * it: with S = {v : labels[v] == v},
 *   (a) v is in S iff no neighbour in S has a smaller rank (S is the greedy
 *       maximal independent set of G in pi order);
 *   (b) every v outside S carries the id of its lowest-rank neighbour in S.
 * By induction over ranks, (a) fixes S uniquely and (b) is KwikCluster's
 * assignment (a vertex joins the first center in pi order adjacent to it).
 * Returns the number of vertices that break (a) or (b) (0 = equal), or a
 * negative code; *first_bad (if given) receives the first such vertex.
 */
int64_t orc_check_kc(int64_t n, const int64_t *off, const int32_t *col, const int32_t *order,
                     const int32_t *labels, int64_t *first_bad) {
  int32_t *rank = malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!rank) return ORC_ENOMEM;
  if (orc_invert(n, order, rank) != ORC_OK) {
    free(rank);
    return ORC_EINVAL;
  }
  int64_t bad = 0;
  if (first_bad) *first_bad = -1;
  for (int64_t v = 0; v < n; v++) {
    int ok = 1;
    if (labels[v] < 0 || labels[v] >= n) {
      ok = 0;
    } else {
      int32_t best = ORC_INF;
      for (int64_t e = off[v]; e < off[v + 1]; e++) {
        int32_t u = col[e];
        if (labels[u] == u && rank[u] < best) best = rank[u];
      }
      const int is_center = labels[v] == v;
      if (is_center) ok = !(best < rank[v]);
      else ok = (best < rank[v]) && labels[v] == order[best];
    }
    if (!ok) {
      if (first_bad && *first_bad < 0) *first_bad = v;
      bad++;
    }
  }
  free(rank);
  return bad;
}

/* =====================================================================
 * The paper's practical schedule (Implementation Details: "Estimating but
 * not computing Delta" and "Binomial sampling instead of fixed-size
 * batches").
 *
 * Readings taken here:
 *  - Delta-hat starts at Delta_0, the largest degree of G, and is halved
 *    every K = ceil((2/eps) ln(n log2(Delta_0) / delta)) rounds, with
 *    log2(Delta_0) read as max(log2 Delta_0, 1) and delta the failure
 *    probability of the high-probability bound (a parameter; the paper gives
 *    no value).  In round i, Delta-hat = Delta_0 / 2^floor(i/K).
 *  - Round i draws B_i ~ Binomial(N_i, p_i) with N_i = the pi positions not
 *    yet passed (the unprocessed suffix: unclustered and already-clustered
 *    vertices) and p_i = min(1, eps / Delta-hat) (1 when Delta_0 = 0), and
 *    takes the next B_i positions; the unclustered vertices among them are
 *    the active set.  B_i = 0 makes an empty round.
 *  - The loop runs while vertices are unclustered (Algorithm 2's while).
 *  - Round i's draw uses the uniform variates u_{i,0}, u_{i,1}, ...:
 *    u_{i,k} = (x >> 11) * 2^-53 with x the output number (i * 2^32 + k) of
 *    the SplitMix64 stream keyed by the seed (Steele, Lea and Flood, 2014).
 *  - The Binomial variate: B = N - Binomial(N, 1 - p) when p > 1/2;
 *    otherwise inversion by sequential search (the BINV algorithm of
 *    Kachitvichyanukul and Schmeiser, 1988) when N p < 10, and Hormann's
 *    transformed rejection with decomposition (BTRD, 1993) when N p >= 10.
 * ===================================================================== */

static uint64_t orc_splitmix(uint64_t key, uint64_t idx) {
  /* output number idx (from 0) of the SplitMix64 generator seeded with key */
  uint64_t z = key + (idx + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct {
  uint64_t seed, stream, k;
} orc_uniforms;

static double orc_uniform(orc_uniforms *g) {
  const uint64_t x = orc_splitmix(g->seed, (g->stream << 32) + g->k);
  g->k++;
  return (double)(x >> 11) * 0x1.0p-53;
}

/* Inversion: walk the probabilities P(0), P(1), ... (each from the last by
 * P(x) = P(x-1) (N - x + 1) p / (x q)) until they add up past u. */
static int64_t orc_binv(int64_t n, double p, orc_uniforms *g) {
  const double q = 1.0 - p;
  const double s = p / q;
  const double a = (double)(n + 1) * s;
  const double p0 = pow(q, (double)n);
  for (;;) {
    double u = orc_uniform(g);
    double f = p0;
    int64_t x = 0;
    while (u > f) {
      u -= f;
      x++;
      if (x > n) break;
      f *= a / (double)x - s;
    }
    if (x <= n) return x;
  }
}

/* Stirling-series remainder of log(k!): log k! - [(k+1/2) log(k+1) - (k+1) + log(2 pi)/2]. */
static double orc_stirling_rest(int64_t k) {
  if (k <= 9) {
    const double x = (double)k + 1.0;
    return lgamma(x) - ((double)k + 0.5) * log(x) + x - 0.91893853320467274178; /* log(2 pi) / 2 */
  }
  const double x = (double)k + 1.0;
  const double x2 = x * x;
  return (1.0 / 12.0 - (1.0 / 360.0 - 1.0 / 1260.0 / x2) / x2) / x;
}

/* BTRD: a uniform point under a hat built from a transformed uniform is
 * accepted at once in the hat's central part, else checked against f(k)/f(m)
 * (m the mode) -- by the product of ratios near the mode, by a squeeze on its
 * logarithm farther out, and finally by Stirling's formula. */
static int64_t orc_btrd(int64_t n, double p, orc_uniforms *g) {
  const double q = 1.0 - p;
  const double npq = (double)n * p * q;
  const double spq = sqrt(npq);
  const double b = 1.15 + 2.53 * spq;
  const double a = -0.0873 + 0.0248 * b + 0.01 * p;
  const double c = (double)n * p + 0.5;
  const double alpha = (2.83 + 5.1 / b) * spq;
  const double vr = 0.92 - 4.2 / b;
  const double urvr = 0.86 * vr;
  const int64_t m = (int64_t)floor((double)(n + 1) * p);
  const double r = p / q;
  const double nr = (double)(n + 1) * r;
  for (;;) {
    double v = orc_uniform(g);
    double u;
    if (v <= urvr) {
      u = v / vr - 0.43;
      return (int64_t)floor((2.0 * a / (0.5 - fabs(u)) + b) * u + c);
    }
    if (v >= vr) {
      u = orc_uniform(g) - 0.5;
    } else {
      u = v / vr - 0.93;
      u = (u < 0.0 ? -0.5 : 0.5) - u;
      v = orc_uniform(g) * vr;
    }
    const double us = 0.5 - fabs(u);
    const double kf = floor((2.0 * a / us + b) * u + c);
    if (kf < 0.0 || kf > (double)n) continue;
    const int64_t k = (int64_t)kf;
    v = v * alpha / (a / (us * us) + b);
    const int64_t km = k > m ? k - m : m - k;
    if (km <= 15) {
      double f = 1.0;
      if (m < k) {
        for (int64_t i = m + 1; i <= k; i++) f *= nr / (double)i - r;
      } else if (m > k) {
        for (int64_t i = k + 1; i <= m; i++) v *= nr / (double)i - r;
      }
      if (v <= f) return k;
      continue;
    }
    v = log(v);
    const double dkm = (double)km;
    const double rho = (dkm / npq) * (((dkm / 3.0 + 0.625) * dkm + 1.0 / 6.0) / npq + 0.5);
    const double t = -dkm * dkm / (2.0 * npq);
    if (v < t - rho) return k;
    if (v > t + rho) continue;
    const double nm = (double)(n - m + 1);
    const double h = ((double)m + 0.5) * log(((double)m + 1.0) / (r * nm)) + orc_stirling_rest(m) +
                     orc_stirling_rest(n - m);
    const double nk = (double)(n - k + 1);
    if (v <= h + (double)(n + 1) * log(nm / nk) + ((double)k + 0.5) * log(nk * r / ((double)k + 1.0)) -
                 orc_stirling_rest(k) - orc_stirling_rest(n - k))
      return k;
  }
}

/* One Binomial(n, p) variate from the uniforms of stream `stream`. */
int64_t orc_binomial(uint64_t seed, uint64_t stream, int64_t n, double p) {
  orc_uniforms g = {seed, stream, 0};
  if (n <= 0 || p <= 0.0) return 0;
  if (p >= 1.0) return n;
  if (p > 0.5) {
    const double pc = 1.0 - p;
    if ((double)n * pc < 10.0) return n - orc_binv(n, pc, &g);
    return n - orc_btrd(n, pc, &g);
  }
  if ((double)n * p < 10.0) return orc_binv(n, p, &g);
  return orc_btrd(n, p, &g);
}

/* K: rounds between two halvings of Delta-hat. */
int64_t orc_halving_period(int64_t n, int64_t delta0, double eps, double delta) {
  double lg = delta0 > 1 ? log2((double)delta0) : 1.0;
  if (lg < 1.0) lg = 1.0;
  const double arg = (double)(n > 1 ? n : 1) * lg / delta;
  const double k = ceil(2.0 / eps * log(arg));
  return k < 1.0 ? 1 : (int64_t)k;
}

/* p_i = min(1, eps / Delta-hat_i), Delta-hat_i = Delta_0 / 2^floor(i/K). */
static double orc_sample_prob(int64_t round, int64_t period, int64_t delta0, double eps) {
  if (delta0 <= 0) return 1.0;
  const int64_t h = round / period;
  if (h > 1000) return 1.0;
  const double pr = ldexp(eps / (double)delta0, (int)h);
  return pr < 1.0 ? pr : 1.0;
}

/*
 * The whole position schedule B_0, B_1, ... (it depends on n, Delta_0, eps,
 * delta and the seed only, never on the graph's state): drawn until the
 * positions run out.  Writes at most cap entries; returns the number of
 * rounds the schedule has (which may exceed cap), or a negative code.
 */
int64_t orc_binomial_schedule(int64_t n, int64_t delta0, double eps, double delta, uint64_t seed, int64_t *out,
                              int64_t cap) {
  if (n < 0 || delta0 < 0 || !(eps > 0.0) || !(delta > 0.0 && delta < 1.0)) return ORC_EINVAL;
  const int64_t period = orc_halving_period(n, delta0, eps, delta);
  int64_t left = n, i = 0;
  while (left > 0) {
    const int64_t b = orc_binomial(seed, (uint64_t)i, left, orc_sample_prob(i, period, delta0, eps));
    if (out && i < cap) out[i] = b;
    left -= b;
    i++;
  }
  return i;
}

/*
 * C4 / ClusterWild! with the practical schedule: round i takes the next B_i
 * positions of pi (drawn as above); the unclustered vertices among them are
 * the active set; election, claims and peeling as in orc_bsp.  The trace
 * records n_i, Delta-hat_i (rounded down), B_i (positions), the last
 * position taken, centers, claimed and blocked vertices.  Returns the number
 * of rounds or a negative code.
 */
/*
 * Rounds that take the next sched[i] positions of pi (the unclustered
 * vertices among them are active); the schedule must cover all n positions.
 * delta0 and period only fill the trace's delta_i field (delta0 >> (i /
 * period); pass period <= 0 for zeros).  Used with the Binomial draws below,
 * and with fixed position batches (64 positions a round is what one
 * asynchronous wave does when it runs alone).
 */
int64_t orc_bsp_positions(int algo, int64_t n, const int64_t *off, const int32_t *col, const int32_t *order,
                          const int64_t *sched, int64_t sched_len, int64_t delta0, int64_t period, int32_t *labels,
                          orc_round *trace, int64_t trace_cap, int32_t *round_of) {
  if ((algo != ORC_C4 && algo != ORC_CW) || n < 0 || sched_len < 0) return ORC_EINVAL;
  int64_t covered = 0;
  for (int64_t i = 0; i < sched_len; i++) {
    if (sched[i] < 0) return ORC_ETRACE;
    covered += sched[i];
  }
  if (covered < n) return ORC_ETRACE;
  const int64_t maxdeg = delta0;
  int32_t *rank = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *best = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *active_list = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *touched = malloc(sizeof(int32_t) * (size_t)(n + 1));
  uint8_t *active = calloc((size_t)(n + 1), 1);
  uint8_t *center = calloc((size_t)(n + 1), 1);
  int64_t rounds = ORC_ENOMEM;
  if (!rank || !best || !active_list || !touched || !active || !center) goto done;
  if (orc_invert(n, order, rank) != ORC_OK) {
    rounds = ORC_EINVAL;
    goto done;
  }
  for (int64_t v = 0; v < n; v++) {
    labels[v] = ORC_NONE;
    best[v] = ORC_INF;
  }
  int64_t n_rem = n, cursor = 0;
  rounds = 0;
  while (n_rem > 0) {
    /* the schedule covers every position, so it lasts */
    const int64_t b = sched[rounds] < n - cursor ? sched[rounds] : n - cursor;
    const int64_t h = period > 0 ? rounds / period : 63;
    const int64_t dhat = h >= 63 ? 0 : (maxdeg >> h);
    /* the next b positions; their unclustered vertices are active */
    int64_t na = 0;
    for (int64_t k = cursor; k < cursor + b; k++)
      if (labels[order[k]] == ORC_NONE) active_list[na++] = order[k];
    cursor += b;
    for (int64_t i = 0; i < na; i++) active[active_list[i]] = 1;
    int64_t conflicts = 0;
    for (int64_t i = 0; i < na; i++) {
      int32_t a = active_list[i];
      for (int64_t e = off[a]; e < off[a + 1]; e++)
        if (active[col[e]] && rank[col[e]] < rank[a]) {
          conflicts++;
          break;
        }
    }
    int64_t ncenters = 0;
    for (int64_t i = 0; i < na; i++) {
      int32_t a = active_list[i];
      int ok = 1;
      if (algo == ORC_C4) {
        for (int64_t e = off[a]; e < off[a + 1]; e++)
          if (center[col[e]]) {
            ok = 0;
            break;
          }
      }
      center[a] = (uint8_t)ok;
      ncenters += ok;
    }
    int64_t ntouched = 0;
    for (int64_t i = 0; i < na; i++) {
      int32_t c = active_list[i];
      if (!center[c]) continue;
      for (int64_t e = off[c]; e < off[c + 1]; e++) {
        int32_t u = col[e];
        if (labels[u] != ORC_NONE || center[u]) continue;
        if (algo == ORC_CW && active[u]) continue;
        if (best[u] == ORC_INF) touched[ntouched++] = u;
        if (rank[c] < best[u]) best[u] = rank[c];
      }
    }
    for (int64_t i = 0; i < na; i++)
      if (center[active_list[i]]) labels[active_list[i]] = active_list[i];
    for (int64_t i = 0; i < ntouched; i++) labels[touched[i]] = order[best[touched[i]]];
    if (round_of) {
      for (int64_t i = 0; i < na; i++)
        if (center[active_list[i]]) round_of[active_list[i]] = (int32_t)rounds;
      for (int64_t i = 0; i < ntouched; i++) round_of[touched[i]] = (int32_t)rounds;
    }
    if (rounds < trace_cap && trace) {
      orc_round *r = &trace[rounds];
      r->n_i = n_rem;
      r->delta_i = dhat;
      r->b_i = b;
      r->r_i = cursor - 1;
      r->centers = ncenters;
      r->claimed = ntouched;
      r->conflicts = conflicts;
    }
    n_rem -= ncenters + ntouched;
    for (int64_t i = 0; i < na; i++) active[active_list[i]] = center[active_list[i]] = 0;
    for (int64_t i = 0; i < ntouched; i++) best[touched[i]] = ORC_INF;
    rounds++;
  }
done:
  free(rank);
  free(best);
  free(active_list);
  free(touched);
  free(active);
  free(center);
  return rounds;
}

int64_t orc_bsp_binomial(int algo, int64_t n, const int64_t *off, const int32_t *col, const int32_t *order,
                         double eps, double delta, uint64_t seed, int32_t *labels, orc_round *trace,
                         int64_t trace_cap, int32_t *round_of) {
  if ((algo != ORC_C4 && algo != ORC_CW) || n < 0) return ORC_EINVAL;
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; v++)
    if (off[v + 1] - off[v] > maxdeg) maxdeg = off[v + 1] - off[v];
  const int64_t len = orc_binomial_schedule(n, maxdeg, eps, delta, seed, NULL, 0);
  if (len < 0) return len;
  int64_t *sched = malloc(sizeof(int64_t) * (size_t)(len + 1));
  if (!sched) return ORC_ENOMEM;
  orc_binomial_schedule(n, maxdeg, eps, delta, seed, sched, len + 1);
  const int64_t rounds = orc_bsp_positions(algo, n, off, col, order, sched, len, maxdeg,
                                           orc_halving_period(n, maxdeg, eps, delta), labels, trace, trace_cap,
                                           round_of);
  free(sched);
  return rounds;
}
