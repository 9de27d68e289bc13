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
