/*
 * cc.h -- C ABI of the MI355X (gfx950) correlation-clustering library:
 * bulk-synchronous C4 and ClusterWild! (Pan, Papailiopoulos, Oymak, Recht,
 * Ramchandran, Jordan, "Parallel Correlation Clustering on Big Graphs",
 * arXiv 1507.05086).
 *
 * Problem (Section 2, "Correlation Clustering"): a complete graph on n
 * vertices whose pairs are either positive (similar) or negative.  Only the
 * positive edges are passed in; every other pair is negative.  A clustering
 * is scored by its disagreements: positive edges cut between clusters plus
 * negative pairs placed inside a cluster.
 *
 * Conventions shared by every call:
 *  - The positive graph is symmetric CSR: offsets int64[n+1], cols
 *    int32[offsets[n]]; row v lists the positive neighbours N(v) in strictly
 *    ascending order; no self-loops, no duplicates, every edge in both rows.
 *    n < 2^31 and offsets[n] < 2^33.
 *  - The order pi is passed as `order`, order[k] = the vertex of rank k (the
 *    position-to-vertex reading of pi in Algorithm 1); it must be a
 *    permutation of 0..n-1.
 *  - Labels are int32[n]: labels[v] = the vertex id of v's cluster center
 *    (the paper's clusterID holds the center's rank pi(center); the id is
 *    the same information, one-to-one).
 *  - `stream` is a hipStream_t passed as an opaque pointer (NULL = the null
 *    stream).  Work is queued on it and every call returns after that work
 *    has finished, so the status it returns covers the GPU work.
 *  - Pointers are host pointers unless a flag says they are device pointers.
 *    Caller-owned buffers are only read or written during the call.
 *  - No call throws; each returns a cc_status.  On failure the outputs are
 *    left untouched and cc_last_error() describes the failure.
 *  - Calls that use the same cc_graph must not overlap (they share its
 *    device workspace); different graphs may be used from different threads.
 */
#ifndef CC_H_
#define CC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define CC_API __attribute__((visibility("default")))
#else
#define CC_API
#endif

typedef struct cc_graph cc_graph; /* opaque: device CSR + run workspace */

typedef enum cc_status {
  CC_OK = 0,
  CC_ERR_INVALID_ARG = 1,     /* bad pointer, size, flag or eps */
  CC_ERR_NOT_SYMMETRIC = 2,   /* edge (u,v) without (v,u) (CC_VALIDATE) */
  CC_ERR_SELF_LOOP = 3,       /* edge (v,v) (CC_VALIDATE) */
  CC_ERR_DUPLICATE_EDGE = 4,  /* repeated or unsorted entry in a row (CC_VALIDATE) */
  CC_ERR_NOT_PERMUTATION = 5, /* order is not a permutation of 0..n-1 */
  CC_ERR_OUT_OF_MEMORY = 6,   /* device or host allocation failed */
  CC_ERR_DEVICE = 7,          /* a HIP call failed */
  CC_ERR_NO_PROGRESS = 8,     /* round loop exceeded its round limit or a bounded wait expired */
  CC_ERR_POLICY = 9,          /* invalid epsilon-policy parameters or schedule */
  CC_ERR_OUT_OF_RANGE = 10    /* a column index outside 0..n-1 (always checked) */
} cc_status;

enum cc_flags {
  CC_VALIDATE = 1u,         /* graph: check symmetry, self-loops, duplicates, sort order */
  CC_INPUT_ON_DEVICE = 2u,  /* offsets/cols (graph) or order (run) are device pointers */
  CC_BORROW = 4u,           /* graph: keep the caller's device offsets/cols, no copy */
  CC_OUTPUT_ON_DEVICE = 8u  /* labels (run) are a device pointer */
};

/* One record per round of the bulk-synchronous loop (Algorithm 2). */
typedef struct cc_round_record {
  int64_t n_i;       /* vertices unclustered when the round starts */
  int64_t delta_i;   /* maximum remaining positive degree when it starts */
  int64_t b_i;       /* active-set size used */
  int64_t r_i;       /* rank (position in pi) of the last active vertex */
  int64_t centers;   /* cluster centers created */
  int64_t claimed;   /* non-center vertices clustered */
  int64_t conflicts; /* active vertices with an earlier-ranked active neighbour */
  double eps_used;   /* epsilon that produced b_i (b_i as given for a schedule) */
  int64_t t_ns;      /* device time of the round, nanoseconds */
} cc_round_record;

/* Optional statistics of a run (pass NULL to skip). */
typedef struct cc_run_stats {
  int64_t rounds;        /* out: rounds executed */
  int64_t scanned_elect; /* out: adjacency entries read by the C4 election (listed active rows) */
  int64_t scanned_claim; /* out: adjacency entries read by claims (listed centers' rows) */
  int64_t scanned_peel;  /* out: adjacency entries read by peeling */
  int64_t scanned_delta; /* out: adjacency entries read to refresh remaining degrees (Delta) */
  int64_t blocked;       /* out: sum of conflicts over rounds */
  int64_t atomics;       /* out: atomic read-modify-writes (claims, degree decrements, bit clears) */
  double loop_ms;        /* out: device time of the round loop (HIP events on `stream`) */
  int32_t policy_fallback; /* out: 1 if the learned policy fell back to the fixed rule */
  int32_t truncated;       /* out: 1 if more rounds ran than trace_capacity */
  cc_round_record *trace;  /* in: host buffer of trace_capacity records, or NULL */
  int64_t trace_capacity;  /* in */
  int32_t *graph_rounds;   /* in: host int32[num_graphs] receiving each graph's rounds
                              (batches; rounds then holds their maximum), or NULL */
  int64_t max_rounds;      /* in: 0 runs to completion; k > 0 stops after k rounds (single
                              graphs only): a partial run whose still-unclustered vertices
                              get label -1, used to measure one round from a replayed state */
  int64_t fault_round;     /* in: 0 in normal use.  Test hook of the error path (single
                              graphs): k > 0 makes the device report an error at the end of
                              round k, as a failing round would, so the call returns
                              CC_ERR_DEVICE with every kernel having exited normally */
  int64_t async_waves;     /* in: asynchronous calls only.  0 fills the device; k > 0 runs
                              k waves (1: pi strictly in order, 64 positions at a time, which
                              makes ClusterWild!'s interleaving reproducible) */
} cc_run_stats;

/*
 * Upload (or borrow) a positive-edge graph.
 *   num_graphs  1 for one graph; >1 for a batch of independent graphs whose
 *               rows are stacked: vtx_ptr[num_graphs+1] (host) gives each
 *               graph's first row, offsets index the shared cols array, and
 *               cols hold LOCAL ids (0..n_g-1) of the same graph.
 *               vtx_ptr may be NULL when num_graphs == 1.
 *   n_total     total rows.
 *   offsets, cols  CSR as described above; host pointers, or device
 *               pointers with CC_INPUT_ON_DEVICE (copied) or CC_BORROW (kept;
 *               the caller keeps them alive and unchanged until destroy).
 *   flags       CC_VALIDATE / CC_INPUT_ON_DEVICE / CC_BORROW.
 *   out         receives the handle.
 * Column ranges are always checked (CC_ERR_OUT_OF_RANGE); CC_VALIDATE adds
 * the symmetry, self-loop and duplicate/sort checks.
 * Device memory: a single graph (num_graphs == 1) also keeps a renumbered
 * copy of its CSR (one more column array, 24 bytes per vertex), and its
 * first run allocates a workspace of one column array plus about 170 bytes
 * per vertex (about 20 GB at n = 2^26 with 2.1 G stored entries), held until
 * destroy.  An allocation failure returns CC_ERR_OUT_OF_MEMORY.
 */
CC_API int32_t cc_graph_from_csr(int32_t num_graphs, const int64_t *vtx_ptr, int64_t n_total,
                          const int64_t *offsets, const int32_t *cols, uint32_t flags,
                          void *stream, cc_graph **out);

/* Release the handle and its device memory (borrowed CSR is not freed). */
CC_API int32_t cc_graph_destroy(cc_graph *g);

/* Rows and stored entries of a handle (either pointer may be NULL). */
CC_API int32_t cc_graph_info(const cc_graph *g, int64_t *n_total, int64_t *nnz, int32_t *num_graphs);

/*
 * C4 (Algorithm 2, concurrency-control branch): rounds of
 *   Delta_i = max remaining degree;  A = next B_i = ceil(eps n_i / Delta_i)
 *   unclustered vertices of pi;  an active vertex becomes a center iff no
 *   earlier-ranked active neighbour is one (concurrency rule 1);  every
 *   other unclustered neighbour of a center joins the adjacent center of
 *   lowest rank (rule 2);  clustered vertices are peeled.
 * Its labels equal serial KwikCluster's under the same pi (Section 3,
 * "C4 is serializable"), whatever the schedule.
 *   order   int32[n_total]: pi (per graph, local ids, for a batch).
 *   eps     0 < eps <= 1000, used in millionths: B_i = ceil(round(eps*1e6) *
 *           n_i / (1e6 * Delta_i)), kept in [1, n_i]; B_i = n_i when
 *           Delta_i = 0.  The process-wide policy (cc_set_eps_policy) may
 *           replace this rule.
 *   labels  int32[n_total] out (center ids; local ids for a batch).
 *   stats   optional.
 *   flags   CC_INPUT_ON_DEVICE (order), CC_OUTPUT_ON_DEVICE (labels).
 */
CC_API int32_t cc_c4(const cc_graph *g, const int32_t *order, double eps, int32_t *labels,
              cc_run_stats *stats, uint32_t flags, void *stream);

/*
 * ClusterWild! (Algorithm 2, coordination-free branch): the same rounds,
 * but every active vertex is a center (rule 1 is ignored) and centers claim
 * only their non-active unclustered neighbours (createCluster's
 * Gamma(v) \ A), the lowest-rank center winning.  Same arguments as cc_c4.
 */
CC_API int32_t cc_clusterwild(const cc_graph *g, const int32_t *order, double eps, int32_t *labels,
                       cc_run_stats *stats, uint32_t flags, void *stream);

/*
 * Asynchronous C4 and ClusterWild! (Algorithm 3 and section "BSP Algorithms
 * as a Proxy for Asynchronous Algorithms"): the same vertex rules without
 * rounds or bulk synchronisation, and without eps.  One persistent launch:
 * waves take the next 64 positions of pi from a shared counter.  C4 makes a
 * vertex still unclustered when reached a center iff no earlier-ranked
 * neighbour is one, waiting for earlier neighbours still being decided
 * (isCenter); its labels equal KwikCluster's, as the round loop's do.
 * ClusterWild! makes every vertex still unclustered when reached a center,
 * with no waiting; its labels depend on how the waves interleave (a center
 * never changes cluster; a claimed vertex joins the lowest-rank center that
 * claims it).  Single graphs only; order, labels, flags and errors as for
 * cc_c4.  stats: rounds = 0, scanned_elect = adjacency entries read by
 * isCenter, scanned_claim = entries read by claims, atomics = claims that
 * lowered a label, loop_ms = the asynchronous kernel's time; async_waves as
 * described above; max_rounds and fault_round must be 0.
 */
CC_API int32_t cc_c4_async(const cc_graph *g, const int32_t *order, int32_t *labels, cc_run_stats *stats,
                           uint32_t flags, void *stream);
CC_API int32_t cc_clusterwild_async(const cc_graph *g, const int32_t *order, int32_t *labels, cc_run_stats *stats,
                                    uint32_t flags, void *stream);

/*
 * Batches (num_graphs > 1).  cc_c4 and cc_clusterwild cluster every graph of
 * a batch in ONE persistent kernel launch: a group of threads takes a graph
 * from a queue (largest first), keeps its vertex state in LDS and runs the
 * whole round loop of Algorithm 2 on it with the fixed eps rule, then takes
 * the next graph.  Graphs of at most `wave_max_n` vertices run on a single
 * wave (several per workgroup); with block >= 512, graphs of at most
 * `quad_max_n` vertices run on a sub-group of 4 waves (block / 256 graphs
 * per workgroup); larger ones on the whole workgroup of `block` threads.
 * Each graph may hold at most CC_BATCH_MAX_N vertices (the LDS of one
 * workgroup).  Labels are per graph, local ids; per-graph rounds come
 * back in cc_run_stats.graph_rounds; no per-round trace is recorded.  A
 * batch run with a LEARNED or TRACE policy set fails with CC_ERR_POLICY.
 */
#define CC_BATCH_MAX_N 7168
enum cc_algo { CC_ALGO_C4 = 0, CC_ALGO_CLUSTERWILD = 1 };

typedef struct cc_batch_config {
  int32_t block;      /* threads per workgroup: 256, 512 or 1024 */
  int32_t wave_max_n; /* graphs with n_g <= wave_max_n run one per wave (0: none) */
  int32_t quad_max_n; /* block >= 512: graphs with wave_max_n < n_g <= quad_max_n run one
                         per 4-wave sub-group (0: none) */
  int32_t reserved;   /* 0 */
  double ms;          /* cc_batch_autotune: best measured time of one launch */
} cc_batch_config;

/*
 * Fix the launch shape of a batch handle (cfg->ms is ignored).  Without a
 * call, a handle uses the shape cc_batch_autotune last chose for a batch of
 * the same size class (number of graphs, largest and median graph, rounded
 * up to powers of two, and the device) in this process, else a built-in
 * default.  CC_ERR_INVALID_ARG if the shape does not fit the device's LDS.
 */
CC_API int32_t cc_batch_set_config(cc_graph *g, const cc_batch_config *cfg);

/*
 * Time every launch shape that fits (block in {256, 512, 1024} x ladders of
 * wave_max_n and quad_max_n values) on this batch with `algo` (cc_algo),
 * `order` and `eps` (as for cc_c4; flags: CC_INPUT_ON_DEVICE only), keep the fastest for the
 * handle and for its size class, and return it in *best (may be NULL).
 * Runs the batch three times per shape; labels are not returned.
 */
CC_API int32_t cc_batch_autotune(cc_graph *g, int32_t algo, const int32_t *order, double eps,
                                 uint32_t flags, void *stream, cc_batch_config *best);

/*
 * Disagreements of a clustering (the objective of Section 2):
 *   cost = sum over clusters of C(size, 2) + m - 2 * m_in,
 * with m positive edges and m_in of them inside clusters.
 *   labels  int32[n_total], each in 0..n_g-1 (any cluster ids, not only
 *           centers); device pointer with CC_INPUT_ON_DEVICE.
 *   cost    int64[num_graphs] host output, one value per graph.
 */
CC_API int32_t cc_cost(const cc_graph *g, const int32_t *labels, int64_t *cost, uint32_t flags,
                void *stream);

/* Epsilon policies for the active-set size of each round. */
enum cc_eps_policy_kind {
  CC_EPS_FIXED = 0,   /* the paper's rule with the per-call eps (default) */
  CC_EPS_LEARNED = 1, /* params: 6->64->1 MLP, CC_MLP_PARAMS floats (see below) */
  CC_EPS_TRACE = 2,   /* params: int64 B_i schedule (each >= 1); rounds past its end use the fixed rule */
  CC_EPS_BINOMIAL = 3 /* params: cc_binomial_params; the paper's practical schedule (below) */
};

/*
 * The practical schedule of Implementation Details ("Estimating but not
 * computing Delta", "Binomial sampling instead of fixed-size batches"): no
 * remaining degree is kept.  Delta-hat starts at Delta_0 (the largest degree)
 * and halves every K = ceil((2/eps) ln(n max(log2 Delta_0, 1) / delta))
 * rounds; round i draws B_i ~ Binomial(N_i, min(1, eps / Delta-hat_i)), N_i
 * the pi positions not yet passed, and its active set is the unclustered
 * vertices among the next B_i positions (B_i may be 0: an empty round).  C4's
 * labels are still KwikCluster's.  The B_i sequence depends on (n, Delta_0,
 * eps, delta, seed) only; the library draws it on the host before the loop
 * (cc_binomial_schedule shows it).  Round i's variates come from SplitMix64
 * outputs i*2^32, i*2^32 + 1, ... of `seed`; Binomial(N, p) is N minus a
 * Binomial(N, 1-p) draw for p > 1/2, inversion (BINV) for N p < 10, else
 * Hormann's BTRD.  In the trace, delta_i is floor(Delta-hat_i), b_i the
 * positions taken and r_i the last of them.  Single graphs only.
 */
typedef struct cc_binomial_params {
  uint64_t seed; /* seed of the variates */
  double delta;  /* failure probability in K, 0 < delta < 1 (the paper gives no value; 0.1 is used here) */
} cc_binomial_params;

/*
 * The practical schedule on the host: B_0, B_1, ... until the n positions
 * are used up.  out (host) receives the first min(capacity, rounds) entries;
 * *rounds (if not NULL) the schedule's length, *period (if not NULL) K.
 * CC_ERR_INVALID_ARG for n < 0, delta0 < 0, eps outside (0, 1000] or delta
 * outside (0, 1).  Touches no device.
 */
CC_API int32_t cc_binomial_schedule(int64_t n, int64_t delta0, double eps, uint64_t seed, double delta,
                                    int64_t *out, int64_t capacity, int64_t *rounds, int64_t *period);

/*
 * Set the process-wide policy (not thread-safe; call between runs).
 * LEARNED: params = float32[CC_MLP_PARAMS] laid out W1[64][6] row-major, b1[64],
 *   w2[64], b2; features per round x = [ln n_i, ln max(Delta_i,1),
 *   conflicts/B, claimed/n, eps, i] of the previous round (zeros and the
 *   per-call eps in round 0); eps_i = clamp(exp(w2 . relu(W1 x + b1) + b2),
 *   eps_min, eps_max); a non-finite output falls back to the fixed rule.
 * TRACE: params = int64[nbytes/8] schedule of B_i.
 * BINOMIAL: params = one cc_binomial_params (nbytes = its size).
 * FIXED: params ignored.
 */
CC_API int32_t cc_set_eps_policy(int32_t kind, const void *params, size_t nbytes, double eps_min,
                          double eps_max);

#define CC_MLP_IN 6
#define CC_MLP_HIDDEN 64
#define CC_MLP_PARAMS (CC_MLP_HIDDEN * CC_MLP_IN + CC_MLP_HIDDEN + CC_MLP_HIDDEN + 1)

/*
 * Training and batch inference of the learned policy's network (float32,
 * parameter layout as for CC_EPS_LEARNED).  The paper fixes eps for a run;
 * this network and its training are an addition.  All pointers are DEVICE
 * pointers; x is float32[n][CC_MLP_IN] row-major (the per-round features of
 * cc_set_eps_policy).  Work is queued on `stream`; the call returns after it
 * has finished.  0 <= n < 2^31.
 *
 * cc_mlp_forward: y[i] = w2 . relu(W1 x_i + b1) + b2.
 */
CC_API int32_t cc_mlp_forward(const float *params, const float *x, int64_t n, float *y, void *stream);

/*
 * cc_mlp_train_step: the gradient of L = mean_i (y_i - target_i)^2 at
 * `params` (backpropagation; written to grad[CC_MLP_PARAMS] unless NULL, L
 * to *loss unless NULL), then, when lr > 0, one Adam step (beta1 = 0.9,
 * beta2 = 0.999, eps = 1e-8, bias correction with step >= 1) that updates
 * params, adam_m and adam_v (float32[CC_MLP_PARAMS] each; zero them before
 * step 1).  lr == 0 computes the gradient only.
 */
CC_API int32_t cc_mlp_train_step(float *params, float *adam_m, float *adam_v, const float *x, const float *target,
                                 int64_t n, int64_t step, float lr, float *grad, float *loss, void *stream);

/*
 * cc_mlp_train_step without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight training loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * cc_mlp_train_step; the partial gradient rows (one per workgroup of the
 * gradient kernel, at most 1024, about 2 MB) live in a static device buffer
 * that each device holds until the process ends.  Calls that overlap on one
 * device share that buffer and race: serialise them.  CC_ERR_INVALID_ARG if
 * a gradient would need more partial rows than the buffer holds (it never
 * does: the kernel uses at most 1024 workgroups).
 */
CC_API int32_t cc_mlp_train_step_noalloc(float *params, float *adam_m, float *adam_v, const float *x,
                                         const float *target, int64_t n, int64_t step, float lr, float *grad,
                                         float *loss, void *stream);

/* Text of the calling thread's last failure ("" if none). */
CC_API const char *cc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CC_H_ */
