// cc_launch.h -- host-side entry points of the kernels (C++ linkage, internal).
#pragma once
#include <hip/hip_runtime.h>

#include "cc_device.h"

namespace ccd {

struct LaunchShape {
  unsigned select_grid;  // workgroups of the active-set scan
  unsigned edge_grid;    // workgroups of the edge-balanced passes
  unsigned vertex_grid;  // workgroups of per-vertex list passes
  unsigned scan_grid;    // unused
  int exact_seen;        // the host saw the run switch to exact degrees
};

hipError_t launch_init(const Ws &w, const unsigned *lvl_init_cnt, hipStream_t s);
hipError_t launch_round(const Ws &w, hipStream_t s, const LaunchShape &ls);
hipError_t launch_finalize(const Ws &w, int32_t *labels, hipStream_t s);

// Graph set-up: row-weight prefix wall[n+1] (the "all rows" list of the
// edge-balanced walk), per-row graph ids (batches), column-range check and,
// with validate, the symmetry / self-loop / duplicate checks.  *err receives
// the smallest failing cc_status code (it must hold 0x7fffffff beforehand).
hipError_t launch_graph_setup(const int64_t *off, const int32_t *col, int64_t n, const int64_t *vtx_ptr,
                              int32_t num_graphs, int32_t *gid, int64_t *wall, int64_t *blocksum,
                              int validate, int *err, hipStream_t s);

// Bucket levels of the degree bounds: count[k] = vertices with
// floor(log2(deg)) == k (k >= LVL_MIN), and the maximum degree.
hipError_t launch_level_count(const int64_t *off, int64_t n, unsigned *count, int *max_deg, hipStream_t s);
// Places every vertex with deg >= DSW at lvl[lvl_off[k] + i], k = its level.
hipError_t launch_level_fill(const int64_t *off, int64_t n, const int64_t *lvl_off, unsigned *cursor,
                             int32_t *lvl, hipStream_t s);

// Batched C4 / ClusterWild!: one persistent launch over many small graphs.
struct BatchLaunch {
  const int64_t *off;
  const int32_t *col;
  const int64_t *vtx_ptr;
  const int32_t *order;
  int32_t *labels;
  const int32_t *queue;
  int32_t n_big, n_quad, num_graphs, cap_big, cap_quad, cap_wave;
  unsigned *heads;
  int32_t *rounds;
  unsigned long long *stat;
  int *err;
  int algo;
  int64_t eps_q;
  int block, grid;
};
hipError_t launch_batched(const BatchLaunch &bl, hipStream_t s);
size_t batched_lds_bytes(int block, int cap_big, int cap_quad, int cap_wave);
hipError_t batched_max_grid(int block, size_t lds, int *grid);

// Internal renumbering of a single graph (hubs first): perm (input id ->
// internal id), iperm, and the renumbered CSR roff / rcol.  count: 2 x
// (NLVL + 1) unsigned scratch, bin_off: NLVL + 1 int64, rdeg: n int64,
// blocksum: n / (4 BS) + 2 int64.  On the host: *first_low = the first
// internal id of degree below DSW, *first_isolated = the first of degree 0
// (degrees fall with the id level by level, so each is the start of a range).
hipError_t launch_relabel(const int64_t *off, const int32_t *col, const int64_t *wall, int64_t n, unsigned *count,
                          int64_t *bin_off_dev, int32_t *perm, int32_t *iperm, int64_t *rdeg, int64_t *roff,
                          int64_t *blocksum, int32_t *rcol, int64_t *first_low, int64_t *first_isolated,
                          hipStream_t s);

// pi mapped into internal ids and checked as a permutation, in bucketed
// passes (cc_order.hip) for OM_MIN_N < n <= OM_MAX_BUCKETS * OM_SIZE; other
// sizes gather directly.  Bucket kb of positions and bucket vb of ids hold
// OM_SIZE each.  The scratch (order_map_bytes(n), one device allocation) is
// laid out by order_map_layout.  A failed check sets ERR_PERM in ctrl.
constexpr int OM_SHIFT = 15;
constexpr int64_t OM_SIZE = int64_t(1) << OM_SHIFT;
constexpr int OM_MAX_BUCKETS = 2048;
constexpr int64_t OM_MIN_N = int64_t(1) << 22;
struct OrderMap {
  int nk, nv;               // position buckets, id buckets
  int nkt, nvt;             // 64-bucket tiles of each
  unsigned *cnt;            // [nk][nv] entries of kb in vb; then where (kb, vb) starts in ent, by row
  unsigned *pt;             // [nv][nk] where (kb, vb) starts in ent, by column
  unsigned *qt;             // [nv][nk] where (kb, vb) starts in pent, by column
  unsigned *csum, *rsum;    // [nkt][nv] column and [nvt][nk] row sums of 64 x 64 tiles
  unsigned *vstart;         // [nv + 1] start of each id bucket in ent
  unsigned *ent;            // [n] k low bits | (id low bits << OM_SHIFT), by id bucket, then kb
  unsigned long long *pent; // [n] (internal id << OM_SHIFT) | k low bits, by position bucket
};
bool order_map_applies(int64_t n);
size_t order_map_bytes(int64_t n);
OrderMap order_map_layout(int64_t n, void *base);
// rank (optional): also rank[iorder[k]] = k, the inverse of pi in internal ids.
hipError_t launch_order_map(const OrderMap &m, const int32_t *order_in, const int32_t *perm, int64_t n,
                            int32_t *iorder, Ctrl *ctrl, hipStream_t s, int32_t *rank = nullptr);

// Asynchronous C4 / ClusterWild! (Algorithm 3): one persistent launch, no
// rounds.  rank and lab are workspace arrays of n; order is pi in internal
// ids (written by the launch from order_in through perm into iorder).
struct AsyncArgs {
  const int64_t *off;
  const int32_t *col;
  int64_t n;
  int64_t iso_start;
  const int32_t *order;
  int32_t *rank;
  int32_t *lab;
  Ctrl *ctrl;
  int32_t *big_v, *big_p;  // C4 centers whose claims are spread over the device (vertex, rank)
  int64_t big_cap;
};
// waves > 0 limits the launch to that many waves (1: pi strictly in order,
// 64 positions at a time); 0 fills the device.  ev0 / ev1 (optional) bracket
// the asynchronous kernel itself.
// om: the bucketed mapping of pi when it applies to this n, else nullptr.
hipError_t launch_async(const AsyncArgs &a, int algo, const int32_t *order_in, const int32_t *perm, int32_t *iorder,
                        int32_t *labels, int waves, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                        const OrderMap *om);

// Learned-policy network: inference over a batch, one training step.
int mlp_grad_blocks(int n);
// The current device's static partial-row buffer (no allocation): its
// device address and how many rows it holds.
hipError_t mlp_scratch(float **ptr, int *rows);
hipError_t launch_mlp_forward(const float *p, const float *x, int n, float *y, hipStream_t s);
hipError_t launch_mlp_train_step(float *p, float *m, float *v, const float *x, const float *t, int n, long long step,
                                 float lr, float *partial, int nblk, float *grad, float *loss, hipStream_t s);

// Disagreement cost per graph: acc[2g] = pairs inside clusters, acc[2g+1] =
// same-label adjacency entries (2 m_in); size is scratch [n].
hipError_t launch_cost(const int64_t *off, const int32_t *col, const int64_t *wall, int64_t n,
                       const int64_t *vtx_ptr, const int32_t *gid, const int32_t *labels, int32_t *size,
                       long long *acc, int32_t num_graphs, int *err, hipStream_t s);

}  // namespace ccd
