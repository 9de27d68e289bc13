// cc_device.h -- device-side data layout and helpers of the C4 / ClusterWild!
// round loop (arXiv 1507.05086, Algorithm 2) on gfx950.
//
// Memory layout of a run (all in HBM, sized for one graph of n vertices and
// nnz stored adjacency entries):
//   rank   int32[n]   position of each vertex in pi (rank = order^-1)
//   lab    int32[n]   clusterID: rank of the vertex's center, INF while unclustered
//   ub     int32[n]   remaining-degree bound: an upper bound while Delta is
//                     large, the exact remaining degree once the run switches
//   unc    uint32[n/32] one bit per vertex, set while it is unclustered (8 MB at
//                     2^26 vertices: gathers stay in L2 / the Infinity Cache)
//   state  uint8[n]   ACTIVE / CENTER / NONCENTER marks of the current round
//   flag   uint8[n]   per-round scratch mark (blocked / waiting / conflict)
//   work lists: active set, centers, newly clustered, rescans; each a vertex
//   array plus the exclusive prefix of the row weights max(deg, 1), so that
//   adjacency passes can hand out equal numbers of entries to every workgroup.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ccd {

constexpr int BS = 256;             // threads per workgroup (4 wave64s)
constexpr int WAVES = BS / 64;
constexpr int IPT = 4;              // adjacency items per thread per tile
constexpr int TW = BS * IPT;        // adjacency items per tile
constexpr int SIPT = 8;            // pi positions per thread in the active-set scan
constexpr int SEL_BS = 512;         // threads of an active-set scan workgroup
constexpr int TSEL = SEL_BS * SIPT; // pi positions per scan tile
constexpr int32_t INF = 0x7fffffff;

enum : uint8_t { UNCL = 0, ACTIVE = 1, CENTER = 2, NONCENTER = 3, ORDER_SEEN = 4 };
constexpr int DSW = 64;            // bounds below this never need a bucket entry
constexpr int LVL_MIN = 6;         // log2(DSW): lowest bucket level of the bound buckets
constexpr int NLVL = 32;           // bucket levels (level = floor(log2(ub)))
constexpr int DITER = 3;           // band passes of the lazy Delta search per round
constexpr int SWL = 128;           // a band floor below this switches to exact degrees
constexpr int HLDS = 256;          // degree-histogram bins kept per workgroup in LDS
// pass j rescans candidates with bound >= ceil(BAND_j * T_j)
__host__ __device__ inline float band_factor(int pass) { return pass == 0 ? 0.7f : (pass == 1 ? 0.3f : 0.05f); }
enum : int { ALGO_C4 = 0, ALGO_CW = 1 };
enum : int { POL_FIXED = 0, POL_LEARNED = 1, POL_TRACE = 2, POL_BINOMIAL = 3 };
enum : int { ERR_NONE = 0, ERR_PERM = 5, ERR_NO_PROGRESS = 8, ERR_OVERFLOW = 11, ERR_LABEL = 12, ERR_INJECTED = 13 };
enum : int { PHASE_LAZY = 0, PHASE_EXACT = 1 };

// A list is packed in one 64-bit counter: (total weight << 31) | count, so a
// single atomic reserves both a slot range and its weight range, and the
// stored weight offsets come out sorted in slot order.
__host__ __device__ inline unsigned long long pk(int64_t work, int64_t cnt) {
  return ((unsigned long long)work << 31) | (unsigned long long)cnt;
}
__host__ __device__ inline int64_t pk_cnt(unsigned long long p) { return (int64_t)(p & 0x7fffffffULL); }
__host__ __device__ inline int64_t pk_work(unsigned long long p) { return (int64_t)(p >> 31); }

struct RoundRec {  // mirrors cc_round_record
  int64_t n_i, delta_i, b_i, r_i, centers, claimed, conflicts;
  double eps_used;
  int64_t t_ns;  // raw wall-clock ticks here; the host converts
};

// The fields a round kernel reads before it starts its work, at the front of
// Ctrl and in the layout of CtrlHead, so one wide load brings them all (a
// chain of dependent scalar loads of these fields was most of the 4-5 us an
// idle kernel cost).
struct CtrlHead {
  int done;                  // the run is finished (or failed)
  int phase;                 // PHASE_LAZY (upper bounds) or PHASE_EXACT (exact degrees)
  unsigned int n_blocked;    // C4: blocked active vertices of this round
  unsigned int n_cedges;     // C4: conflict edges listed this round
  long long delta;           // Delta_i of the current round
  long long b;               // active-set size of the current round
  long long cursor;          // first pi position not yet passed
  long long n_rem;           // unclustered vertices
  int d_max[DITER];          // lazy Delta search: largest exact degree found by each band pass
  unsigned int tile_counter; // active-set scan tiles taken this round
  unsigned long long a_pack, c_pack, n_pack, p_pack;  // active / center / newly / peel lists
  unsigned long long r_pack[DITER];  // per band pass, the rescan list
  unsigned long long x_pack;  // rows of degree >= DSW recounted when switching to exact degrees
};

struct Ctrl {
  // ---- the head (same layout as CtrlHead) ----
  int done;
  int phase;
  unsigned int n_blocked, n_cedges;
  long long delta;
  long long b;
  long long cursor;
  long long n_rem;
  int d_max[DITER];
  unsigned int tile_counter;
  unsigned long long a_pack, c_pack, n_pack, p_pack;
  unsigned long long r_pack[DITER];
  unsigned long long x_pack;
  // ---- carried across rounds ----
  long long round;         // rounds finished
  long long n_start;       // n_i of the current round
  long long r_last;        // rank of the last active vertex
  int error;
  int has_round;           // a round has been run since the start
  int fallback;            // learned policy fell back to the fixed rule
  int select_done;         // per round: the active set is complete
  double eps_used;         // eps behind b
  float feat_conf, feat_claim, feat_eps;  // previous-round features for the learned policy
  int pad1;
  long long t_start;       // wall clock at round start
  unsigned long long conflicts;  // per round: ClusterWild! conflict marks counted by k_clear
  unsigned long long x_low[64];  // adjacency entries of the lower-degree rows recounted at the switch (spread)
  // bound buckets: entries per level (capacity fixed per graph)
  unsigned int lvl_cnt[NLVL];
  // run totals
  unsigned long long sum_elect, sum_claim, sum_rescan, sum_peel, sum_blocked, sum_atomics;
  // per-round statistics spread over 64 slots (slot = workgroup mod 64): one
  // address taken by every workgroup would serialise their atomics
  unsigned long long spread_atom[64], spread_conf[64];
  // active vertices of this round settled by the selection itself (no
  // unclustered neighbour: a center that claims nobody), spread the same way
  unsigned long long spread_lone[64];
};
static_assert(sizeof(CtrlHead) == 128, "the head is one 128-byte line");
static_assert(offsetof(Ctrl, done) == offsetof(CtrlHead, done) && offsetof(Ctrl, phase) == offsetof(CtrlHead, phase) &&
                  offsetof(Ctrl, n_blocked) == offsetof(CtrlHead, n_blocked) &&
                  offsetof(Ctrl, n_cedges) == offsetof(CtrlHead, n_cedges) &&
                  offsetof(Ctrl, delta) == offsetof(CtrlHead, delta) && offsetof(Ctrl, b) == offsetof(CtrlHead, b) &&
                  offsetof(Ctrl, cursor) == offsetof(CtrlHead, cursor) &&
                  offsetof(Ctrl, n_rem) == offsetof(CtrlHead, n_rem) &&
                  offsetof(Ctrl, d_max) == offsetof(CtrlHead, d_max) &&
                  offsetof(Ctrl, tile_counter) == offsetof(CtrlHead, tile_counter) &&
                  offsetof(Ctrl, a_pack) == offsetof(CtrlHead, a_pack) &&
                  offsetof(Ctrl, c_pack) == offsetof(CtrlHead, c_pack) &&
                  offsetof(Ctrl, n_pack) == offsetof(CtrlHead, n_pack) &&
                  offsetof(Ctrl, p_pack) == offsetof(CtrlHead, p_pack) &&
                  offsetof(Ctrl, r_pack) == offsetof(CtrlHead, r_pack) &&
                  offsetof(Ctrl, x_pack) == offsetof(CtrlHead, x_pack),
              "Ctrl starts with CtrlHead's layout");

// The head as the kernel starts: eight independent 16-byte scalar loads
// issued together (the values were written by earlier kernels of the
// stream).  The empty asm takes every loaded value, so the compiler can
// neither split the head into loads made one after another behind each
// test nor sink them past the early exits.
__device__ inline CtrlHead ctrl_head(const Ctrl *c) {
  const uint4 *p = reinterpret_cast<const uint4 *>(c);
  uint4 q[8];
#pragma unroll
  for (int i = 0; i < 8; i++) q[i] = p[i];
#pragma unroll
  for (int i = 0; i < 8; i++) asm volatile("" ::"s"(q[i].x), "s"(q[i].y), "s"(q[i].z), "s"(q[i].w));
  CtrlHead h;
  __builtin_memcpy(&h, q, sizeof(h));
  return h;
}

// A listed vertex's row: start of its adjacency in col, its degree and its
// rank in pi.  Carried along the active and center lists so the passes over
// those rows never look the offsets or the rank up again.
struct RowInfo {
  int64_t start;
  int32_t deg;
  int32_t rank;
};

struct Ws {
  // graph: the full renumbered rows are col[off[v] .. rend[v]) (rend = off +
  // 1).  The switch to exact degrees writes compacted rows, xcol[off[v] ..
  // xend[v]), holding only the neighbours then unclustered, at the start of
  // each row's original slot; every round after the switch walks those.
  const int64_t *off;
  const int64_t *rend;
  const int32_t *col;
  int32_t *xcol;        // compacted rows (col-sized; written at the switch)
  int64_t *xend;        // their ends (n)
  int64_t n;
  int64_t max_deg;
  int64_t low_start;        // internal ids from here on have degree < DSW ...
  int64_t iso_start;        // ... and from here on degree 0 (they sort last)
  // run input
  const int32_t *order;     // pi in internal ids (written by k_check_order)
  int32_t *iorder;          // the same buffer, writable
  const int32_t *order_in;  // the caller's pi (input ids)
  const int32_t *perm;      // input id -> internal id
  const int32_t *iperm;     // internal id -> input id
  int order_mapped;         // pi was mapped and checked by the bucketed passes: no marks in state
  // per-vertex arrays
  int32_t *rank, *lab, *ub;
  uint32_t *unc;
  uint8_t *state, *flag;
  // lists
  int32_t *alist, *clist, *nlist, *blist, *rlist, *xlist, *plist;
  int64_t *awork, *cwork, *rwork, *xwork, *pwork;
  RowInfo *ainfo, *cinfo;  // row info of alist / clist entries
  unsigned long long *racc;  // rescan accumulators (items covered << 32 | count), DITER * rcap
  int64_t rcap;         // capacity of one pass's rescan list
  int2 *cedge;
  int64_t cedge_cap;
  // C4's blocked vertices (k_resolve): the blocked index of a vertex (by
  // vertex id), and per blocked index its undecided earlier blocked
  // neighbours, its decision, the range of its later blocked neighbours in
  // bradj, and the queue of decided indices
  int32_t *bpos, *bpend, *bdec, *bdep, *bq, *bradj;
  unsigned long long *tstat;
  int64_t tstat_cap;
  // bound buckets
  int32_t *lvl;         // entries of all levels
  const int64_t *lvl_off;  // [NLVL+1] start of each level in lvl (device)
  int *hist;            // exact phase: vertices per remaining degree, [max_deg + 1]
  Ctrl *ctrl;
  RoundRec *trace;
  int64_t trace_cap;
  // epsilon policy
  int policy;
  int algo;
  int64_t eps_q;        // per-call eps in millionths
  double eps;
  const int64_t *sched; // TRACE: B_i schedule; BINOMIAL: pi positions per round (device)
  int64_t sched_len;
  int64_t bin_period;   // BINOMIAL: rounds between two halvings of Delta-hat
  const float *mlp;     // LEARNED: 6-64-1 weights (device)
  float eps_min, eps_max;
  int64_t max_rounds;   // > 0: stop after this many rounds (partial run)
  int64_t fault_round;  // > 0: test hook, the loop reports a device error after this round
  // progress word in pinned host memory, written by k_close at the end of
  // every round: rounds finished (bits 0..31), done (32), exact phase (33),
  // error (34)
  unsigned long long *progress;
};

constexpr int PROGRESS_DONE = 32, PROGRESS_EXACT = 33, PROGRESS_ERROR = 34;

__host__ __device__ inline int level_of(int64_t x) {  // floor(log2(x)), x >= 1
  int l = 0;
  while ((x >> 1) > 0) {
    x >>= 1;
    l++;
  }
  return l;
}

// ------------------------------------------------------------- atomics ----

template <class T>
__device__ inline T ld_acq(T *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline T ld_rlx(T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline void st_rel(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
// Relaxed device-scope atomic store: coherent across the XCDs like any
// device-scope atomic, without the release's write-back of the whole L2.
template <class T>
__device__ inline void st_rlx(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline T add_rlx(T *p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void set_error(Ctrl *c, int code) { atomicCAS(&c->error, 0, code); }

__device__ inline int lane_id() { return (int)(threadIdx.x & 63); }
__device__ inline int wave_id() { return (int)(threadIdx.x >> 6); }
__device__ inline unsigned long long lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive wave64 scan of 64-bit values.
__device__ inline int64_t wave_incl_scan(int64_t x) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t y = __shfl_up(x, d, 64);
    if (l >= d) x += y;
  }
  return x;
}
__device__ inline int64_t wave_sum(int64_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}
__device__ inline int wave_max(int x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = max(x, __shfl_xor(x, d, 64));
  return x;
}

// Workgroup exclusive scan of 64-bit values for NT threads; *total receives
// the sum.  Uses `sh` (NT/64 + 1 slots of shared memory); two barriers.
template <int NT = BS>
__device__ inline int64_t wg_excl_scan(int64_t x, int64_t *total, int64_t *sh) {
  constexpr int NW = NT / 64;
  const int64_t inc = wave_incl_scan(x);
  if (lane_id() == 63) sh[wave_id()] = inc;
  __syncthreads();
  int64_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; w++) {
    if (w < wave_id()) base += sh[w];
    tot += sh[w];
  }
  __syncthreads();
  *total = tot;
  return base + inc - x;
}

// Append the calling lanes' vertices (pred true) to a packed list, one atomic
// per wave.  weight = max(deg, 1) of the vertex.
__device__ inline void wave_append(bool pred, int32_t v, int64_t weight, unsigned long long *packc,
                                   int32_t *list, int64_t *work) {
  const unsigned long long m = __ballot(pred);
  if (m == 0) return;
  const int64_t w = pred ? weight : 0;
  const int64_t winc = wave_incl_scan(w);
  const int64_t wtot = __shfl(winc, 63, 64);
  const int leader = __ffsll((long long)m) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(packc, pk(wtot, __popcll(m)));
  base = __shfl(base, leader, 64);
  if (pred) {
    const int64_t slot = pk_cnt(base) + __popcll(m & lanemask_lt());
    list[slot] = v;
    work[slot] = pk_work(base) + winc - w;
  }
}

// wave_append for a list that carries row info (weight = max(deg, 1)).
__device__ inline void wave_append_info(bool pred, int32_t v, RowInfo ri, unsigned long long *packc, int32_t *list,
                                        int64_t *work, RowInfo *info) {
  const unsigned long long m = __ballot(pred);
  if (m == 0) return;
  const int64_t w = pred ? (ri.deg > 0 ? ri.deg : 1) : 0;
  const int64_t winc = wave_incl_scan(w);
  const int64_t wtot = __shfl(winc, 63, 64);
  const int leader = __ffsll((long long)m) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(packc, pk(wtot, __popcll(m)));
  base = __shfl(base, leader, 64);
  if (pred) {
    const int64_t slot = pk_cnt(base) + __popcll(m & lanemask_lt());
    list[slot] = v;
    work[slot] = pk_work(base) + winc - w;
    info[slot] = ri;
  }
}


// Largest i in [0, cnt) with work[i] <= s (work[0] = 0 <= s): a 64-ary search
// by one wave, about log64(cnt) dependent loads.
__device__ inline int64_t wave_find_entry(const int64_t *work, int64_t cnt, int64_t s) {
  int64_t lo = 0, hi = cnt;
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t idx = lo + (int64_t)lane_id() * step;
    const bool pred = idx < hi && work[idx] <= s;
    const unsigned long long m = __ballot(pred);
    const int k = __popcll(m);  // lanes 0..k-1 hold true (work is sorted)
    lo = lo + (int64_t)(k - 1) * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

__device__ inline bool unc_bit(const uint32_t *unc, int32_t v) { return (unc[v >> 5] >> (v & 31)) & 1u; }

}  // namespace ccd

namespace ccd {

// Workgroup-staged appends to a packed list: threads push (vertex, weight)
// into LDS; a flush reserves the whole batch with one atomic on the list
// counter and writes it out with coalesced stores.  Same-address device
// atomics serialise, so this keeps them to one per flush instead of one per
// wave and item group.
template <int CAP>
struct StageBuf {
  int32_t id[CAP];
  int32_t wt[CAP];
  int cnt;
  unsigned long long base;
  int64_t sh[WAVES + 1];
};

// Staging buffer of bare ids for a list nobody walks edge-balanced: one
// atomic reservation per flush, no weights and no work prefix.
template <int CAP>
struct IdBuf {
  int32_t id[CAP];
  int cnt;
  unsigned long long base;
};

template <int CAP>
__device__ inline void id_init(IdBuf<CAP> &b) {
  if (threadIdx.x == 0) b.cnt = 0;
  __syncthreads();
}

template <int CAP>
__device__ inline void id_push(IdBuf<CAP> &b, int32_t v) {
  b.id[atomicAdd(&b.cnt, 1)] = v;
}

// Collective: every thread of the workgroup calls it.
template <int CAP>
__device__ inline void id_flush(IdBuf<CAP> &b, unsigned long long *packc, int32_t *list) {
  __syncthreads();
  const int cnt = b.cnt;
  if (cnt == 0) return;
  if (threadIdx.x == 0) b.base = atomicAdd(packc, pk(0, cnt));
  __syncthreads();
  const int64_t slot0 = pk_cnt(b.base);
  for (int i = threadIdx.x; i < cnt; i += BS) list[slot0 + i] = b.id[i];
  __syncthreads();
  if (threadIdx.x == 0) b.cnt = 0;
  __syncthreads();
}

// Staging buffer whose entries also carry row info.
template <int CAP>
struct StageBufI : StageBuf<CAP> {
  RowInfo info[CAP];
};

template <int CAP>
__device__ inline void stage_push_info(StageBufI<CAP> &b, int32_t v, RowInfo ri) {
  const int p = atomicAdd(&b.cnt, 1);
  b.id[p] = v;
  b.wt[p] = ri.deg > 0 ? ri.deg : 1;
  b.info[p] = ri;
}

template <int CAP>
__device__ inline void stage_init(StageBuf<CAP> &b) {
  if (threadIdx.x == 0) b.cnt = 0;
  __syncthreads();
}

template <int CAP>
__device__ inline void stage_push(StageBuf<CAP> &b, int32_t v, int32_t weight) {
  const int p = atomicAdd(&b.cnt, 1);
  b.id[p] = v;
  b.wt[p] = weight;
}

// Collective: every thread of the workgroup calls it.
template <int CAP>
__device__ inline void stage_flush(StageBuf<CAP> &b, unsigned long long *packc, int32_t *list, int64_t *work,
                                   unsigned long long *zero_acc = nullptr, RowInfo *info = nullptr,
                                   const RowInfo *staged = nullptr) {
  __syncthreads();
  const int cnt = b.cnt;
  if (cnt == 0) return;
  constexpr int PER = (CAP + BS - 1) / BS;
  const int i0 = threadIdx.x * PER;
  int64_t s = 0;
  for (int i = i0; i < i0 + PER && i < cnt; i++) s += b.wt[i];
  int64_t tot;
  int64_t pre = wg_excl_scan(s, &tot, b.sh);
  if (threadIdx.x == 0) b.base = atomicAdd(packc, pk(tot, cnt));
  __syncthreads();
  const int64_t slot0 = pk_cnt(b.base), w0 = pk_work(b.base);
  for (int i = i0; i < i0 + PER && i < cnt; i++) {
    work[slot0 + i] = w0 + pre;
    pre += b.wt[i];
  }
  for (int i = threadIdx.x; i < cnt; i += BS) {
    list[slot0 + i] = b.id[i];
    if (zero_acc) zero_acc[slot0 + i] = 0;
    if (info) info[slot0 + i] = staged[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) b.cnt = 0;
  __syncthreads();
}

}  // namespace ccd
