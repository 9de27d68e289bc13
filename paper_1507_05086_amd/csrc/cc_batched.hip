// cc_batched.hip -- C4 / ClusterWild! (arXiv 1507.05086, Algorithm 2) on a
// batch of small graphs in one persistent launch.
//
// A graph of a few thousand vertices fits in LDS, so the whole round loop of
// one graph runs inside one group of threads with its vertex state in LDS:
// a workgroup for large graphs, a single wave for small ones (several graphs
// per workgroup).  Groups take graphs from two queues (large first, most work
// first), so the launch is balanced by longest-processing-time order.
// Inside a graph the remaining degrees are kept exactly (LDS atomics are
// cheap), and the adjacency passes (election, claims, peeling) are
// edge-balanced: each wave walks a contiguous range of the concatenated rows,
// streaming long rows with several loads in flight and locating row
// boundaries inside mixed windows with one LDS scatter and a wave scan.
#include "cc_device.h"
#include "cc_launch.h"

namespace ccd {

enum : uint8_t { F_UNC = 1, F_ACT = 2, F_CEN = 4, F_NON = 8, F_BLK = 16, F_MC = 32, F_MU = 64 };

// Packed per-vertex word: clusterID (rank of the center, INF16 while
// unclustered) in the high half, remaining positive degree in the low half.
// Ranks and degrees of a batch member are below 2^15.
constexpr uint32_t INF16 = 0x7FFF;
__device__ inline uint32_t lw_pack(uint32_t lab, uint32_t deg) { return (lab << 16) | deg; }

// Barrier of a sub-group of nw waves inside a workgroup (sense reversal on a
// generation counter in LDS).  Every wave of a workgroup is resident, so the
// waiting lanes always see the last arrival.
struct SubBar {
  int count, gen;
};

__device__ __forceinline__ void sub_sync(SubBar *b, int nw) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if (lane_id() == 0) {
    const int g = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const int arrived = __hip_atomic_fetch_add(&b->count, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (arrived == nw - 1) {
      __hip_atomic_store(&b->count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_store(&b->gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
      while (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == g)
        __builtin_amdgcn_s_sleep(1);
    }
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// A group of G threads working on one graph: one wave (G = 64), a sub-group
// of G / 64 waves of a larger workgroup (SUB), or the whole workgroup.
template <int G, bool SUB = false>
struct Grp {
  static constexpr int size = G;
  int tid;      // 0 .. G-1
  int64_t *sh;  // G/64 + 1 slots of scratch
  SubBar *bar;  // SUB only
  int wave0;    // first wave of the group in the workgroup
  __device__ __forceinline__ int wave() const { return G == 64 ? 0 : wave_id() - wave0; }
  __device__ __forceinline__ void sync() const {
    if (G == 64) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else if (SUB) {
      sub_sync(bar, G / 64);
    } else {
      __syncthreads();
    }
  }
  // exclusive scan; *tot = sum over the group
  __device__ __forceinline__ int64_t scan(int64_t x, int64_t *tot) const {
    const int64_t inc = wave_incl_scan(x);
    if (G == 64) {
      *tot = __shfl(inc, 63, 64);
      return inc - x;
    }
    if (lane_id() == 63) sh[wave()] = inc;
    sync();
    int64_t base = 0, t = 0;
    for (int w = 0; w < G / 64; w++) {
      if (w < wave()) base += sh[w];
      t += sh[w];
    }
    sync();
    *tot = t;
    return base + inc - x;
  }
  __device__ __forceinline__ int64_t max(int64_t x) const {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const int64_t y = __shfl_xor(x, d, 64);
      x = y > x ? y : x;
    }
    if (G == 64) return x;
    if (lane_id() == 0) sh[wave()] = x;
    sync();
    int64_t m = sh[0];
    for (int i = 1; i < G / 64; i++) m = sh[i] > m ? sh[i] : m;
    sync();
    return m;
  }
  __device__ __forceinline__ bool any(bool p) const { return max(p ? 1 : 0) != 0; }
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct BStats {
  unsigned long long elect, claim, peel, atom;
};

struct BatchArgs {
  const int64_t *off;      // global offsets (rows of all graphs)
  const int32_t *col;      // local ids
  const int64_t *vtx_ptr;  // [num_graphs + 1]
  const int32_t *order;    // per graph local permutation (concatenated)
  int32_t *labels;         // out: local center ids
  const int32_t *queue;    // graph ids, large-graph queue first, each part most work first
  int32_t n_big;           // queue[0, n_big): one graph per workgroup
  int32_t n_quad;          // queue[n_big, n_big + n_quad): one per 4-wave sub-group; rest: one per wave
  int32_t num_graphs;
  int32_t cap_big, cap_quad, cap_wave;  // LDS vertex capacity of a workgroup / sub-group / wave slot
  unsigned *heads;         // [3] queue heads
  int32_t *rounds;         // out: rounds per graph
  unsigned long long *stat;  // [4]: elect, claim, peel entries, atomics
  int *err;
  int algo;
  int64_t eps_q;
};

// LDS slot of capacity N vertices (21 bytes per vertex plus a few words):
//   lw     packed clusterID | remaining degree
//   pref   [N+1] prefix of row lengths of the list being walked
//   rstart [N+1] start of each row in the graph's cols
//   ctr    list counter
//   fl     flag byte, padded to whole words (word atomics touch 4 flags)
//   rank   pi^-1 (int16)
//   ordl   pi, position -> vertex (int16)
//   alist  active vertices; compacted in place to the centers
//   nlist  undecided actives during the election, then the newly clustered
struct Slot {
  uint32_t *lw;
  int32_t *pref, *rstart;
  int *ctr;
  uint8_t *fl;
  int16_t *rank, *ordl, *alist, *nlist;
  __host__ __device__ static size_t bytes(int N) {
    return (((size_t)N * 20 + 12 + (((size_t)N + 3) & ~(size_t)3)) + 15) / 16 * 16;
  }
  __device__ void carve(uint8_t *p, int N) {
    lw = (uint32_t *)p;
    pref = (int32_t *)(lw + N);
    rstart = pref + N + 1;
    ctr = rstart + N + 1;
    fl = (uint8_t *)(ctr + 1);
    rank = (int16_t *)(fl + ((N + 3) & ~3));
    ordl = rank + N;
    alist = ordl + N;
    nlist = alist + N;
  }
};

__device__ inline long long bt_batch(long long eps_q, long long n_rem, long long delta) {
  if (delta <= 0) return n_rem;
  const long long num = eps_q * n_rem, den = 1000000LL * delta;
  long long b = (num + den - 1) / den;
  if (b < 1) b = 1;
  if (b > n_rem) b = n_rem;
  return b;
}

// Edge-balanced pass over the rows of list[0..cnt): f(i, v, u) for every
// entry u of row v = list[i]; row v is col0[rstart[v] .. rstart[v+1]).  `rs`
// is the calling wave's 64 ints of LDS scratch.  Each wave walks a contiguous
// range of the concatenated rows: a row covering the next 64 or more entries
// is streamed with K loads in flight; otherwise up to W windows of 64 entries
// have their rows located (LDS only) before their loads are issued together.
// Returns the number of entries walked.
template <class GR, int K, int W, class F>
__device__ __forceinline__ int rows_pass(const GR &g, const int16_t *list, int cnt, Slot &s, const int32_t *col0,
                                int *rs, F &&f) {
  constexpr int G = GR::size;
  int carry = 0;
  for (int i0 = 0; i0 < cnt; i0 += G) {
    const int i = i0 + g.tid;
    int d = 0;
    if (i < cnt) {
      const int32_t v = list[i];
      d = s.rstart[v + 1] - s.rstart[v];
    }
    int64_t tot;
    const int pre = (int)g.scan(d, &tot);
    if (i < cnt) s.pref[i] = carry + pre;
    carry += (int)tot;
  }
  const int total = carry;
  if (g.tid == 0) s.pref[cnt] = total;
  g.sync();
  if (total == 0) return 0;
  constexpr int NW = G / 64;
  const int lane = lane_id();
  const int w = NW == 1 ? 0 : g.wave();
  int chunk = (total + NW - 1) / NW;
  chunk = (chunk + 63) & ~63;
  const int c0 = min(total, w * chunk), c1 = min(total, c0 + chunk);
  if (c0 < c1) {
    // lo: the last row whose prefix is <= c0 (the same search in every lane);
    // row 0 already satisfies the invariant below when c0 = 0
    int lo = 0, hi = c0 > 0 ? cnt : 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s.pref[mid] <= c0) lo = mid;
      else hi = mid;
    }
    // invariant: pref[lo] <= e0 <= pref[lo + 1] and lo < cnt
    int e0 = c0;
    while (e0 < c1) {
      const int b0 = s.pref[lo + 1];
      if (b0 >= e0 + 64) {
        // row lo covers the next 64 or more entries: stream them
        const int end = min(b0, c1);
        const int32_t v = list[lo];
        const int32_t *cp = col0 + (s.rstart[v] - s.pref[lo]);
        for (int e = e0 + lane; e < end; e += 64 * K) {
          int32_t u[K];
#pragma unroll
          for (int k = 0; k < K; k++) u[k] = e + 64 * k < end ? cp[e + 64 * k] : -1;
#pragma unroll
          for (int k = 0; k < K; k++)
            if (u[k] >= 0) f(lo, v, u[k]);
        }
        e0 = end;
        if (e0 == b0) lo++;
        continue;
      }
      // up to W windows [e0, e0 + 64) holding row starts: the row of entry
      // e0 + l is lo + #{j : pref[lo + 1 + j] <= e0 + l}
      int rowk[W], ek[W];
#pragma unroll
      for (int k = 0; k < W; k++) {
        rowk[k] = -1;
        ek[k] = -1;
        if (e0 >= c1 || (k > 0 && s.pref[lo + 1] >= e0 + 64)) continue;  // uniform
        const int j = lo + 1 + lane;
        const int bj = j <= cnt ? s.pref[j] : 0x7fffffff;
        const bool in = bj <= e0 + 63;
        const bool full = __ballot(in) == ~0ull;
        int wend = full ? __shfl(bj, 63, 64) : e0 + 64;
        if (wend > c1) wend = c1;
        rs[lane] = 0;
        wave_sync();
        const int bn = __shfl_down(bj, 1, 64);
        if (in && (lane == 63 || bn != bj)) rs[bj - e0] = lane + 1;
        wave_sync();
        int r = rs[lane];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const int t = __shfl_up(r, d, 64);
          if (lane >= d) r = t > r ? t : r;
        }
        if (e0 + lane < wend) {
          rowk[k] = lo + r;
          ek[k] = e0 + lane;
        }
        lo += __popcll(__ballot(bj <= wend));
        e0 = wend;
        wave_sync();
      }
      int32_t vk[W], ck[W], uk[W];
#pragma unroll
      for (int k = 0; k < W; k++) {
        vk[k] = 0;
        ck[k] = 0;
        if (rowk[k] >= 0) {
          vk[k] = list[rowk[k]];
          ck[k] = s.rstart[vk[k]] + (ek[k] - s.pref[rowk[k]]);
        }
      }
#pragma unroll
      for (int k = 0; k < W; k++) uk[k] = rowk[k] >= 0 ? col0[ck[k]] : -1;
#pragma unroll
      for (int k = 0; k < W; k++)
        if (rowk[k] >= 0) f(rowk[k], vk[k], uk[k]);
    }
  }
  g.sync();
  return total;
}

// Inlined into the kernel so that every Slot pointer is known to address LDS
// (an out-of-line call would turn them into generic pointers).
template <class GR>
__device__ __forceinline__ void solve_graph(const GR &g, const BatchArgs &a, int gi, int cap, Slot &s, int *rs, BStats &st) {
  constexpr int G = GR::size;
  const int64_t v0 = a.vtx_ptr[gi];
  const int n = (int)(a.vtx_ptr[gi + 1] - v0);
  if (n > cap) {  // the host sizes the slots; never taken
    if (g.tid == 0) atomicCAS(a.err, 0, ERR_OVERFLOW);
    return;
  }
  const int64_t *off = a.off + v0;
  const int64_t obase = off[0];
  const int32_t *col0 = a.col + obase;
  const int32_t *ord = a.order + v0;
  const bool c4 = a.algo == ALGO_C4;
  constexpr int K = 4, W = 4;
  // init: row starts, packed words, pi in LDS; rank = pi^-1 with a permutation check
  for (int v = g.tid; v <= n; v += G) {
    const int64_t o = off[v];
    s.rstart[v] = (int32_t)(o - obase);
    if (v < n) {
      s.lw[v] = lw_pack(INF16, (uint32_t)(off[v + 1] - o));
      s.fl[v] = F_UNC;
      s.rank[v] = -1;
    }
  }
  g.sync();
  bool bad = false;
  for (int k = g.tid; k < n; k += G) {
    const int32_t v = ord[k];
    s.ordl[k] = (int16_t)v;
    if (v < 0 || v >= n) bad = true;
    else s.rank[v] = (int16_t)k;
  }
  g.sync();
  for (int v = g.tid; v < n; v += G) {
    const int r = s.rank[v];
    if (r < 0 || s.ordl[r] != v) bad = true;
  }
  if (g.any(bad)) {
    if (g.tid == 0) atomicCAS(a.err, 0, ERR_PERM);
    return;
  }
  int n_rem = n, cur = 0, rounds = 0;
  while (n_rem > 0 && rounds <= n) {
    // Delta over the unclustered vertices
    int64_t m = 0;
    for (int v = g.tid; v < n; v += G) {
      const int64_t d = (int64_t)(s.lw[v] & 0xFFFFu);
      if ((s.fl[v] & F_UNC) && d > m) m = d;
    }
    const long long delta = g.max(m);
    const int B = (int)bt_batch(a.eps_q, n_rem, delta);
    // active set: the next B unclustered vertices of pi from the cursor
    int na = 0;
    while (na < B && cur < n) {
      const int p = cur + g.tid;
      int32_t v = 0;
      bool un = false;
      if (p < n) {
        v = s.ordl[p];
        un = (s.fl[v] & F_UNC) != 0;
      }
      int64_t tot;
      const int64_t pre = g.scan(un ? 1 : 0, &tot);
      if (un && na + pre < B) {
        s.alist[na + pre] = (int16_t)v;
        s.fl[v] |= F_ACT;
      }
      // position of the B-th unclustered vertex, if in this chunk
      const int64_t last = g.max((un && na + pre == B - 1) ? (int64_t)p + 1 : 0);
      if (last > 0) {
        cur = (int)last;
        na = B;
      } else {
        cur += G;
        na += (int)tot;
      }
    }
    g.sync();
    // centers
    int nc = 0;
    if (c4) {
      // blocked: an earlier-ranked active neighbour
      const int t_elect = rows_pass<GR, K, W>(g, s.alist, B, s, col0, rs, [&](int, int32_t av, int32_t u) {
        if ((s.fl[u] & F_ACT) && s.rank[u] < s.rank[av]) s.fl[av] |= F_BLK;
      });
      if (g.tid == 0) st.elect += (unsigned long long)t_elect;
      for (int i = g.tid; i < B; i += G) {
        const int32_t av = s.alist[i];
        if (!(s.fl[av] & F_BLK)) s.fl[av] |= F_CEN;
      }
      g.sync();
      // fixed point over the blocked vertices: a vertex becomes a center once
      // no earlier active neighbour is a center or undecided, and a
      // non-center once an earlier active neighbour is a center
      for (int it = 0; it <= B; it++) {
        int nb = 0;
        for (int i0 = 0; i0 < B; i0 += G) {
          const int i = i0 + g.tid;
          bool und = false;
          if (i < B) {
            const int32_t av = s.alist[i];
            und = !(s.fl[av] & (F_CEN | F_NON));
          }
          int64_t tot;
          const int64_t pre = g.scan(und ? 1 : 0, &tot);
          if (und) s.nlist[nb + pre] = s.alist[i];
          nb += (int)tot;
        }
        g.sync();
        if (nb == 0) break;
        const int t_res = rows_pass<GR, K, W>(g, s.nlist, nb, s, col0, rs, [&](int, int32_t av, int32_t u) {
          const uint8_t fu = s.fl[u];
          if ((fu & F_ACT) && s.rank[u] < s.rank[av]) {
            const unsigned bit = (fu & F_CEN) ? (unsigned)F_MC : ((fu & F_NON) ? 0u : (unsigned)F_MU);
            if (bit) atomicOr((unsigned *)(s.fl + (av & ~3)), bit << (8 * (av & 3)));
          }
        });
        if (g.tid == 0) st.elect += (unsigned long long)t_res;
        for (int i = g.tid; i < nb; i += G) {
          const int32_t av = s.nlist[i];
          const uint8_t f = s.fl[av];
          uint8_t nf = (uint8_t)(f & ~(F_MC | F_MU));
          if (f & F_MC) nf |= F_NON;
          else if (!(f & F_MU)) nf |= F_CEN;
          s.fl[av] = nf;
        }
        g.sync();
      }
      // compact the centers to the front of alist, in place: every write
      // lands at or before the chunk whose entries are already read
      for (int i0 = 0; i0 < B; i0 += G) {
        const int i = i0 + g.tid;
        bool cen = false;
        int16_t av = 0;
        if (i < B) {
          av = s.alist[i];
          cen = (s.fl[av] & F_CEN) != 0;
        }
        int64_t tot;
        const int64_t pre = g.scan(cen ? 1 : 0, &tot);
        if (cen) s.alist[nc + pre] = av;
        nc += (int)tot;
      }
    } else {
      for (int i = g.tid; i < B; i += G) s.fl[s.alist[i]] |= F_CEN;
      nc = B;
    }
    g.sync();
    // claims: lowest-rank adjacent center wins; newly = centers + first claims
    int *nn_ptr = s.ctr;
    if (g.tid == 0) *nn_ptr = 0;
    g.sync();
    for (int i = g.tid; i < nc; i += G) {
      const int32_t cv = s.alist[i];
      s.lw[cv] = lw_pack((uint32_t)s.rank[cv], 0);
      s.nlist[atomicAdd(nn_ptr, 1)] = (int16_t)cv;
    }
    g.sync();
    const int t_claim = rows_pass<GR, K, W>(g, s.alist, nc, s, col0, rs, [&](int, int32_t cv, int32_t u) {
      const uint8_t fu = s.fl[u];
      if (!(fu & F_UNC) || (fu & F_CEN)) return;
      if (!c4 && (fu & F_ACT)) return;  // ClusterWild! claims Gamma(c) \ A
      const uint32_t rc = (uint32_t)s.rank[cv];
      if (rc < (s.lw[u] >> 16)) {
        const uint32_t old = atomicMin(&s.lw[u], lw_pack(rc, 0xFFFFu));
        st.atom++;
        if ((old >> 16) == INF16) s.nlist[atomicAdd(nn_ptr, 1)] = (int16_t)u;
      }
    });
    if (g.tid == 0) st.claim += (unsigned long long)t_claim;
    const int nn = *nn_ptr;
    // the newly clustered leave; the unclustered neighbours of the claimed
    // ones lose one degree.  Centers (nlist[0, nc)) have none left: every
    // unclustered neighbour of a center was claimed this round.
    for (int i = g.tid; i < nn; i += G) s.fl[s.nlist[i]] = 0;
    g.sync();
    const int t_peel = rows_pass<GR, K, W>(g, s.nlist + nc, nn - nc, s, col0, rs, [&](int, int32_t, int32_t u) {
      if (s.fl[u] & F_UNC) {
        atomicSub(&s.lw[u], 1u);
        st.atom++;
      }
    });
    if (g.tid == 0) st.peel += (unsigned long long)t_peel;
    n_rem -= nn;
    rounds++;
    g.sync();
  }
  for (int v = g.tid; v < n; v += G) {
    const uint32_t l = s.lw[v] >> 16;
    a.labels[v0 + v] = l < (uint32_t)n ? (int32_t)s.ordl[l] : -1;
    if (l >= (uint32_t)n) atomicCAS(a.err, 0, ERR_LABEL);
  }
  if (g.tid == 0) a.rounds[gi] = rounds;
  if (n_rem > 0 && g.tid == 0) atomicCAS(a.err, 0, ERR_NO_PROGRESS);
}

constexpr int QG = 256;  // threads of a sub-group (4 waves)

template <int T>
__global__ void __launch_bounds__(T) k_batched(BatchArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  BStats st{0, 0, 0, 0};
  constexpr int NQ = T / QG > 0 ? T / QG : 1;
  __shared__ int s_gi[NQ];
  __shared__ int64_t sh[T / 64 + 1];
  __shared__ int64_t shq[NQ][QG / 64 + 1];
  __shared__ SubBar sbar[NQ];
  __shared__ int rsb[T / 64][64];
  int *rs = rsb[wave_id()];
  if (threadIdx.x < NQ) sbar[threadIdx.x] = SubBar{0, 0};
  __syncthreads();
  // phase 1: large graphs, one per workgroup
  Grp<T> gw{(int)threadIdx.x, sh, nullptr, 0};
  Slot sl;
  sl.carve(lds, a.cap_big);
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned q = atomicAdd(&a.heads[0], 1u);
      s_gi[0] = (int)q < a.n_big ? a.queue[q] : -1;
    }
    __syncthreads();
    const int gi = s_gi[0];
    __syncthreads();
    if (gi < 0) break;
    solve_graph(gw, a, gi, a.cap_big, sl, rs, st);
    __syncthreads();
  }
  // phase 2: mid-size graphs, one per sub-group of 4 waves (workgroups of 512+)
  if (T > QG && a.n_quad > 0) {
    const int sg = (int)threadIdx.x / QG;
    Grp<QG, true> gq{(int)threadIdx.x % QG, shq[sg], &sbar[sg], sg * (QG / 64)};
    Slot sq;
    sq.carve(lds + (size_t)sg * Slot::bytes(a.cap_quad), a.cap_quad);
    for (;;) {
      if (gq.tid == 0) {
        const unsigned q = atomicAdd(&a.heads[2], 1u);
        s_gi[sg] = (int)q < a.n_quad ? a.queue[a.n_big + q] : -1;
      }
      gq.sync();
      const int gi = s_gi[sg];
      gq.sync();
      if (gi < 0) break;
      solve_graph(gq, a, gi, a.cap_quad, sq, rs, st);
      gq.sync();
    }
    __syncthreads();
  }
  // phase 3: small graphs, one per wave
  Grp<64> gv{lane_id(), nullptr, nullptr, 0};
  Slot sv;
  sv.carve(lds + (size_t)wave_id() * Slot::bytes(a.cap_wave), a.cap_wave);
  const int n0 = a.n_big + a.n_quad, nsmall = a.num_graphs - n0;
  for (;;) {
    int q = 0;
    if (lane_id() == 0) q = (int)atomicAdd(&a.heads[1], 1u);
    q = __shfl(q, 0, 64);
    if (q >= nsmall) break;
    solve_graph(gv, a, a.queue[n0 + q], a.cap_wave, sv, rs, st);
  }
  // statistics: one reduction per workgroup, one atomic per counter
  __syncthreads();
  unsigned long long v4[4] = {st.elect, st.claim, st.peel, st.atom};
  for (int k = 0; k < 4; k++) {
    int64_t tot;
    const int64_t pre = gw.scan((int64_t)v4[k], &tot);
    (void)pre;
    if (threadIdx.x == 0 && tot) atomicAdd(&a.stat[k], (unsigned long long)tot);
  }
}

// Kernels with more than 64 KB of dynamic LDS must say so before launch.
static hipError_t allow_lds(int block, size_t lds) {
  const void *k = block == 256 ? (const void *)k_batched<256>
                  : block == 512 ? (const void *)k_batched<512> : (const void *)k_batched<1024>;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_batched(const BatchLaunch &bl, hipStream_t s) {
  BatchArgs a{bl.off, bl.col, bl.vtx_ptr, bl.order, bl.labels, bl.queue, bl.n_big, bl.n_quad, bl.num_graphs,
              bl.cap_big, bl.cap_quad, bl.cap_wave, bl.heads, bl.rounds, bl.stat, bl.err, bl.algo, bl.eps_q};
  const size_t lds = batched_lds_bytes(bl.block, bl.cap_big, bl.cap_quad, bl.cap_wave);
  hipError_t e = allow_lds(bl.block, lds);
  if (e != hipSuccess) return e;
  if (bl.block == 256) hipLaunchKernelGGL(k_batched<256>, dim3(bl.grid), dim3(256), lds, s, a);
  else if (bl.block == 512) hipLaunchKernelGGL(k_batched<512>, dim3(bl.grid), dim3(512), lds, s, a);
  else hipLaunchKernelGGL(k_batched<1024>, dim3(bl.grid), dim3(1024), lds, s, a);
  return hipGetLastError();
}

size_t batched_lds_bytes(int block, int cap_big, int cap_quad, int cap_wave) {
  const size_t a = Slot::bytes(cap_big), b = (size_t)(block / 64) * Slot::bytes(cap_wave);
  const size_t q = block > QG ? (size_t)(block / QG) * Slot::bytes(cap_quad) : 0;
  const size_t m = a > b ? a : b;
  return m > q ? m : q;
}

hipError_t batched_max_grid(int block, size_t lds, int *grid) {
  int occ = 0;
  hipError_t e = allow_lds(block, lds);
  if (e != hipSuccess) return e;
  if (block == 256) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_batched<256>, 256, lds);
  else if (block == 512) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_batched<512>, 512, lds);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_batched<1024>, 1024, lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  *grid = occ * cus;
  return e;
}

}  // namespace ccd
