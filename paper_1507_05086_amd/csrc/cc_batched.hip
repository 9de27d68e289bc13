// cc_batched.hip -- C4 / ClusterWild! (arXiv 1507.05086, Algorithm 2) on a
// batch of small graphs in one persistent launch.
//
// A graph of a few thousand vertices fits in LDS, so the whole round loop of
// one graph runs inside one group of threads with its vertex state in LDS:
// a workgroup for large graphs, a single wave for small ones (several graphs
// per workgroup).  Groups take graphs from two queues (large first, largest
// graph first), so the launch is balanced by longest-processing-time order.
// Inside a graph the remaining degrees are kept exactly (LDS atomics are
// cheap), every adjacency pass is edge-balanced over the group through a
// prefix of row lengths in LDS, and the C4 election is the same wait-free
// fixed point as the single-graph path.
#include "cc_device.h"
#include "cc_launch.h"

namespace ccd {

enum : uint8_t { F_UNC = 1, F_ACT = 2, F_CEN = 4, F_NON = 8, F_BLK = 16 };

// A group of G threads working on one graph (G = 64: one wave; G = block).
template <int G>
struct Grp {
  int tid;
  int64_t *sh;  // G/64 + 1 slots of scratch
  __device__ void sync() const {
    if (G == 64) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  }
  // exclusive scan; *tot = sum over the group
  __device__ int64_t scan(int64_t x, int64_t *tot) const {
    if (G == 64) {
      const int64_t inc = wave_incl_scan(x);
      *tot = __shfl(inc, 63, 64);
      return inc - x;
    }
    return wg_excl_scan<G>(x, tot, sh);
  }
  __device__ int64_t max(int64_t x) const {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const int64_t y = __shfl_xor(x, d, 64);
      x = y > x ? y : x;
    }
    if (G == 64) return x;
    if (lane_id() == 0) sh[wave_id()] = x;
    __syncthreads();
    int64_t m = sh[0];
    for (int i = 1; i < G / 64; i++) m = sh[i] > m ? sh[i] : m;
    __syncthreads();
    return m;
  }
  __device__ bool any(bool p) const { return max(p ? 1 : 0) != 0; }
};

struct BStats {
  unsigned long long elect, claim, peel, atom;
};

struct BatchArgs {
  const int64_t *off;      // global offsets (rows of all graphs)
  const int32_t *col;      // local ids
  const int64_t *vtx_ptr;  // [num_graphs + 1]
  const int32_t *order;    // per graph local permutation (concatenated)
  int32_t *labels;         // out: local center ids
  const int32_t *queue;    // graph ids, large-graph queue first, each part largest first
  int32_t n_big;           // queue[0, n_big): one graph per workgroup; rest: one per wave
  int32_t num_graphs;
  int32_t cap_big, cap_wave;  // LDS vertex capacity of a workgroup slot / a wave slot
  unsigned *heads;         // [2] queue heads
  int32_t *rounds;         // out: rounds per graph
  unsigned long long *stat;  // [4]: elect, claim, peel entries, atomics
  int *err;
  int algo;
  int64_t eps_q;
};

// LDS slot of capacity N vertices: 21 bytes per vertex plus a counter.
struct Slot {
  int32_t *lab, *rdeg, *pref;
  int16_t *rank, *alist, *clist, *nlist;
  uint8_t *fl;
  int *ctr;
  __host__ __device__ static size_t bytes(int N) { return (((size_t)N * 21 + 4 + 15) / 16) * 16; }
  __device__ void carve(uint8_t *p, int N) {
    lab = (int32_t *)p;
    rdeg = lab + N;
    pref = rdeg + N;
    rank = (int16_t *)(pref + N);
    alist = rank + N;
    clist = alist + N;
    nlist = clist + N;
    fl = (uint8_t *)(nlist + N);
    ctr = (int *)(p + (((size_t)N * 21 + 3) / 4) * 4);
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
// entry u of row v = list[i].  Row lengths are prefix-summed into pref.
template <int G, class F>
__device__ inline int64_t rows_pass(const Grp<G> &g, const int16_t *list, int cnt, int32_t *pref,
                                    const int64_t *off, const int32_t *col, F &&f) {
  int64_t carry = 0;
  for (int i0 = 0; i0 < cnt; i0 += G) {
    const int i = i0 + g.tid;
    const int64_t d = i < cnt ? off[list[i] + 1] - off[list[i]] : 0;
    int64_t tot;
    const int64_t pre = g.scan(d, &tot);
    if (i < cnt) pref[i] = (int32_t)(carry + pre);
    carry += tot;
  }
  g.sync();
  const int64_t total = carry;
  for (int64_t e = g.tid; e < total; e += G) {
    int lo = 0, hi = cnt;  // last i with pref[i] <= e
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pref[mid] <= e) lo = mid;
      else hi = mid;
    }
    const int32_t v = list[lo];
    const int32_t u = col[off[v] + (e - pref[lo])];
    f(lo, v, u);
  }
  g.sync();
  return total;
}

template <int G>
__device__ void solve_graph(const Grp<G> &g, const BatchArgs &a, int gi, int cap, Slot &s, BStats &st) {
  const int64_t v0 = a.vtx_ptr[gi];
  const int n = (int)(a.vtx_ptr[gi + 1] - v0);
  if (n > cap) {  // the host sizes the slots; never taken
    if (g.tid == 0) atomicCAS(a.err, 0, ERR_OVERFLOW);
    return;
  }
  const int64_t *off = a.off + v0;
  const int32_t *col = a.col;
  const int32_t *ord = a.order + v0;
  const bool c4 = a.algo == ALGO_C4;
  // init; rank = ord^-1 with a permutation check
  for (int v = g.tid; v < n; v += G) {
    s.lab[v] = INF;
    s.rdeg[v] = (int32_t)(off[v + 1] - off[v]);
    s.fl[v] = F_UNC;
    s.rank[v] = -1;
  }
  g.sync();
  bool bad = false;
  for (int k = g.tid; k < n; k += G) {
    const int32_t v = ord[k];
    if (v < 0 || v >= n) bad = true;
    else s.rank[v] = (int16_t)k;
  }
  g.sync();
  for (int v = g.tid; v < n; v += G) {
    const int r = s.rank[v];
    if (r < 0 || ord[r] != v) bad = true;
  }
  if (g.any(bad)) {
    if (g.tid == 0) atomicCAS(a.err, 0, ERR_PERM);
    return;
  }
  int n_rem = n, cur = 0, rounds = 0;
  while (n_rem > 0 && rounds <= n) {
    // Delta over the unclustered vertices
    int64_t m = 0;
    for (int v = g.tid; v < n; v += G)
      if ((s.fl[v] & F_UNC) && s.rdeg[v] > m) m = s.rdeg[v];
    const long long delta = g.max(m);
    const int B = (int)bt_batch(a.eps_q, n_rem, delta);
    // active set: the next B unclustered vertices of pi from the cursor
    int na = 0;
    while (na < B && cur < n) {
      const int p = cur + g.tid;
      int32_t v = 0;
      bool un = false;
      if (p < n) {
        v = ord[p];
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
      const int64_t t_elect = rows_pass(g, s.alist, B, s.pref, off, col, [&](int, int32_t av, int32_t u) {
        if ((s.fl[u] & F_ACT) && s.rank[u] < s.rank[av]) s.fl[av] |= F_BLK;
      });
      if (g.tid == 0) st.elect += (unsigned long long)t_elect;
      for (int i = g.tid; i < B; i += G) {
        const int32_t av = s.alist[i];
        if (!(s.fl[av] & F_BLK)) s.fl[av] |= F_CEN;
      }
      g.sync();
      // fixed point over the blocked vertices (row rescans; blocked sets are small)
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
        const int64_t t_res = rows_pass(g, s.nlist, nb, s.pref, off, col, [&](int, int32_t av, int32_t u) {
          if ((s.fl[u] & F_ACT) && s.rank[u] < s.rank[av]) {
            // marks in the two top bits of rdeg (degrees < 2^30): bit 30 = an
            // earlier center, bit 31 = an earlier undecided vertex
            const int bit = (s.fl[u] & F_CEN) ? 1 : ((s.fl[u] & F_NON) ? 0 : 2);
            if (bit) atomicOr((unsigned *)&s.rdeg[av], (unsigned)bit << 30);
          }
        });
        if (g.tid == 0) st.elect += (unsigned long long)t_res;
        for (int i = g.tid; i < nb; i += G) {
          const int32_t av = s.nlist[i];
          const unsigned mark = ((unsigned)s.rdeg[av]) >> 30;
          s.rdeg[av] &= 0x3FFFFFFF;
          if (mark & 1) s.fl[av] |= F_NON;
          else if (!(mark & 2)) s.fl[av] |= F_CEN;
        }
        g.sync();
      }
      for (int i0 = 0; i0 < B; i0 += G) {
        const int i = i0 + g.tid;
        bool cen = false;
        int32_t av = 0;
        if (i < B) {
          av = s.alist[i];
          cen = (s.fl[av] & F_CEN) != 0;
        }
        int64_t tot;
        const int64_t pre = g.scan(cen ? 1 : 0, &tot);
        if (cen) s.clist[nc + pre] = (int16_t)av;
        nc += (int)tot;
      }
    } else {
      for (int i = g.tid; i < B; i += G) {
        const int32_t av = s.alist[i];
        s.fl[av] |= F_CEN;
        s.clist[i] = (int16_t)av;
      }
      nc = B;
    }
    g.sync();
    // claims: lowest-rank adjacent center wins; newly = centers + first claims
    int *nn_ptr = s.ctr;
    if (g.tid == 0) *nn_ptr = 0;
    g.sync();
    for (int i = g.tid; i < nc; i += G) {
      const int32_t cv = s.clist[i];
      s.lab[cv] = s.rank[cv];
      s.nlist[atomicAdd(nn_ptr, 1)] = (int16_t)cv;
    }
    g.sync();
    const int64_t t_claim = rows_pass(g, s.clist, nc, s.pref, off, col, [&](int i, int32_t cv, int32_t u) {
      const uint8_t fu = s.fl[u];
      if (!(fu & F_UNC) || (fu & F_CEN)) return;
      if (!c4 && (fu & F_ACT)) return;  // ClusterWild! claims Gamma(c) \ A
      const int32_t rc = s.rank[cv];
      if (rc < s.lab[u]) {
        const int32_t old = atomicMin(&s.lab[u], rc);
        st.atom++;
        if (old == INF) s.nlist[atomicAdd(nn_ptr, 1)] = (int16_t)u;
      }
    });
    if (g.tid == 0) st.claim += (unsigned long long)t_claim;
    const int nn = *nn_ptr;
    // the newly clustered leave; their unclustered neighbours lose one degree
    for (int i = g.tid; i < nn; i += G) s.fl[s.nlist[i]] = 0;
    g.sync();
    const int64_t t_peel = rows_pass(g, s.nlist, nn, s.pref, off, col, [&](int, int32_t, int32_t u) {
      if (s.fl[u] & F_UNC) {
        atomicSub(&s.rdeg[u], 1);
        st.atom++;
      }
    });
    if (g.tid == 0) st.peel += (unsigned long long)t_peel;
    // active marks of this round are done (every active vertex is now clustered)
    n_rem -= nn;
    rounds++;
    g.sync();
  }
  for (int v = g.tid; v < n; v += G) {
    const int32_t l = s.lab[v];
    a.labels[v0 + v] = (l >= 0 && l < n) ? ord[l] : -1;
    if (l < 0 || l >= n) atomicCAS(a.err, 0, ERR_LABEL);
  }
  if (g.tid == 0) a.rounds[gi] = rounds;
  if (n_rem > 0 && g.tid == 0) atomicCAS(a.err, 0, ERR_NO_PROGRESS);
}

template <int T>
__global__ void __launch_bounds__(T) k_batched(BatchArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  BStats st{0, 0, 0, 0};
  __shared__ int s_gi;
  __shared__ int64_t sh[T / 64 + 1];
  // phase 1: large graphs, one per workgroup
  Grp<T> gw{(int)threadIdx.x, sh};
  Slot sl;
  sl.carve(lds, a.cap_big);
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned q = atomicAdd(&a.heads[0], 1u);
      s_gi = (int)q < a.n_big ? a.queue[q] : -1;
    }
    __syncthreads();
    const int gi = s_gi;
    __syncthreads();
    if (gi < 0) break;
    solve_graph<T>(gw, a, gi, a.cap_big, sl, st);
    __syncthreads();
  }
  // phase 2: small graphs, one per wave
  Grp<64> gv{lane_id(), nullptr};
  Slot sv;
  sv.carve(lds + (size_t)wave_id() * Slot::bytes(a.cap_wave), a.cap_wave);
  const int nsmall = a.num_graphs - a.n_big;
  for (;;) {
    int q = 0;
    if (lane_id() == 0) q = (int)atomicAdd(&a.heads[1], 1u);
    q = __shfl(q, 0, 64);
    if (q >= nsmall) break;
    solve_graph<64>(gv, a, a.queue[a.n_big + q], a.cap_wave, sv, st);
  }
  // statistics: one reduction per workgroup, one atomic per counter
  __syncthreads();
  unsigned long long v4[4] = {st.elect, st.claim, st.peel, st.atom};
  for (int k = 0; k < 4; k++) {
    int64_t tot;
    wg_excl_scan<T>((int64_t)v4[k], &tot, sh);
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
  BatchArgs a{bl.off, bl.col, bl.vtx_ptr, bl.order, bl.labels, bl.queue, bl.n_big, bl.num_graphs,
              bl.cap_big, bl.cap_wave, bl.heads, bl.rounds, bl.stat, bl.err, bl.algo, bl.eps_q};
  const size_t lds = batched_lds_bytes(bl.block, bl.cap_big, bl.cap_wave);
  hipError_t e = allow_lds(bl.block, lds);
  if (e != hipSuccess) return e;
  if (bl.block == 256) hipLaunchKernelGGL(k_batched<256>, dim3(bl.grid), dim3(256), lds, s, a);
  else if (bl.block == 512) hipLaunchKernelGGL(k_batched<512>, dim3(bl.grid), dim3(512), lds, s, a);
  else hipLaunchKernelGGL(k_batched<1024>, dim3(bl.grid), dim3(1024), lds, s, a);
  return hipGetLastError();
}

size_t batched_lds_bytes(int block, int cap_big, int cap_wave) {
  const size_t a = Slot::bytes(cap_big), b = (size_t)(block / 64) * Slot::bytes(cap_wave);
  return a > b ? a : b;
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
