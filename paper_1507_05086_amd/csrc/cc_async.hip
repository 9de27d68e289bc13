// cc_async.hip -- asynchronous C4 and ClusterWild! (arXiv 1507.05086,
// Algorithm 3: the round loop without its bulk synchronisation).
//
// Threads take the vertices of pi in order and never wait for a round to
// end.  On the GPU a wave takes the next 64 positions of pi (a chunk; lane l
// holds position 64 c + l) from a shared counter and settles them:
//
//   C4 (attemptCluster / isCenter): a vertex still unclustered when reached
//   is a center iff none of its earlier-ranked neighbours is one.  An earlier
//   neighbour in an earlier chunk is waited for until it is decided; one in
//   the same chunk is settled by a short in-order pass over the 64 lanes.
//   The labels are KwikCluster's whatever the interleaving (C4 is
//   serializable).
//   ClusterWild! (createCluster): a vertex still unclustered when reached
//   becomes a center (compare-and-swap from "unclustered"), no waiting.  Its
//   labels depend on the interleaving.
//
// Centers then claim their neighbours with atomicMin on the center's rank
// (concurrency rule 2).  The label word of a vertex holds everything the
// waits need:
//   INF          not decided yet
//   -(rank + 1)  a center (rank = its position in pi); never changes again
//   INF - 1      a C4 vertex decided not to be a center, not yet claimed
//   r >= 0       claimed by the center of rank r (only ever decreases)
// and is read and written only with device-scope atomics, so a wave on one
// XCD sees another XCD's decisions.
//
// Progress: chunks are handed out in pi order (a run of AS_BATCH
// consecutive chunks per visit to the counter, worked through in order), and
// a wave waits only for vertices of earlier chunks: its own, finished, or
// ones handed out before its run, which running waves hold and whose own
// waits point further back still.  The earliest unfinished chunk is the one
// its wave is working on, and it never waits.  A wave takes a new run only
// after finishing the last, so no resident-set assumption is needed.  Every
// wait is bounded (and stops when another wave has reported an error);
// every wave leaves when the counter passes the last chunk.
#include "cc_device.h"
#include "cc_launch.h"

namespace ccd {

constexpr int AS_BS = 256;  // 4 waves per workgroup, each on its own chunks
constexpr int AS_BIG = 2048;  // C4 centers with longer rows claim in a second, device-wide pass
// chunks a wave takes per visit to the shared counter (one device-scope
// atomic on one address serialises with every other wave's)
constexpr int AS_BATCH = 8;
constexpr int32_t LAB_NONCENTER = INF - 1;
constexpr unsigned AS_SPIN_LIMIT = 1u << 24;

__device__ inline int32_t lab_load(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Row of each pending lane walked edge-balanced by the whole wave: entry e
// of the concatenated rows belongs to the first lane j whose inclusive
// prefix incl_j exceeds e (six steps of a lane-indexed binary search).
__device__ inline int owner_lane(int64_t incl, int64_t e) {
  int j = 0;
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1) {
    const int64_t pj = __shfl(incl, j + step - 1, 64);
    if (pj <= e) j += step;
  }
  return j;
}

__device__ inline unsigned long long wave_or(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x |= __shfl_xor(x, d, 64);
  return x;
}

template <int ALGO>
__global__ void __launch_bounds__(AS_BS) k_async(AsyncArgs a) {
  Ctrl *c = a.ctrl;
  const int lane = lane_id();
  __shared__ unsigned long long s_intra[AS_BS / 64][64];
  unsigned long long *intra = s_intra[wave_id()];
  const int64_t nchunks = (a.n + 63) / 64;
  unsigned long long walked = 0, claimed = 0, atoms = 0, waits = 0;
  int64_t chunk = 0, chunk_end = 0;  // the wave's current run of AS_BATCH chunks
  for (;; chunk++) {
    if (chunk >= chunk_end) {
      int64_t b = 0;
      if (lane == 0) b = (int64_t)atomicAdd(&c->tile_counter, 1u) * AS_BATCH;
      chunk = __shfl(b, 0, 64);
      chunk_end = chunk + AS_BATCH < nchunks ? chunk + AS_BATCH : nchunks;
    }
    if (chunk >= nchunks) break;
    if (ld_rlx(&c->error)) break;
    const int64_t c0 = chunk * 64, p = c0 + lane;
    int32_t v = -1;
    if (p < a.n) v = a.order[p];
    // isolated vertices are their own clusters: k_async_finalize labels them
    const bool live = v >= 0 && v < a.iso_start;
    const bool pending = live && lab_load(&a.lab[v]) == INF;  // else claimed already: not a center
    int64_t start = 0;
    int32_t deg = 0;
    if (pending) {
      start = a.off[v];
      deg = (int32_t)(a.off[v + 1] - start);
    }
    unsigned long long centers = 0;
    if (ALGO == ALGO_C4) {
      // isCenter: earlier-ranked neighbours, edge-balanced over the pending rows
      intra[lane] = 0;
      const int64_t incl = wave_incl_scan(deg);
      const int64_t total = __shfl(incl, 63, 64);
      const unsigned long long pend = __ballot(pending);
      unsigned long long blocked = 0;
      for (int64_t base = 0; base < total; base += 64) {
        if ((blocked & pend) == pend) break;  // every pending vertex already has an earlier center
        // lane-indexed shuffles run with the whole wave active
        const int64_t e = base + lane;
        const int j = owner_lane(incl, e < total ? e : total - 1);
        const int64_t row_start = __shfl(start, j, 64);
        const int64_t row_first = __shfl(incl, j, 64) - __shfl((int64_t)deg, j, 64);
        bool found = false;
        if (e < total && !(blocked >> j & 1)) {
          const int32_t u = a.col[row_start + (e - row_first)];
          const int64_t pj = c0 + j;
          const int32_t ru = a.rank[u];
          walked++;
          if (ru < pj) {
            if (ru >= c0) {
              atomicOr(&intra[j], 1ull << (ru - c0));  // same chunk: settled below
            } else {
              int32_t x = lab_load(&a.lab[u]);
              unsigned spins = 0;
              while (x == INF) {  // wait until the earlier neighbour is decided
                if (++spins > AS_SPIN_LIMIT) {
                  set_error(c, ERR_NO_PROGRESS);
                  break;
                }
                if ((spins & 255) == 0 && ld_rlx(&c->error)) break;
                __builtin_amdgcn_s_sleep(2);
                x = lab_load(&a.lab[u]);
              }
              waits += spins;
              found = x < 0;  // a center
            }
          }
        }
        blocked |= wave_or(found ? 1ull << j : 0ull);
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // same-chunk dependences: in pi order, lane by lane
      const unsigned long long my_intra = intra[lane];
      const unsigned long long cand = pend & ~blocked;
      if (__ballot((cand >> lane & 1) && my_intra != 0)) {
        for (int l = 0; l < 64; l++) {
          const unsigned long long il = __shfl(my_intra, l, 64);
          if ((cand >> l & 1) && !(il & centers)) centers |= 1ull << l;
        }
      } else {
        centers = cand;
      }
      if (pending) {
        if (centers >> lane & 1) __hip_atomic_store(&a.lab[v], -(int32_t)p - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else atomicMin(&a.lab[v], LAB_NONCENTER);
      }
    } else {
      // createCluster: a vertex still unclustered becomes a center
      bool won = false;
      if (pending) won = atomicCAS(&a.lab[v], INF, -(int32_t)p - 1) == INF;
      centers = __ballot(won);
    }
    // claims: the centers' rows, edge-balanced over the wave.  A C4 center
    // with a long row is listed and claims in k_async_big instead, spread over
    // the whole device: a label only decides whether its vertex is still
    // unclustered when reached, and a C4 vertex that should have been claimed
    // already finds its earlier center in isCenter anyway.  (ClusterWild! has
    // no such check, so its claims are never put off.)
    bool defer = false;
    if (ALGO == ALGO_C4 && (centers >> lane & 1) && deg > AS_BIG) {
      const unsigned slot = atomicAdd(&c->n_blocked, 1u);
      if ((int64_t)slot < a.big_cap) {
        a.big_v[slot] = v;
        a.big_p[slot] = (int32_t)p;
        defer = true;
      } else {
        set_error(c, ERR_OVERFLOW);  // cannot happen: a list slot per vertex
      }
    }
    const int32_t cdeg = (centers >> lane & 1) && !defer ? deg : 0;
    const int64_t incl = wave_incl_scan(cdeg);
    const int64_t total = __shfl(incl, 63, 64);
    for (int64_t base = 0; base < total; base += 64) {
      const int64_t e = base + lane;
      const int j = owner_lane(incl, e < total ? e : total - 1);
      const int64_t row_start = __shfl(start, j, 64);
      const int64_t row_first = __shfl(incl, j, 64) - __shfl((int64_t)cdeg, j, 64);
      if (e < total) {
        const int32_t u = a.col[row_start + (e - row_first)];
        const int32_t pj = (int32_t)(c0 + j);
        claimed++;
        if (a.lab[u] > pj) {  // stale reads are safe: a label only decreases
          atomicMin(&a.lab[u], pj);
          atoms++;
        }
      }
    }
  }
  const int64_t s0 = wave_sum((int64_t)walked), s1 = wave_sum((int64_t)claimed), s2 = wave_sum((int64_t)atoms),
                s3 = wave_sum((int64_t)waits);
  if (lane == 0) {
    const int slot = (blockIdx.x * (AS_BS / 64) + wave_id()) & 63;
    if (s0) atomicAdd(&c->spread_lone[slot], (unsigned long long)s0);
    if (s1) atomicAdd(&c->x_low[slot], (unsigned long long)s1);
    if (s2) atomicAdd(&c->spread_atom[slot], (unsigned long long)s2);
    if (s3) atomicAdd(&c->spread_conf[slot], (unsigned long long)s3);
  }
}

// The listed long-row claims: slice k of listed row i goes to workgroup
// (i + k) mod gridDim.x, so each row is spread over the device.
constexpr int AS_SLICE = 4096;

__global__ void __launch_bounds__(BS) k_async_big(AsyncArgs a) {
  Ctrl *c = a.ctrl;
  const int64_t nbig = c->n_blocked < a.big_cap ? (int64_t)c->n_blocked : a.big_cap;
  unsigned long long claimed = 0, atoms = 0;
  for (int64_t i = 0; i < nbig; i++) {
    const int32_t v = a.big_v[i], p = a.big_p[i];
    const int64_t start = a.off[v], deg = a.off[v + 1] - start;
    const int64_t nslices = (deg + AS_SLICE - 1) / AS_SLICE;
    for (int64_t k = ((int64_t)blockIdx.x - i % gridDim.x + gridDim.x) % gridDim.x; k < nslices; k += gridDim.x) {
      const int64_t e1 = (k + 1) * AS_SLICE < deg ? (k + 1) * AS_SLICE : deg;
      for (int64_t e = k * AS_SLICE + threadIdx.x; e < e1; e += BS) {
        const int32_t u = a.col[start + e];
        claimed++;
        if (a.lab[u] > p) {
          atomicMin(&a.lab[u], p);
          atoms++;
        }
      }
    }
  }
  const int64_t s1 = wave_sum((int64_t)claimed), s2 = wave_sum((int64_t)atoms);
  if (lane_id() == 0) {
    const int slot = (blockIdx.x * (BS / 64) + wave_id()) & 63;
    if (s1) atomicAdd(&c->x_low[slot], (unsigned long long)s1);
    if (s2) atomicAdd(&c->spread_atom[slot], (unsigned long long)s2);
  }
}

// pi in internal ids, each vertex's rank, and the permutation check: rank
// starts at -1 everywhere, and n entries in range that leave no vertex
// without a rank name every vertex once.
__global__ void __launch_bounds__(BS) k_async_order(AsyncArgs a, const int32_t *order_in, const int32_t *perm,
                                                    int32_t *iorder) {
  for (int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x; k < a.n; k += (int64_t)gridDim.x * BS) {
    const int32_t v = order_in[k];
    if (v < 0 || (int64_t)v >= a.n) {
      set_error(a.ctrl, ERR_PERM);
      iorder[k] = -1;
    } else {
      const int32_t vi = perm[v];
      iorder[k] = vi;
      a.rank[vi] = (int32_t)k;
    }
  }
}

// check: the permutation check still to finish (after k_async_order; the
// bucketed mapping checks by itself)
__global__ void __launch_bounds__(BS) k_async_init(AsyncArgs a, int check) {
  for (int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x; v < a.n; v += (int64_t)gridDim.x * BS) {
    if (check && a.rank[v] < 0) set_error(a.ctrl, ERR_PERM);  // no entry of pi names v
    a.lab[v] = INF;
  }
}

// Output labels by input id: a center's own id, a claimed vertex the id at
// its center's position; an isolated vertex is alone.
__global__ void __launch_bounds__(BS) k_async_finalize(AsyncArgs a, const int32_t *order_in, const int32_t *perm,
                                                       int32_t *labels) {
  for (int64_t vin = (int64_t)blockIdx.x * BS + threadIdx.x; vin < a.n; vin += (int64_t)gridDim.x * BS) {
    const int32_t v = perm[vin];
    if (v >= a.iso_start) {
      labels[vin] = (int32_t)vin;
      continue;
    }
    const int32_t l = a.lab[v];
    if (l < 0) {
      labels[vin] = (int32_t)vin;  // a center
    } else if (l >= LAB_NONCENTER || (int64_t)l >= a.n) {
      set_error(a.ctrl, ERR_LABEL);  // every vertex is settled when the kernel ends
      labels[vin] = -1;
    } else {
      labels[vin] = order_in[l];
    }
  }
}

static unsigned grid_n(int64_t n) {
  int64_t g = (n + BS - 1) / BS;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (unsigned)g;
}

hipError_t launch_async(const AsyncArgs &a, int algo, const int32_t *order_in, const int32_t *perm, int32_t *iorder,
                        int32_t *labels, int waves, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                        const OrderMap *om) {
  hipError_t e;
  if (om) {
    if ((e = launch_order_map(*om, order_in, perm, a.n, iorder, a.ctrl, s, a.rank)) != hipSuccess) return e;
  } else {
    if ((e = hipMemsetAsync(a.rank, 0xFF, sizeof(int32_t) * (size_t)a.n, s)) != hipSuccess) return e;  // every rank -1
    hipLaunchKernelGGL(k_async_order, dim3(grid_n(a.n)), dim3(BS), 0, s, a, order_in, perm, iorder);
  }
  hipLaunchKernelGGL(k_async_init, dim3(grid_n(a.n)), dim3(BS), 0, s, a, om ? 0 : 1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  auto kern = algo == ALGO_C4 ? k_async<ALGO_C4> : k_async<ALGO_CW>;
  int block = AS_BS, grid = 1;
  if (waves > 0 && waves < AS_BS / 64) {
    block = 64 * waves;
  } else if (waves > 0) {
    grid = (waves + AS_BS / 64 - 1) / (AS_BS / 64);
  } else {
    int dev = 0, cus = 0, per_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, AS_BS, 0)) != hipSuccess) return e;
    grid = cus * (per_cu > 0 ? per_cu : 1);
    const int64_t need = ((a.n + 63) / 64 + AS_BS / 64 - 1) / (AS_BS / 64);
    if (need < grid) grid = (int)(need > 0 ? need : 1);
  }
  if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, a);
  if (algo == ALGO_C4) hipLaunchKernelGGL(k_async_big, dim3(1024), dim3(BS), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev1 && (e = hipEventRecord(ev1, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_async_finalize, dim3(grid_n(a.n)), dim3(BS), 0, s, a, order_in, perm, labels);
  return hipGetLastError();
}

}  // namespace ccd
