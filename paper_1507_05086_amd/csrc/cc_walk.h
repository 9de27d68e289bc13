// cc_walk.h -- edge-balanced walk over the adjacency rows of a vertex list.
//
// A list (vertices + exclusive prefix of their row weights max(deg,1)) is cut
// into equal item ranges, one per workgroup, so a hub row of 10^6 entries is
// shared by many workgroups while thousands of short rows share one.  Inside
// a workgroup the items are processed in tiles of TW: the row weights of the
// tile's rows are staged in LDS and each lane finds its row by binary search
// there (load-balanced search), then reads the adjacency entry with coalesced
// loads along the row.
#pragma once
#include <type_traits>

#include "cc_device.h"

namespace ccd {

// Items of one tile held by one thread.  Item k is an adjacency entry when
// bit k of `edge` is set (u[k] valid) and the first item of its row when bit
// k of `vert` is set (rows of degree 0 own exactly one such item).
struct Items {
  int ent[IPT];      // row index within the tile (LDS slot), -1 if no item
  int32_t v[IPT];    // row vertex
  int32_t u[IPT];    // neighbour (edge items)
  int32_t val[IPT];  // staged per-row value (e.g. rank or lab of v)
  int32_t deg[IPT];  // degree of v
  int64_t pos[IPT];  // position of the entry in col (edge items)
  unsigned edge, vert;
};

// first index in a[0..len) with a[i] > x (a sorted; a[len-1] may be a sentinel)
__device__ inline int lds_upper_bound(const int64_t *a, int len, int64_t x) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

struct NoEpilogue {
  __device__ void operator()(int, int64_t, int32_t, int32_t, int64_t) const {}
};
struct NoPost {
  __device__ void operator()() const {}
};

// Calls f(Items&) once per tile in every thread of the workgroup (uniformly,
// so f may use wave-wide operations).  Row v is col[off[v] .. end[v]) (end =
// off + 1 for a plain CSR).  `vals` (may be null) is gathered per row into
// Items::val.  A null `list` means the rows 0..cnt-1 themselves.
// With `info` (per list entry), rows come from it and Items::val is the rank.
// After f, ep(j, slot, v, deg, covered) runs once for every row j the tile
// touched (slot = list index, covered = items of that row in this tile), so
// per-row partial results kept in LDS by f can be combined across tiles; then
// post() runs in every thread (it may use barriers).
template <class F, class E = NoEpilogue, class P = NoPost>
__device__ void lb_walk(const int32_t *__restrict__ list, const int64_t *__restrict__ work, int64_t cnt,
                        int64_t total, const int64_t *__restrict__ off, const int64_t *__restrict__ end,
                        const int32_t *__restrict__ col,
                        const int32_t *__restrict__ vals, const RowInfo *__restrict__ info, F &&f, E &&ep = E(),
                        P &&post = P()) {
  __shared__ int64_t lw[TW + 1];
  __shared__ int32_t lv[TW];
  __shared__ int64_t loff[TW];
  __shared__ int32_t ldeg[TW];
  __shared__ int32_t lval[TW];
  __shared__ int64_t s_ent;
  __shared__ int s_nent, s_next;
  if (total <= 0 || cnt <= 0) return;
  const int64_t ntiles = (total + TW - 1) / TW;
  const int64_t nwg = ntiles < (int64_t)gridDim.x ? ntiles : (int64_t)gridDim.x;
  if ((int64_t)blockIdx.x >= nwg) return;
  const int64_t per = (ntiles + nwg - 1) / nwg;  // tiles per workgroup
  const int64_t s0 = (int64_t)blockIdx.x * per * TW;
  if (s0 >= total) return;
  const int64_t s1 = (s0 + per * TW) < total ? (s0 + per * TW) : total;
  if (threadIdx.x < 64) {
    const int64_t e = wave_find_entry(work, cnt, s0);
    if (threadIdx.x == 0) {
      s_ent = e;
      s_nent = 0;
      s_next = 0;
    }
  }
  __syncthreads();
  int64_t ent0 = s_ent;
  // the tile's window of row prefixes, held in registers so that the next
  // tile's window is in flight while this tile is processed
  constexpr int NPW = (TW + 1 + BS - 1) / BS;
  int64_t pw[NPW];
  auto load_window = [&](int64_t e0) {
#pragma unroll
    for (int q = 0; q < NPW; q++) {
      const int j = (int)threadIdx.x + q * BS;
      const int64_t idx = e0 + j;
      pw[q] = (j <= TW && idx < cnt) ? work[idx] : INT64_MAX;
    }
  };
  load_window(ent0);
  for (int64_t s = s0; s < s1; s += TW) {
    const int64_t send = (s + TW) < s1 ? (s + TW) : s1;
    // the window is sorted, so counting its entries below a bound is the
    // upper-bound search: rows touched by this tile, and where the next starts
    int c_rows = 0, c_next = 0;
#pragma unroll
    for (int q = 0; q < NPW; q++) {
      const int j = (int)threadIdx.x + q * BS;
      if (j <= TW) {
        lw[j] = pw[q];
        c_rows += pw[q] <= send - 1;
        c_next += pw[q] <= s + TW;
      }
    }
    const int64_t w_rows = wave_sum((int64_t)c_rows), w_next = wave_sum((int64_t)c_next);
    if (lane_id() == 0) {
      atomicAdd(&s_nent, (int)w_rows);
      atomicAdd(&s_next, (int)w_next);
    }
    __syncthreads();
    const int nent = s_nent;
    const int next = (s + TW < s1) ? s_next - 1 : 0;
    if (s + TW < s1) load_window(ent0 + next);  // the next tile's window
    for (int j = threadIdx.x; j < nent; j += BS) {
      const int32_t v = list ? list[ent0 + j] : (int32_t)(ent0 + j);
      lv[j] = v;
      if (info) {  // row info carried by the list: no offset or rank lookups
        const RowInfo ri = info[ent0 + j];
        loff[j] = ri.start;
        ldeg[j] = ri.deg;
        lval[j] = ri.rank;
      } else {
        const int64_t o = off[v];
        loff[j] = o;
        ldeg[j] = (int32_t)(end[v] - o);
        lval[j] = vals ? vals[v] : 0;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // every thread has read them; the next tile counts afresh
      s_nent = 0;
      s_next = 0;
    }
    Items it;
    it.edge = 0;
    it.vert = 0;
    int64_t epos[IPT];
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      const int64_t item = s + (int64_t)k * BS + threadIdx.x;
      it.v[k] = 0;
      it.u[k] = 0;
      it.val[k] = 0;
      it.deg[k] = 0;
      it.pos[k] = -1;
      it.ent[k] = -1;
      epos[k] = -1;
      if (item < send) {
        const int j = lds_upper_bound(lw, nent, item) - 1;
        const int64_t local = item - lw[j];
        it.ent[k] = j;
        it.v[k] = lv[j];
        it.val[k] = lval[j];
        it.deg[k] = ldeg[j];
        if (local == 0) it.vert |= 1u << k;
        if (local < ldeg[j]) {
          it.edge |= 1u << k;
          epos[k] = loff[j] + local;
          it.pos[k] = epos[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < IPT; k++)
      if (epos[k] >= 0) it.u[k] = col[epos[k]];
    f(it);
    if constexpr (!std::is_same<typename std::decay<E>::type, NoEpilogue>::value) {
      __syncthreads();
      for (int j = threadIdx.x; j < nent; j += BS) {
        const int64_t w0 = lw[j], w1 = w0 + (ldeg[j] > 0 ? ldeg[j] : 1);
        const int64_t lo = w0 > s ? w0 : s, hi = w1 < send ? w1 : send;
        ep(j, ent0 + j, lv[j], ldeg[j], hi - lo);
      }
    }
    if constexpr (!std::is_same<typename std::decay<P>::type, NoPost>::value) post();
    ent0 += next;
    __syncthreads();
  }
}

}  // namespace ccd
