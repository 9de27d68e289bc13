// cc_graph.hip -- graph set-up (row weights, input checks) and the
// disagreement cost of a clustering (the objective of Section 2 of
// arXiv 1507.05086):
//   cost = sum_k C(s_k, 2) + m - 2 m_in
// counted per graph of a batch.  Both passes over the adjacency use the
// edge-balanced walk, so hub rows do not serialise on one wave.
#include "cc_device.h"
#include "cc_launch.h"
#include "cc_walk.h"

namespace ccd {

// ------------------------------------------------------ prefix of weights --
// wall[v] = sum_{x<v} max(deg(x), 1): the "all rows" list of the walk.

constexpr int SCAN_T = 4;  // items per thread in the block scan

__global__ void __launch_bounds__(BS) k_wscan_local(const int64_t *off, int64_t n, int64_t *wall,
                                                    int64_t *blocksum) {
  __shared__ int64_t sh[WAVES + 1];
  const int64_t base = ((int64_t)blockIdx.x * BS + threadIdx.x) * SCAN_T;
  int64_t x[SCAN_T], s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_T; k++) {
    const int64_t v = base + k;
    x[k] = 0;
    if (v < n) {
      const int64_t d = off[v + 1] - off[v];
      x[k] = d > 0 ? d : 1;
    }
    s += x[k];
  }
  int64_t tot;
  int64_t pre = wg_excl_scan(s, &tot, sh);
#pragma unroll
  for (int k = 0; k < SCAN_T; k++) {
    const int64_t v = base + k;
    if (v < n) wall[v] = pre;
    pre += x[k];
  }
  if (threadIdx.x == 0) blocksum[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the block sums in place; total -> *out.
__global__ void __launch_bounds__(BS) k_wscan_blocks(int64_t *blocksum, int64_t nb, int64_t *out) {
  __shared__ int64_t sh[WAVES + 1];
  int64_t carry = 0;
  for (int64_t i0 = 0; i0 < nb; i0 += BS) {
    const int64_t i = i0 + threadIdx.x;
    const int64_t x = i < nb ? blocksum[i] : 0;
    int64_t tot;
    const int64_t pre = wg_excl_scan(x, &tot, sh);
    if (i < nb) blocksum[i] = carry + pre;
    carry += tot;
  }
  if (threadIdx.x == 0) *out = carry;
}

__global__ void __launch_bounds__(BS) k_wscan_add(int64_t *wall, int64_t n, const int64_t *blocksum,
                                                  const int64_t *total) {
  const int64_t base = ((int64_t)blockIdx.x * BS + threadIdx.x) * SCAN_T;
  const int64_t add = blocksum[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_T; k++) {
    const int64_t v = base + k;
    if (v < n) wall[v] += add;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) wall[n] = *total;
}

hipError_t launch_row_weights(const int64_t *off, int64_t n, int64_t *wall, int64_t *blocksum,
                              hipStream_t s) {
  const int64_t per = (int64_t)BS * SCAN_T;
  const int64_t nb = (n + per - 1) / per;
  if (nb == 0) {
    return hipMemsetAsync(wall, 0, sizeof(int64_t), s);
  }
  hipLaunchKernelGGL(k_wscan_local, dim3((unsigned)nb), dim3(BS), 0, s, off, n, wall, blocksum);
  hipLaunchKernelGGL(k_wscan_blocks, dim3(1), dim3(BS), 0, s, blocksum, nb, blocksum + nb);
  hipLaunchKernelGGL(k_wscan_add, dim3((unsigned)nb), dim3(BS), 0, s, wall, n, blocksum, blocksum + nb);
  return hipGetLastError();
}

// ---------------------------------------------------------------- checks --

struct CheckArgs {
  const int64_t *off;
  const int32_t *col;
  const int64_t *wall;
  int64_t n;
  const int64_t *vtx_ptr;  // device, or null
  const int32_t *gid;      // device per-row graph id, or null
  int validate;
  int *err;                // (priority << 8 | cc_status code) of the worst failure, 0x7fffffff = none
};

// A column outside its graph outranks every other finding (the others may be
// its consequences); then the smallest code wins.
__device__ inline void report(int *err, int code) { atomicMin(err, ((code == 10 ? 0 : 1) << 8) | code); }

__device__ inline bool row_contains(const int64_t *off, const int32_t *col, int64_t row, int32_t x) {
  int64_t lo = off[row], hi = off[row + 1];
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (col[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < off[row + 1] && col[lo] == x;
}

__global__ void __launch_bounds__(BS) k_check(CheckArgs a) {
  lb_walk(nullptr, a.wall, a.n, a.wall[a.n], a.off, a.off + 1, a.col, nullptr, nullptr, [&](Items &it) {
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      if (!(it.edge >> k & 1)) continue;
      const int32_t v = it.v[k], u = it.u[k];
      int64_t base = 0, ng = a.n;
      if (a.gid) {
        const int32_t g = a.gid[v];
        base = a.vtx_ptr[g];
        ng = a.vtx_ptr[g + 1] - base;
      }
      if (u < 0 || (int64_t)u >= ng) {
        report(a.err, 10);  // CC_ERR_OUT_OF_RANGE
        continue;
      }
      if (!a.validate) continue;
      const int32_t vl = (int32_t)(v - base);
      if (u == vl) report(a.err, 3);  // CC_ERR_SELF_LOOP
      const int64_t e = it.pos[k];
      if (e + 1 < a.off[v + 1] && a.col[e + 1] <= u) report(a.err, 4);  // CC_ERR_DUPLICATE_EDGE
      if (!row_contains(a.off, a.col, base + u, vl)) report(a.err, 2);   // CC_ERR_NOT_SYMMETRIC
    }
  });
}

__global__ void k_gid(const int64_t *vtx_ptr, int32_t num_graphs, int32_t *gid) {
  for (int32_t g = blockIdx.x; g < num_graphs; g += gridDim.x)
    for (int64_t v = vtx_ptr[g] + threadIdx.x; v < vtx_ptr[g + 1]; v += blockDim.x) gid[v] = g;
}

hipError_t launch_graph_setup(const int64_t *off, const int32_t *col, int64_t n, const int64_t *vtx_ptr,
                              int32_t num_graphs, int32_t *gid, int64_t *wall, int64_t *blocksum,
                              int validate, int *err, hipStream_t s) {
  hipError_t e = launch_row_weights(off, n, wall, blocksum, s);
  if (e != hipSuccess) return e;
  if (gid) hipLaunchKernelGGL(k_gid, dim3(num_graphs < 4096 ? num_graphs : 4096), dim3(BS), 0, s, vtx_ptr,
                              num_graphs, gid);
  if (n > 0) {
    CheckArgs a{off, col, wall, n, vtx_ptr, gid, validate, err};
    hipLaunchKernelGGL(k_check, dim3(4096), dim3(BS), 0, s, a);
  }
  return hipGetLastError();
}

// ------------------------------------------------------ bound buckets ----

__global__ void __launch_bounds__(BS) k_level_count(const int64_t *off, int64_t n, unsigned *count, int *max_deg) {
  __shared__ unsigned s_cnt[NLVL];
  __shared__ int s_max;
  if (threadIdx.x < NLVL) s_cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  int mx = 0;
  for (int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x; v < n; v += (int64_t)gridDim.x * BS) {
    const int64_t d = off[v + 1] - off[v];
    if (d > mx) mx = (int)d;
    if (d >= DSW) atomicAdd(&s_cnt[level_of(d)], 1u);
  }
  mx = wave_max(mx);
  if (lane_id() == 0) atomicMax(&s_max, mx);
  __syncthreads();
  if (threadIdx.x < NLVL && s_cnt[threadIdx.x]) atomicAdd(&count[threadIdx.x], s_cnt[threadIdx.x]);
  if (threadIdx.x == 0 && s_max) atomicMax(max_deg, s_max);
}

// Each workgroup takes a contiguous chunk: counts per level in LDS, reserves
// its ranges with one atomic per level, then writes.
__global__ void __launch_bounds__(BS) k_level_fill(const int64_t *off, int64_t n, const int64_t *lvl_off,
                                                   unsigned *cursor, int32_t *lvl) {
  __shared__ unsigned s_cnt[NLVL], s_base[NLVL];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t v0 = (int64_t)blockIdx.x * per, v1 = v0 + per < n ? v0 + per : n;
  if (threadIdx.x < NLVL) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t v = v0 + threadIdx.x; v < v1; v += BS) {
    const int64_t d = off[v + 1] - off[v];
    if (d >= DSW) atomicAdd(&s_cnt[level_of(d)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < NLVL) {
    s_base[threadIdx.x] = s_cnt[threadIdx.x] ? atomicAdd(&cursor[threadIdx.x], s_cnt[threadIdx.x]) : 0u;
    s_cnt[threadIdx.x] = 0;
  }
  __syncthreads();
  for (int64_t v = v0 + threadIdx.x; v < v1; v += BS) {
    const int64_t d = off[v + 1] - off[v];
    if (d >= DSW) {
      const int k = level_of(d);
      const unsigned p = s_base[k] + atomicAdd(&s_cnt[k], 1u);
      lvl[lvl_off[k] + p] = (int32_t)v;
    }
  }
}

hipError_t launch_level_count(const int64_t *off, int64_t n, unsigned *count, int *max_deg, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t g = (n + BS - 1) / BS < 2048 ? (n + BS - 1) / BS : 2048;
  hipLaunchKernelGGL(k_level_count, dim3((unsigned)g), dim3(BS), 0, s, off, n, count, max_deg);
  return hipGetLastError();
}

hipError_t launch_level_fill(const int64_t *off, int64_t n, const int64_t *lvl_off, unsigned *cursor,
                             int32_t *lvl, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t g = (n + BS - 1) / BS < 4096 ? (n + BS - 1) / BS : 4096;
  hipLaunchKernelGGL(k_level_fill, dim3((unsigned)g), dim3(BS), 0, s, off, n, lvl_off, cursor, lvl);
  return hipGetLastError();
}

// ----------------------------------------------------------- renumbering --
// Internal vertex ids group the vertices by degree level floor(log2 deg),
// highest level first and isolated vertices last.  A neighbour scan touches
// a vertex about as often as its degree, so the per-vertex state it reads
// most (that of the hubs) sits in a few contiguous lines that stay cached.
// Within a level the order is whatever the atomics give: no result depends
// on internal ids (labels and every record are mapped back or id-free).
constexpr int RBINS = NLVL + 1;
__device__ inline int relabel_bin(int64_t d) { return d > 0 ? NLVL - 1 - level_of(d) : NLVL; }

__global__ void __launch_bounds__(BS) k_relabel_count(const int64_t *off, int64_t n, unsigned *count) {
  __shared__ unsigned s_cnt[RBINS];
  if (threadIdx.x < RBINS) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x; v < n; v += (int64_t)gridDim.x * BS)
    atomicAdd(&s_cnt[relabel_bin(off[v + 1] - off[v])], 1u);
  __syncthreads();
  if (threadIdx.x < RBINS && s_cnt[threadIdx.x]) atomicAdd(&count[threadIdx.x], s_cnt[threadIdx.x]);
}

// Each workgroup takes a contiguous chunk, reserves its range in every bin
// with one atomic, then places its vertices.
__global__ void __launch_bounds__(BS) k_relabel_assign(const int64_t *off, int64_t n, const int64_t *bin_off,
                                                       unsigned *cursor, int32_t *perm, int32_t *iperm) {
  __shared__ unsigned s_cnt[RBINS], s_base[RBINS];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t v0 = (int64_t)blockIdx.x * per, v1 = v0 + per < n ? v0 + per : n;
  if (threadIdx.x < RBINS) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t v = v0 + threadIdx.x; v < v1; v += BS) atomicAdd(&s_cnt[relabel_bin(off[v + 1] - off[v])], 1u);
  __syncthreads();
  if (threadIdx.x < RBINS) {
    s_base[threadIdx.x] = s_cnt[threadIdx.x] ? atomicAdd(&cursor[threadIdx.x], s_cnt[threadIdx.x]) : 0u;
    s_cnt[threadIdx.x] = 0;
  }
  __syncthreads();
  for (int64_t v = v0 + threadIdx.x; v < v1; v += BS) {
    const int b = relabel_bin(off[v + 1] - off[v]);
    const int64_t p = bin_off[b] + s_base[b] + atomicAdd(&s_cnt[b], 1u);
    perm[v] = (int32_t)p;
    iperm[p] = (int32_t)v;
  }
}

// rdeg[i] = degree of internal vertex i (its original row's length)
__global__ void __launch_bounds__(BS) k_relabel_degrees(const int64_t *off, int64_t n, const int32_t *iperm,
                                                        int64_t *rdeg) {
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const int32_t v = iperm[i];
    rdeg[i] = off[v + 1] - off[v];
  }
}

// Exclusive scan of rdeg into roff (block partial sums, then their scan, then add).
__global__ void __launch_bounds__(BS) k_plain_scan_local(const int64_t *x_in, int64_t n, int64_t *out,
                                                         int64_t *blocksum) {
  __shared__ int64_t sh[WAVES + 1];
  const int64_t base = ((int64_t)blockIdx.x * BS + threadIdx.x) * SCAN_T;
  int64_t x[SCAN_T], s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_T; k++) {
    x[k] = base + k < n ? x_in[base + k] : 0;
    s += x[k];
  }
  int64_t tot;
  int64_t pre = wg_excl_scan(s, &tot, sh);
#pragma unroll
  for (int k = 0; k < SCAN_T; k++) {
    if (base + k < n) out[base + k] = pre;
    pre += x[k];
  }
  if (threadIdx.x == 0) blocksum[blockIdx.x] = tot;
}

// rcol[roff[perm[v]] + j] = perm[col[off[v] + j]], edge-balanced over the input rows.
__global__ void __launch_bounds__(BS) k_relabel_cols(const int64_t *off, const int32_t *col, const int64_t *wall,
                                                     int64_t n, const int32_t *perm, const int64_t *roff,
                                                     int32_t *rcol) {
  lb_walk(nullptr, wall, n, wall[n], off, off + 1, col, perm, nullptr, [&](Items &it) {
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      if (!(it.edge >> k & 1)) continue;
      const int64_t local = it.pos[k] - off[it.v[k]];
      rcol[roff[it.val[k]] + local] = perm[it.u[k]];
    }
  });
}

hipError_t launch_relabel(const int64_t *off, const int32_t *col, const int64_t *wall, int64_t n, unsigned *count,
                          int64_t *bin_off_dev, int32_t *perm, int32_t *iperm, int64_t *rdeg, int64_t *roff,
                          int64_t *blocksum, int32_t *rcol, int64_t *first_low, int64_t *first_isolated,
                          hipStream_t s) {
  *first_low = n;
  *first_isolated = n;
  if (n == 0) return hipMemsetAsync(roff, 0, sizeof(int64_t), s);
  const unsigned g = (unsigned)((n + BS - 1) / BS < 4096 ? (n + BS - 1) / BS : 4096);
  hipError_t e = hipMemsetAsync(count, 0, sizeof(unsigned) * 2 * RBINS, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_relabel_count, dim3(g), dim3(BS), 0, s, off, n, count);
  unsigned hc[RBINS];
  e = hipMemcpyAsync(hc, count, sizeof(hc), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  int64_t hb[RBINS], acc = 0;
  for (int b = 0; b < RBINS; b++) {
    hb[b] = acc;
    acc += hc[b];
  }
  *first_isolated = hb[RBINS - 1];
  *first_low = hb[NLVL - 1 - level_of(DSW - 1)];  // the bin of degree DSW - 1
  e = hipMemcpyAsync(bin_off_dev, hb, sizeof(hb), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_relabel_assign, dim3(g), dim3(BS), 0, s, off, n, bin_off_dev, count + RBINS, perm, iperm);
  hipLaunchKernelGGL(k_relabel_degrees, dim3(g), dim3(BS), 0, s, off, n, iperm, rdeg);
  const int64_t per = (int64_t)BS * SCAN_T;
  const int64_t nb = (n + per - 1) / per;
  hipLaunchKernelGGL(k_plain_scan_local, dim3((unsigned)nb), dim3(BS), 0, s, rdeg, n, roff, blocksum);
  hipLaunchKernelGGL(k_wscan_blocks, dim3(1), dim3(BS), 0, s, blocksum, nb, blocksum + nb);
  hipLaunchKernelGGL(k_wscan_add, dim3((unsigned)nb), dim3(BS), 0, s, roff, n, blocksum, blocksum + nb);
  hipLaunchKernelGGL(k_relabel_cols, dim3(4096), dim3(BS), 0, s, off, col, wall, n, perm, roff, rcol);
  return hipGetLastError();
}

// ------------------------------------------------------------------ cost --

struct CostArgs {
  const int64_t *off;
  const int32_t *col;
  const int64_t *wall;
  int64_t n;
  const int64_t *vtx_ptr;
  const int32_t *gid;
  const int32_t *labels;
  int32_t *size;     // [n] cluster sizes, indexed by graph base + label
  long long *acc;    // [2 * num_graphs]: pairs inside clusters, same-label adjacency entries
  int *err;
};

// Per-lane running sums flushed when the graph changes; the whole workgroup
// adds once when every lane ends on the same graph.
__device__ inline void flush_acc(long long *acc, int slot, int g, long long x) {
  __shared__ int s_g, s_mixed;
  __shared__ long long s_sum;
  if (threadIdx.x == 0) {
    s_g = g;
    s_mixed = 0;
    s_sum = 0;
  }
  __syncthreads();
  if (g != s_g) s_mixed = 1;
  __syncthreads();
  if (s_mixed) {
    if (x) atomicAdd((unsigned long long *)&acc[2 * g + slot], (unsigned long long)x);
  } else {
    const long long ws = wave_sum(x);
    if (lane_id() == 0 && ws) atomicAdd((unsigned long long *)&s_sum, (unsigned long long)ws);
    __syncthreads();
    if (threadIdx.x == 0 && s_sum) atomicAdd((unsigned long long *)&acc[2 * g + slot], (unsigned long long)s_sum);
  }
}

__global__ void __launch_bounds__(BS) k_cost_sizes(CostArgs a) {
  for (int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x; v < a.n; v += (int64_t)gridDim.x * BS) {
    int64_t base = 0, ng = a.n;
    if (a.gid) {
      const int32_t g = a.gid[v];
      base = a.vtx_ptr[g];
      ng = a.vtx_ptr[g + 1] - base;
    }
    const int32_t l = a.labels[v];
    if (l < 0 || (int64_t)l >= ng) {
      report(a.err, 1);  // CC_ERR_INVALID_ARG: label outside its graph
      continue;
    }
    atomicAdd(&a.size[base + l], 1);
  }
}

__global__ void __launch_bounds__(BS) k_cost_same(CostArgs a) {
  int g_cur = -1;
  long long run = 0;
  lb_walk(nullptr, a.wall, a.n, a.wall[a.n], a.off, a.off + 1, a.col, a.labels, nullptr, [&](Items &it) {
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      if (!(it.edge >> k & 1)) continue;
      int g = 0;
      int64_t base = 0;
      if (a.gid) {
        g = a.gid[it.v[k]];
        base = a.vtx_ptr[g];
      }
      if (g != g_cur) {
        if (g_cur >= 0 && run) atomicAdd((unsigned long long *)&a.acc[2 * g_cur + 1], (unsigned long long)run);
        g_cur = g;
        run = 0;
      }
      if (a.labels[base + it.u[k]] == it.val[k]) run++;
    }
  });
  flush_acc(a.acc, 1, g_cur < 0 ? 0 : g_cur, run);
}

constexpr int PAIR_T = 64;  // consecutive label slots per thread

__global__ void __launch_bounds__(BS) k_cost_pairs(CostArgs a) {
  int g_cur = -1;
  long long run = 0;
  const int64_t stride = (int64_t)gridDim.x * BS * PAIR_T;
  for (int64_t r0 = ((int64_t)blockIdx.x * BS + threadIdx.x) * PAIR_T; r0 < a.n; r0 += stride) {
    for (int64_t r = r0; r < r0 + PAIR_T && r < a.n; r++) {
      const int g = a.gid ? a.gid[r] : 0;
      if (g != g_cur) {
        if (g_cur >= 0 && run) atomicAdd((unsigned long long *)&a.acc[2 * g_cur], (unsigned long long)run);
        g_cur = g;
        run = 0;
      }
      const long long s = a.size[r];
      run += s * (s - 1) / 2;
    }
  }
  flush_acc(a.acc, 0, g_cur < 0 ? 0 : g_cur, run);
}

hipError_t launch_cost(const int64_t *off, const int32_t *col, const int64_t *wall, int64_t n,
                       const int64_t *vtx_ptr, const int32_t *gid, const int32_t *labels, int32_t *size,
                       long long *acc, int32_t num_graphs, int *err, hipStream_t s) {
  hipError_t e = hipMemsetAsync(size, 0, sizeof(int32_t) * (size_t)(n > 0 ? n : 1), s);
  if (e == hipSuccess) e = hipMemsetAsync(acc, 0, sizeof(long long) * 2 * (size_t)num_graphs, s);
  if (e != hipSuccess || n == 0) return e;
  CostArgs a{off, col, wall, n, vtx_ptr, gid, labels, size, acc, err};
  const unsigned gv = (unsigned)((n + BS - 1) / BS < 4096 ? (n + BS - 1) / BS : 4096);
  hipLaunchKernelGGL(k_cost_sizes, dim3(gv), dim3(BS), 0, s, a);
  hipLaunchKernelGGL(k_cost_same, dim3(4096), dim3(BS), 0, s, a);
  const int64_t pg = (n + (int64_t)BS * PAIR_T - 1) / ((int64_t)BS * PAIR_T);
  hipLaunchKernelGGL(k_cost_pairs, dim3((unsigned)(pg < 2048 ? pg : 2048)), dim3(BS), 0, s, a);
  return hipGetLastError();
}

}  // namespace ccd
