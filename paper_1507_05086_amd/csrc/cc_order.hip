// cc_order.hip -- pi mapped into internal ids, iorder[k] = perm[pi[k]], and
// checked as a permutation of 0..n-1 (the input of Algorithm 2), for large n.
//
// The composition is a gather at random ids: done directly, every 4-byte
// entry of pi costs a whole memory line of perm, and marking the ids seen
// costs another random line.  Here the entries are instead bucketed twice so
// that every HBM access is a run of at least 64 bytes:
//   position bucket kb = k >> OM_SHIFT, id bucket vb = pi[k] >> OM_SHIFT;
//   k_om_count     per kb: how many of its entries fall in each vb (cnt[kb][vb])
//   k_om_tiles     64 x 64 tiles of cnt: column sums and row sums
//   k_om_scan      exclusive scans of the tile sums; id-bucket starts
//   k_om_offsets   every (kb, vb) segment's start on the id side (by kb
//                  row and by vb column) and on the position side (by vb)
//   k_om_scatter   per kb: its entries sorted by id bucket in LDS, then
//                  written into their id bucket's kb segment
//   k_om_gather    per vb: the bucket's slice of perm staged in LDS, each
//                  entry mapped, each id marked in an LDS bitmap (fewer
//                  marks than entries means pi repeats an id), written to
//                  its position bucket's vb segment
//   k_om_place     per kb: entries placed by position in LDS, written out
//                  in order.
// Out-of-range entries are reported and counted as id 0, so every offset
// stays within its array whatever the input holds.  n entries in range with
// no id marked twice is exactly a permutation.  Every workgroup of the
// bucket passes holds 1024 threads and OM_SIZE entries, 32 per thread.
#include "cc_device.h"
#include "cc_launch.h"

namespace ccd {

namespace {

constexpr int OM_BS = 1024;
constexpr unsigned OM_MASK = OM_SIZE - 1;
constexpr int OM_TILE = 64;
constexpr int OM_SCAN_BATCH = 16;
constexpr int OM_TBS = 256;
constexpr int OM_UNROLL = 8;

__global__ void __launch_bounds__(OM_BS) k_om_count(OrderMap m, const int32_t *order_in, int64_t n, Ctrl *ctrl) {
  __shared__ unsigned hist[OM_MAX_BUCKETS];
  for (int i = threadIdx.x; i < m.nv; i += OM_BS) hist[i] = 0;
  __syncthreads();
  const int64_t k0 = (int64_t)blockIdx.x * OM_SIZE, k1 = k0 + OM_SIZE < n ? k0 + OM_SIZE : n;
  bool bad = false;
  for (int64_t kk = k0 + threadIdx.x; kk < k1; kk += (int64_t)OM_UNROLL * OM_BS) {
    int32_t v[OM_UNROLL];
#pragma unroll
    for (int j = 0; j < OM_UNROLL; j++) {
      const int64_t k = kk + (int64_t)j * OM_BS;
      v[j] = k < k1 ? order_in[k] : 0;
    }
#pragma unroll
    for (int j = 0; j < OM_UNROLL; j++) {
      if (kk + (int64_t)j * OM_BS >= k1) break;
      int32_t x = v[j];
      if (x < 0 || (int64_t)x >= n) {
        bad = true;
        x = 0;
      }
      atomicAdd(&hist[x >> OM_SHIFT], 1u);
    }
  }
  if (bad) set_error(ctrl, ERR_PERM);
  __syncthreads();
  unsigned *row = m.cnt + (size_t)blockIdx.x * m.nv;
  for (int i = threadIdx.x; i < m.nv; i += OM_BS) row[i] = hist[i];
}

// Loads tile (tr, tc) of cnt into t, zero outside the matrix.
__device__ inline void load_tile(const OrderMap &m, int tr, int tc, unsigned (*t)[OM_TILE + 1]) {
  for (int i = threadIdx.x; i < OM_TILE * OM_TILE; i += OM_TBS) {
    const int r = i / OM_TILE, c = i % OM_TILE;
    const int kb = tr * OM_TILE + r, vb = tc * OM_TILE + c;
    t[r][c] = (kb < m.nk && vb < m.nv) ? m.cnt[(size_t)kb * m.nv + vb] : 0u;
  }
}

__global__ void __launch_bounds__(OM_TBS) k_om_tiles(OrderMap m) {
  __shared__ unsigned t[OM_TILE][OM_TILE + 1];
  const int tr = blockIdx.x / m.nvt, tc = blockIdx.x % m.nvt;
  load_tile(m, tr, tc, t);
  __syncthreads();
  const int x = threadIdx.x;
  if (x < OM_TILE) {  // column sums
    unsigned s = 0;
    for (int r = 0; r < OM_TILE; r++) s += t[r][x];
    const int vb = tc * OM_TILE + x;
    if (vb < m.nv) m.csum[(size_t)tr * m.nv + vb] = s;
  } else if (x < 2 * OM_TILE) {  // row sums
    const int r = x - OM_TILE;
    unsigned s = 0;
    for (int c = 0; c < OM_TILE; c++) s += t[r][c];
    const int kb = tr * OM_TILE + r;
    if (kb < m.nk) m.rsum[(size_t)tc * m.nk + kb] = s;
  }
}

// One workgroup: exclusive scans of the tile sums down each column and
// along each row, and the start of every id bucket.
__global__ void __launch_bounds__(OM_BS) k_om_scan(OrderMap m) {
  __shared__ unsigned tot[OM_MAX_BUCKETS];
  __shared__ int64_t sh[OM_BS / 64 + 1];
  // a column (row) is read OM_SCAN_BATCH tiles at a time, all in flight together
  for (int vb = threadIdx.x; vb < m.nv; vb += OM_BS) {
    unsigned run = 0;
    for (int t0 = 0; t0 < m.nkt; t0 += OM_SCAN_BATCH) {
      unsigned x[OM_SCAN_BATCH];
#pragma unroll
      for (int j = 0; j < OM_SCAN_BATCH; j++) x[j] = t0 + j < m.nkt ? m.csum[(t0 + j) * m.nv + vb] : 0u;
#pragma unroll
      for (int j = 0; j < OM_SCAN_BATCH; j++) {
        if (t0 + j < m.nkt) m.csum[(t0 + j) * m.nv + vb] = run;
        run += x[j];
      }
    }
    tot[vb] = run;
  }
  for (int kb = threadIdx.x; kb < m.nk; kb += OM_BS) {
    unsigned run = 0;
    for (int t0 = 0; t0 < m.nvt; t0 += OM_SCAN_BATCH) {
      unsigned x[OM_SCAN_BATCH];
#pragma unroll
      for (int j = 0; j < OM_SCAN_BATCH; j++) x[j] = t0 + j < m.nvt ? m.rsum[(t0 + j) * m.nk + kb] : 0u;
#pragma unroll
      for (int j = 0; j < OM_SCAN_BATCH; j++) {
        if (t0 + j < m.nvt) m.rsum[(t0 + j) * m.nk + kb] = run;
        run += x[j];
      }
    }
  }
  __syncthreads();
  // id-bucket starts: thread i owns buckets [i * per, (i + 1) * per)
  constexpr int per = OM_MAX_BUCKETS / OM_BS;
  int64_t s = 0;
  for (int j = 0; j < per; j++) {
    const int vb = threadIdx.x * per + j;
    if (vb < m.nv) s += tot[vb];
  }
  int64_t total;
  int64_t run = wg_excl_scan<OM_BS>(s, &total, sh);
  for (int j = 0; j < per; j++) {
    const int vb = threadIdx.x * per + j;
    if (vb < m.nv) {
      m.vstart[vb] = (unsigned)run;
      run += tot[vb];
    }
  }
  if (threadIdx.x == 0) m.vstart[m.nv] = (unsigned)total;
}

// Segment starts of tile (tr, tc).  Id side: vstart[vb] + the entries of vb
// in position buckets above kb, written by row into cnt (in place) and by
// column into pt.  Position side: kb * OM_SIZE + the entries of kb in id
// buckets left of vb, written by column into qt.
__global__ void __launch_bounds__(OM_TBS) k_om_offsets(OrderMap m) {
  __shared__ unsigned t[OM_TILE][OM_TILE + 1];
  __shared__ unsigned p[OM_TILE][OM_TILE + 1];
  __shared__ unsigned q[OM_TILE][OM_TILE + 1];
  const int tr = blockIdx.x / m.nvt, tc = blockIdx.x % m.nvt;
  load_tile(m, tr, tc, t);
  __syncthreads();
  const int x = threadIdx.x;
  if (x < OM_TILE) {
    const int vb = tc * OM_TILE + x;
    unsigned run = vb < m.nv ? m.csum[(size_t)tr * m.nv + vb] + m.vstart[vb] : 0u;
    for (int r = 0; r < OM_TILE; r++) {
      p[r][x] = run;
      run += t[r][x];
    }
  } else if (x < 2 * OM_TILE) {
    const int r = x - OM_TILE, kb = tr * OM_TILE + r;
    unsigned run = kb < m.nk ? m.rsum[(size_t)tc * m.nk + kb] + (unsigned)kb * OM_SIZE : 0u;
    for (int c = 0; c < OM_TILE; c++) {
      q[r][c] = run;
      run += t[r][c];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < OM_TILE * OM_TILE; i += OM_TBS) {
    {  // by row: consecutive threads take consecutive vb
      const int r = i / OM_TILE, c = i % OM_TILE;
      const int kb = tr * OM_TILE + r, vb = tc * OM_TILE + c;
      if (kb < m.nk && vb < m.nv) m.cnt[(size_t)kb * m.nv + vb] = p[r][c];
    }
    {  // by column: consecutive threads take consecutive kb
      const int c = i / OM_TILE, r = i % OM_TILE;
      const int kb = tr * OM_TILE + r, vb = tc * OM_TILE + c;
      if (kb < m.nk && vb < m.nv) {
        m.pt[(size_t)vb * m.nk + kb] = p[r][c];
        m.qt[(size_t)vb * m.nk + kb] = q[r][c];
      }
    }
  }
}

// The last index i in [0, len) with a[i] <= x[j], for OM_UNROLL keys at once
// (a non-decreasing, a[0] <= every key): a fixed number of steps, so the
// keys' LDS reads are in flight together.
__device__ inline void last_le(const unsigned *a, int len, const unsigned (&x)[OM_UNROLL], int (&at)[OM_UNROLL]) {
#pragma unroll
  for (int j = 0; j < OM_UNROLL; j++) at[j] = 0;
  int top = 1;
  while (top * 2 < len) top *= 2;
  for (int step = top; step > 0; step >>= 1) {
#pragma unroll
    for (int j = 0; j < OM_UNROLL; j++) {
      const int c = at[j] + step;
      if (c < len && a[c] <= x[j]) at[j] = c;
    }
  }
}

// Workgroups are dealt to the 8 XCDs round-robin by block index.  This maps
// block b to a bucket so that each XCD takes a contiguous range of buckets
// in order: neighbouring segments, which share memory lines, are then
// written through the same L2 at about the same time.
__device__ inline int xcd_bucket(int b, int count) {
  constexpr int XCDS = 8;
  const int q = count / XCDS, r = count % XCDS, x = b % XCDS, slot = b / XCDS;
  return x * q + (x < r ? x : r) + slot;
}

// Dynamic LDS of k_om_scatter: the chunk sorted by id bucket, per-bucket
// counts (then local starts) and segment starts in ent.
constexpr size_t OM_SCATTER_LDS = sizeof(unsigned) * OM_SIZE + 2 * sizeof(unsigned) * OM_MAX_BUCKETS;
constexpr int OM_PER_THREAD = OM_SIZE / OM_BS;

// Per position bucket: its entries sorted by id bucket in LDS (counting
// sort), then written out so that consecutive lanes write consecutive
// entries of a segment.
__global__ void __launch_bounds__(OM_BS) k_om_scatter(OrderMap m, const int32_t *order_in, int64_t n) {
  extern __shared__ __align__(16) uint8_t lds[];
  unsigned *buf = reinterpret_cast<unsigned *>(lds);
  unsigned *lstart = buf + OM_SIZE;
  unsigned *gbase = lstart + OM_MAX_BUCKETS;
  __shared__ int64_t sh[OM_BS / 64 + 1];
  const int kb = xcd_bucket(blockIdx.x, m.nk);
  const unsigned *row = m.cnt + (size_t)kb * m.nv;
  for (int i = threadIdx.x; i < OM_MAX_BUCKETS; i += OM_BS) {
    lstart[i] = 0;
    gbase[i] = i < m.nv ? row[i] : 0u;
  }
  __syncthreads();
  const int64_t k0 = (int64_t)kb * OM_SIZE;
  const int len = (int)(n - k0 < OM_SIZE ? n - k0 : OM_SIZE);
  // this thread's entries are k0 + threadIdx.x + j * OM_BS, all loaded at once
  unsigned vlo[OM_PER_THREAD], brk[OM_PER_THREAD];  // id low bits; bucket | local rank << 16
#pragma unroll
  for (int j = 0; j < OM_PER_THREAD; j++) {
    const int i = threadIdx.x + j * OM_BS;
    vlo[j] = i < len ? (unsigned)order_in[k0 + i] : 0u;
  }
#pragma unroll
  for (int j = 0; j < OM_PER_THREAD; j++) {
    const int i = threadIdx.x + j * OM_BS;
    unsigned x = vlo[j];
    if ((int64_t)(int32_t)x < 0 || (int64_t)(int32_t)x >= n) x = 0;  // reported by k_om_count
    const unsigned bk = x >> OM_SHIFT;
    vlo[j] = x & OM_MASK;
    brk[j] = i < len ? bk | (atomicAdd(&lstart[bk], 1u) << 16) : 0u;
  }
  __syncthreads();
  {  // counts -> local starts; thread t owns buckets [t * per, (t + 1) * per)
    constexpr int per = OM_MAX_BUCKETS / OM_BS;
    unsigned c[per];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < per; j++) {
      c[j] = lstart[threadIdx.x * per + j];
      s += c[j];
    }
    int64_t total;
    int64_t run = wg_excl_scan<OM_BS>(s, &total, sh);
#pragma unroll
    for (int j = 0; j < per; j++) {
      lstart[threadIdx.x * per + j] = (unsigned)run;
      run += c[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < OM_PER_THREAD; j++) {
    const unsigned i = threadIdx.x + j * OM_BS;
    if ((int)i < len) buf[lstart[brk[j] & 0xFFFFu] + (brk[j] >> 16)] = i | (vlo[j] << OM_SHIFT);
  }
  __syncthreads();
  for (int ib = threadIdx.x; ib < len; ib += OM_UNROLL * OM_BS) {
    unsigned key[OM_UNROLL], e[OM_UNROLL];
    int bk[OM_UNROLL];
#pragma unroll
    for (int j = 0; j < OM_UNROLL; j++) {
      const int i = ib + j * OM_BS;
      key[j] = i < len ? (unsigned)i : 0u;
      e[j] = i < len ? buf[i] : 0u;
    }
    last_le(lstart, m.nv, key, bk);  // the bucket of sorted entry i
#pragma unroll
    for (int j = 0; j < OM_UNROLL; j++) {
      const int i = ib + j * OM_BS;
      if (i < len) m.ent[gbase[bk[j]] + ((unsigned)i - lstart[bk[j]])] = e[j];
    }
  }
}

// Dynamic LDS of k_om_gather: perm slice, id bitmap, segment starts on both sides.
constexpr size_t OM_GATHER_LDS = sizeof(int32_t) * OM_SIZE + sizeof(unsigned) * (OM_SIZE / 32) +
                                 sizeof(unsigned) * (OM_MAX_BUCKETS + 1) + sizeof(unsigned) * OM_MAX_BUCKETS;
constexpr size_t OM_PLACE_LDS = sizeof(int32_t) * OM_SIZE;

// Per id bucket: every entry mapped through the bucket's slice of perm and
// its id marked; the bucket holds a repeated id exactly when fewer bits are
// set than it has entries.
__global__ void __launch_bounds__(OM_BS) k_om_gather(OrderMap m, const int32_t *perm, int64_t n, Ctrl *ctrl,
                                                    int32_t *rank) {
  extern __shared__ __align__(16) uint8_t lds[];
  int32_t *slice = reinterpret_cast<int32_t *>(lds);
  unsigned *bits = reinterpret_cast<unsigned *>(slice + OM_SIZE);
  unsigned *pcol = bits + OM_SIZE / 32;
  unsigned *qcol = pcol + OM_MAX_BUCKETS + 1;
  __shared__ int64_t sh[OM_BS / 64 + 1];
  const int vb = xcd_bucket(blockIdx.x, m.nv);
  const int64_t v0 = (int64_t)vb * OM_SIZE;
  const int len = (int)(n - v0 < OM_SIZE ? n - v0 : OM_SIZE);
  const int4 *src = reinterpret_cast<const int4 *>(perm + v0);  // v0 is a multiple of 4
  {
    constexpr int per = OM_SIZE / 4 / OM_BS;  // int4 loads per thread, all in flight together
    int4 t[per];
#pragma unroll
    for (int j = 0; j < per; j++) {
      const int i = threadIdx.x + j * OM_BS;
      if (i < len / 4) t[j] = src[i];
    }
#pragma unroll
    for (int j = 0; j < per; j++) {
      const int i = threadIdx.x + j * OM_BS;
      if (i < len / 4) reinterpret_cast<int4 *>(slice)[i] = t[j];
    }
  }
  for (int i = (len & ~3) + threadIdx.x; i < len; i += OM_BS) slice[i] = perm[v0 + i];
  for (int i = threadIdx.x; i < OM_SIZE / 32; i += OM_BS) bits[i] = 0;
  for (int kb = threadIdx.x; kb < m.nk; kb += OM_BS) {
    pcol[kb] = m.pt[(size_t)vb * m.nk + kb];
    qcol[kb] = m.qt[(size_t)vb * m.nk + kb];
  }
  const unsigned e0 = m.vstart[vb], e1 = m.vstart[vb + 1];
  __syncthreads();
  // OM_PER_THREAD entries per thread loaded at once (a valid pi gives every
  // bucket OM_SIZE entries, one such round), then mapped OM_UNROLL at a time
  for (unsigned ec = e0 + threadIdx.x; ec < e1; ec += OM_PER_THREAD * OM_BS) {
    unsigned x[OM_PER_THREAD];
#pragma unroll
    for (int j = 0; j < OM_PER_THREAD; j++) {
      const unsigned e = ec + j * OM_BS;
      x[j] = e < e1 ? m.ent[e] : 0u;
    }
#pragma unroll
    for (int jb = 0; jb < OM_PER_THREAD; jb += OM_UNROLL) {
      unsigned key[OM_UNROLL];
#pragma unroll
      for (int j = 0; j < OM_UNROLL; j++) {
        const unsigned e = ec + (jb + j) * OM_BS;
        key[j] = e < e1 ? e : e0;
      }
      int kb[OM_UNROLL];
      last_le(pcol, m.nk, key, kb);  // the position bucket whose segment holds e
#pragma unroll
      for (int j = 0; j < OM_UNROLL; j++) {
        const unsigned e = ec + (jb + j) * OM_BS;
        if (e < e1) {
          const unsigned kl = x[jb + j] & OM_MASK, vl = x[jb + j] >> OM_SHIFT;
          atomicOr(&bits[vl >> 5], 1u << (vl & 31));
          const int32_t vi = slice[vl];
          m.pent[qcol[kb[j]] + (e - pcol[kb[j]])] = ((unsigned long long)(uint32_t)vi << OM_SHIFT) | kl;
          // the renumbering keeps runs of input ids together, so these land in few runs
          if (rank) rank[vi] = (int32_t)((unsigned)kb[j] * OM_SIZE + kl);
        }
      }
    }
  }
  __syncthreads();
  int64_t set = 0;
  for (int i = threadIdx.x; i < OM_SIZE / 32; i += OM_BS) set += __popc(bits[i]);
  int64_t total;
  (void)wg_excl_scan<OM_BS>(set, &total, sh);
  if (threadIdx.x == 0 && total != (int64_t)(e1 - e0)) set_error(ctrl, ERR_PERM);
}

__global__ void __launch_bounds__(OM_BS) k_om_place(OrderMap m, int64_t n, int32_t *iorder) {
  extern __shared__ __align__(16) uint8_t lds[];
  int32_t *out = reinterpret_cast<int32_t *>(lds);
  const int64_t k0 = (int64_t)blockIdx.x * OM_SIZE;
  const int len = (int)(n - k0 < OM_SIZE ? n - k0 : OM_SIZE);
  for (int ib = threadIdx.x; ib < len; ib += OM_UNROLL * OM_BS) {
    unsigned long long x[OM_UNROLL];
#pragma unroll
    for (int j = 0; j < OM_UNROLL; j++) {
      const int i = ib + j * OM_BS;
      x[j] = i < len ? m.pent[k0 + i] : 0ull;
    }
#pragma unroll
    for (int j = 0; j < OM_UNROLL; j++)
      if (ib + j * OM_BS < len) out[x[j] & OM_MASK] = (int32_t)(x[j] >> OM_SHIFT);
  }
  __syncthreads();
  int4 *dst = reinterpret_cast<int4 *>(iorder + k0);  // k0 is a multiple of 4
  for (int i = threadIdx.x; i < len / 4; i += OM_BS) dst[i] = reinterpret_cast<const int4 *>(out)[i];
  for (int i = (len & ~3) + threadIdx.x; i < len; i += OM_BS) iorder[k0 + i] = out[i];
}

}  // namespace

bool order_map_applies(int64_t n) { return n > OM_MIN_N && n <= (int64_t)OM_MAX_BUCKETS * OM_SIZE; }

size_t order_map_bytes(int64_t n) {
  const int64_t nk = (n + OM_SIZE - 1) / OM_SIZE, nt = (nk + OM_TILE - 1) / OM_TILE;
  return sizeof(unsigned) * (size_t)(3 * nk * nk + 2 * nt * nk + nk + 1 + n) + sizeof(unsigned long long) * (size_t)n;
}

OrderMap order_map_layout(int64_t n, void *base) {
  OrderMap m{};
  m.nk = m.nv = (int)((n + OM_SIZE - 1) / OM_SIZE);
  m.nkt = m.nvt = (m.nk + OM_TILE - 1) / OM_TILE;
  unsigned long long *p64 = static_cast<unsigned long long *>(base);
  m.pent = p64;
  unsigned *p = reinterpret_cast<unsigned *>(p64 + n);
  const size_t mat = (size_t)m.nk * m.nv;
  m.cnt = p;
  m.pt = m.cnt + mat;
  m.qt = m.pt + mat;
  m.csum = m.qt + mat;
  m.rsum = m.csum + (size_t)m.nkt * m.nv;
  m.vstart = m.rsum + (size_t)m.nvt * m.nk;
  m.ent = m.vstart + m.nv + 1;
  return m;
}

hipError_t launch_order_map(const OrderMap &m, const int32_t *order_in, const int32_t *perm, int64_t n,
                            int32_t *iorder, Ctrl *ctrl, hipStream_t s, int32_t *rank) {
  // the LDS these kernels take beyond 64 KB, set for the current device on
  // every launch (a few microseconds; nothing cached across devices or errors)
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_om_scatter),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)OM_SCATTER_LDS);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_om_gather), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)OM_GATHER_LDS);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_om_place), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)OM_PLACE_LDS);
  if (e != hipSuccess) return e;
  if (!order_map_applies(n) || m.nk != (int)((n + OM_SIZE - 1) / OM_SIZE) || m.nv != m.nk) return hipErrorInvalidValue;
  const unsigned tiles = (unsigned)(m.nkt * m.nvt);
  hipLaunchKernelGGL(k_om_count, dim3(m.nk), dim3(OM_BS), 0, s, m, order_in, n, ctrl);
  hipLaunchKernelGGL(k_om_tiles, dim3(tiles), dim3(OM_TBS), 0, s, m);
  hipLaunchKernelGGL(k_om_scan, dim3(1), dim3(OM_BS), 0, s, m);
  hipLaunchKernelGGL(k_om_offsets, dim3(tiles), dim3(OM_TBS), 0, s, m);
  hipLaunchKernelGGL(k_om_scatter, dim3(m.nk), dim3(OM_BS), OM_SCATTER_LDS, s, m, order_in, n);
  hipLaunchKernelGGL(k_om_gather, dim3(m.nv), dim3(OM_BS), OM_GATHER_LDS, s, m, perm, n, ctrl, rank);
  hipLaunchKernelGGL(k_om_place, dim3(m.nk), dim3(OM_BS), OM_PLACE_LDS, s, m, n, iorder);
  return hipGetLastError();
}

}  // namespace ccd
