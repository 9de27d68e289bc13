// cc_rounds.hip -- the bulk-synchronous round loop of C4 and ClusterWild!
// (arXiv 1507.05086, Algorithm 2) as a sequence of gfx950 kernels per round:
//
//   select    next B_i unclustered vertices of pi (lazy deletion: a cursor
//             walks pi once); one pass with decoupled look-back
//   elect     C4 only: does an active vertex have an earlier-ranked active
//             neighbour?  (concurrency rule 1; edge-balanced)
//   classify  C4 only: roots become centers; the last workgroup resolves the
//             blocked ones as a fixed point over the conflict edges (the
//             greedy MIS of G[A] in pi order, wait-free)
//   claim     every center claims its eligible neighbours with atomicMin on
//             the center rank (concurrency rule 2, createCluster)
//   peel      clustered vertices leave; their unclustered neighbours lose one
//             remaining degree each (lazy deletion: the CSR is never changed)
//   delta     max remaining degree Delta_{i+1}; the last workgroup closes the
//             round (trace record) and sizes the next active set
//
// Every kernel returns at once when the run is done, so the host can queue
// rounds in groups and look at the done flag once per group.
#include "cc_device.h"
#include "cc_launch.h"
#include "cc_walk.h"

namespace ccd {

// ------------------------------------------------------------------ init --

__global__ void __launch_bounds__(BS) k_invert(Ws w) {
  const int64_t n = w.n;
  for (int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x; k < n; k += (int64_t)gridDim.x * BS) {
    const int32_t v = w.order[k];
    if (v < 0 || (int64_t)v >= n) {
      set_error(w.ctrl, ERR_PERM);
      continue;
    }
    const int32_t old = atomicExch(&w.rank[v], (int32_t)k);
    if (old != -1) set_error(w.ctrl, ERR_PERM);
  }
}

__global__ void __launch_bounds__(BS) k_init(Ws w) {
  const int64_t n = w.n;
  for (int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x; v < n; v += (int64_t)gridDim.x * BS) {
    w.lab[v] = INF;
    w.state[v] = UNCL;
    w.flag[v] = 0;
    w.resdeg[v] = (int32_t)(w.off[v + 1] - w.off[v]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctrl *c = w.ctrl;
    c->n_rem = n;
    c->n_start = n;
    c->done = (n == 0);
    c->feat_eps = (float)w.eps;
  }
}

// ------------------------------------------------------------ policy ------

__device__ inline long long fixed_batch(long long eps_q, long long n_rem, long long delta) {
  if (delta <= 0) return n_rem;
  const long long num = eps_q * n_rem, den = 1000000LL * delta;
  long long b = (num + den - 1) / den;
  if (b < 1) b = 1;
  if (b > n_rem) b = n_rem;
  return b;
}

// Learned policy: eps = clamp(exp(w2 . relu(W1 x + b1) + b2)).  Wave 0 only;
// lane j computes hidden unit j.  Returns false on a non-finite output.
__device__ inline bool mlp_eps(const Ws &w, const float x[6], float *eps_out) {
  const float *W1 = w.mlp, *b1 = w.mlp + 64 * 6, *w2 = b1 + 64, *b2 = w2 + 64;
  const int j = lane_id();
  float h = b1[j];
#pragma unroll
  for (int k = 0; k < 6; k++) h = fmaf(W1[j * 6 + k], x[k], h);
  h = h > 0.f ? h : 0.f;
  float y = w2[j] * h;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) y += __shfl_xor(y, d, 64);
  y += b2[0];
  if (!isfinite(y)) return false;
  float e = expf(y);
  e = fminf(fmaxf(e, w.eps_min), w.eps_max);
  *eps_out = e;
  return isfinite(e);
}

// Sizes the next round; called by all lanes of wave 0 with the same values.
__device__ void next_batch(const Ws &w, long long n_rem, long long delta, long long round, float fconf,
                           float fclaim, float feps, long long *b_out, double *eps_out, int *fallback) {
  long long b = 0;
  double eps_used = w.eps;
  bool have = false;
  if (w.policy == POL_TRACE && round < w.sched_len) {
    b = w.sched[round];
    if (b > n_rem) b = n_rem;
    eps_used = delta > 0 ? (double)b * (double)delta / (double)n_rem : 0.0;
    have = true;
  } else if (w.policy == POL_LEARNED) {
    float x[6] = {logf((float)n_rem), logf((float)(delta > 1 ? delta : 1)), fconf, fclaim, feps, (float)round};
    float e = 0.f;
    if (mlp_eps(w, x, &e)) {
      const long long q = (long long)((double)e * 1e6 + 0.5);
      b = fixed_batch(q > 0 ? q : 1, n_rem, delta);
      eps_used = (double)e;
      have = true;
    } else {
      *fallback = 1;
    }
  }
  if (!have) b = fixed_batch(w.eps_q, n_rem, delta);
  *b_out = b;
  *eps_out = eps_used;
}

// ------------------------------------------------------------- select -----
// Tile status word: bits 63..62 = 1 (aggregate) or 2 (inclusive prefix),
// bits 61..0 = value.  Tiles are handed out in order by an atomic counter, so
// a tile only ever waits for tiles that are already being processed.

__device__ inline long long lookback(const Ws &w, unsigned t) {
  long long excl = 0;
  long long j = (long long)t - 1;
  unsigned spins = 0;
  while (j >= 0) {
    const unsigned long long s = ld_acq(&w.tstat[j]);
    const unsigned flag = (unsigned)(s >> 62);
    if (flag == 0) {
      if (++spins > (1u << 24)) {
        set_error(w.ctrl, ERR_NO_PROGRESS);
        return excl;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += (long long)(s & ((1ull << 62) - 1));
    if (flag == 2) break;
    j--;
  }
  return excl;
}

__global__ void __launch_bounds__(BS) k_select(Ws w) {
  Ctrl *c = w.ctrl;
  if (c->done) return;
  __shared__ unsigned s_tile;
  __shared__ int s_stop;
  __shared__ long long s_excl;
  __shared__ int64_t sh[WAVES + 1];
  const long long B = c->b, cur0 = c->cursor;
  const int64_t n = w.n;
  for (;;) {
    if (threadIdx.x == 0) {
      s_stop = ld_acq(&c->select_done);
      if (!s_stop) s_tile = atomicAdd(&c->tile_counter, 1u);
    }
    __syncthreads();
    if (s_stop) break;
    const unsigned t = s_tile;
    if ((int64_t)t >= w.tstat_cap) {  // cannot happen while B <= n_rem
      if (threadIdx.x == 0) set_error(c, ERR_OVERFLOW);
      break;
    }
    const int64_t base = cur0 + (int64_t)t * TSEL + (int64_t)threadIdx.x * SIPT;
    int32_t vv[SIPT];
    unsigned un = 0;
#pragma unroll
    for (int k = 0; k < SIPT; k++) {
      const int64_t p = base + k;
      vv[k] = p < n ? w.order[p] : 0;
    }
#pragma unroll
    for (int k = 0; k < SIPT; k++) {
      const int64_t p = base + k;
      if (p < n && w.state[vv[k]] == UNCL) un |= 1u << k;
    }
    int64_t agg;
    const int64_t mine = wg_excl_scan(__popc(un), &agg, sh);
    if (threadIdx.x == 0) {
      long long excl = 0;
      if (t == 0) {
        st_rel(&w.tstat[0], (2ull << 62) | (unsigned long long)agg);
      } else {
        st_rel(&w.tstat[t], (1ull << 62) | (unsigned long long)agg);
        excl = lookback(w, t);
        st_rel(&w.tstat[t], (2ull << 62) | (unsigned long long)(excl + agg));
      }
      s_excl = excl;
    }
    __syncthreads();
    const long long excl = s_excl;
    // the first (B - excl) unclustered positions of this tile are active
    int64_t wsum = 0;
    int cnt = 0;
    unsigned act = 0;
    long long r = excl + mine;
#pragma unroll
    for (int k = 0; k < SIPT; k++) {
      if (un & (1u << k)) {
        if (r < B) {
          act |= 1u << k;
          cnt++;
          wsum += row_weight(w.off, vv[k]);
          if (r == B - 1) {
            c->r_last = base + k;
            st_rel(&c->select_done, 1);
          }
        }
        r++;
      }
    }
    int64_t wtot, ctot;
    const int64_t wpre = wg_excl_scan(wsum, &wtot, sh);
    const int64_t cpre = wg_excl_scan(cnt, &ctot, sh);
    __shared__ unsigned long long s_base;
    if (threadIdx.x == 0 && ctot > 0) s_base = atomicAdd(&c->a_pack, pk(wtot, ctot));
    __syncthreads();
    if (ctot > 0) {
      int64_t slot = pk_cnt(s_base) + cpre, wpos = pk_work(s_base) + wpre;
#pragma unroll
      for (int k = 0; k < SIPT; k++) {
        if (act & (1u << k)) {
          const int32_t v = vv[k];
          w.state[v] = ACTIVE;
          if (w.algo == ALGO_CW) w.lab[v] = (int32_t)(base + k);  // every active vertex is a center
          w.alist[slot] = v;
          w.awork[slot] = wpos;
          slot++;
          wpos += row_weight(w.off, v);
        }
      }
    }
    if (excl + agg >= B) break;
    __syncthreads();
  }
}

// -------------------------------------------------------------- elect -----

__global__ void __launch_bounds__(BS) k_elect(Ws w) {
  Ctrl *c = w.ctrl;
  if (c->done) return;
  const unsigned long long ap = c->a_pack;
  lb_walk(w.alist, w.awork, pk_cnt(ap), pk_work(ap), w.off, w.col, w.rank, [&](Items &it) {
    uint8_t su[IPT];
#pragma unroll
    for (int k = 0; k < IPT; k++) su[k] = (it.edge >> k & 1) ? w.state[it.u[k]] : (uint8_t)CLUST;
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      bool conf = false;
      if (su[k] == ACTIVE) conf = w.rank[it.u[k]] < it.val[k];  // earlier-ranked active neighbour
      if (conf) w.flag[it.v[k]] = 1;
      const unsigned long long m = __ballot(conf);
      if (m) {
        const int leader = __ffsll((long long)m) - 1;
        unsigned base = 0;
        if (lane_id() == leader) base = atomicAdd(&c->n_cedges, (unsigned)__popcll(m));
        base = __shfl(base, leader, 64);
        if (conf) {
          const int64_t slot = (int64_t)base + __popcll(m & lanemask_lt());
          if (slot < w.cedge_cap) w.cedge[slot] = make_int2(it.v[k], it.u[k]);  // else: rescan rows
        }
      }
    }
  });
}

// Roots (no earlier active neighbour) are centers at once; the last
// workgroup then settles the blocked vertices: a blocked vertex is a
// non-center as soon as an earlier active neighbour is a center, and a center
// once all of them are non-centers.  Each sweep settles at least the
// lowest-ranked undecided vertex, so it ends.
__global__ void __launch_bounds__(BS) k_classify(Ws w) {
  Ctrl *c = w.ctrl;
  if (c->done) return;
  const int64_t na = pk_cnt(c->a_pack);
  for (int64_t i0 = (int64_t)blockIdx.x * BS; i0 < na; i0 += (int64_t)gridDim.x * BS) {
    const int64_t i = i0 + threadIdx.x;
    int32_t a = 0;
    bool blocked = false, root = false;
    if (i < na) {
      a = w.alist[i];
      blocked = w.flag[a] != 0;
      root = !blocked;
    }
    if (root) {
      w.state[a] = CENTER;
      w.lab[a] = w.rank[a];
    }
    wave_append(root, a, root ? row_weight(w.off, a) : 0, &c->c_pack, w.clist, w.cwork);
    const unsigned long long m = __ballot(blocked);
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      unsigned base = 0;
      if (lane_id() == leader) base = atomicAdd(&c->n_blocked, (unsigned)__popcll(m));
      base = __shfl(base, leader, 64);
      if (blocked) w.blist[base + __popcll(m & lanemask_lt())] = a;
    }
  }
  if (!last_block(&c->fin[FIN_CLASSIFY])) return;
  // ---- resolve (one workgroup) ----
  const int64_t nb = ld_acq(&c->n_blocked);
  const int64_t ne_all = ld_acq(&c->n_cedges);
  __shared__ int s_any;
  if (ne_all <= w.cedge_cap) {
    // conflict edges (a, u): u is an earlier-ranked active neighbour of a
    const int64_t ne = ne_all;
    for (int64_t iter = 0; iter <= nb && nb > 0; iter++) {
      for (int64_t i = threadIdx.x; i < ne; i += BS) {
        const int2 e = w.cedge[i];
        if (w.state[e.x] == ACTIVE && w.state[e.y] == CENTER) w.state[e.x] = NONCENTER;
      }
      __syncthreads();
      for (int64_t i = threadIdx.x; i < nb; i += BS) w.flag[w.blist[i]] = 0;
      __syncthreads();
      for (int64_t i = threadIdx.x; i < ne; i += BS) {
        const int2 e = w.cedge[i];
        if (w.state[e.x] == ACTIVE && w.state[e.y] == ACTIVE) w.flag[e.x] = 1;  // still waiting
      }
      __syncthreads();
      if (threadIdx.x == 0) s_any = 0;
      __syncthreads();
      for (int64_t i0 = 0; i0 < nb; i0 += BS) {
        const int64_t i = i0 + threadIdx.x;
        int32_t a = 0;
        bool promote = false, waiting = false;
        if (i < nb) {
          a = w.blist[i];
          if (w.state[a] == ACTIVE) {
            if (w.flag[a] == 0) promote = true;
            else waiting = true;
          }
        }
        if (promote) {
          w.state[a] = CENTER;
          w.lab[a] = w.rank[a];
        }
        if (waiting) s_any = 1;
        wave_append(promote, a, promote ? row_weight(w.off, a) : 0, &c->c_pack, w.clist, w.cwork);
      }
      __syncthreads();
      if (!s_any) break;
    }
  } else {
    // too many conflict edges to list: rescan the rows of the blocked vertices
    // (every earlier-ranked unclustered neighbour of an active vertex is active)
    for (int64_t iter = 0; iter <= nb && nb > 0; iter++) {
      if (threadIdx.x == 0) s_any = 0;
      __syncthreads();
      for (int64_t i0 = 0; i0 < nb; i0 += BS) {
        const int64_t i = i0 + threadIdx.x;
        int32_t a = 0;
        bool promote = false;
        if (i < nb) {
          a = w.blist[i];
          if (w.state[a] == ACTIVE) {
            const int32_t ra = w.rank[a];
            bool center_before = false, undecided_before = false;
            for (int64_t e = w.off[a]; e < w.off[a + 1] && !center_before; e++) {
              const int32_t u = w.col[e];
              const uint8_t su = w.state[u];
              if (su == CENTER || su == ACTIVE) {
                if (w.rank[u] < ra) {
                  if (su == CENTER) center_before = true;
                  else undecided_before = true;
                }
              }
            }
            if (center_before) w.state[a] = NONCENTER;
            else if (!undecided_before) promote = true;
            else s_any = 1;
          }
        }
        if (promote) {
          w.state[a] = CENTER;
          w.lab[a] = w.rank[a];
        }
        wave_append(promote, a, promote ? row_weight(w.off, a) : 0, &c->c_pack, w.clist, w.cwork);
      }
      __syncthreads();
      if (!s_any) break;
    }
  }
  for (int64_t i = threadIdx.x; i < nb; i += BS) w.flag[w.blist[i]] = 0;
  if (threadIdx.x == 0) c->fin[FIN_CLASSIFY] = 0;
}

// -------------------------------------------------------------- claim -----

__global__ void __launch_bounds__(BS) k_claim(Ws w) {
  Ctrl *c = w.ctrl;
  if (c->done) return;
  const bool c4 = w.algo == ALGO_C4;
  const unsigned long long lp = c4 ? c->c_pack : c->a_pack;
  const int32_t *list = c4 ? w.clist : w.alist;
  const int64_t *work = c4 ? w.cwork : w.awork;
  __shared__ unsigned s_atom;
  if (threadIdx.x == 0) s_atom = 0;
  __syncthreads();
  lb_walk(list, work, pk_cnt(lp), pk_work(lp), w.off, w.col, w.rank, [&](Items &it) {
    // every center is clustered this round
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      const bool vt = it.vert >> k & 1;
      wave_append(vt, it.v[k], it.deg[k] > 0 ? it.deg[k] : 1, &c->n_pack, w.nlist, w.nwork);
    }
    uint8_t su[IPT];
#pragma unroll
    for (int k = 0; k < IPT; k++) su[k] = (it.edge >> k & 1) ? w.state[it.u[k]] : (uint8_t)CLUST;
    int32_t cur[IPT];
    bool elig[IPT];
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      elig[k] = c4 ? (su[k] == UNCL || su[k] == NONCENTER) : (su[k] == UNCL);
      if (!c4 && su[k] == ACTIVE && w.rank[it.u[k]] < it.val[k]) w.flag[it.v[k]] = 1;  // rule 1 broken
      cur[k] = elig[k] ? w.lab[it.u[k]] : 0;  // stale reads are safe: labels only decrease
    }
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      bool first = false;
      int64_t wt = 0;
      if (elig[k] && it.val[k] < cur[k]) {
        const int32_t old = atomicMin(&w.lab[it.u[k]], it.val[k]);
        atomicAdd(&s_atom, 1u);
        first = (old == INF);
        if (first) wt = row_weight(w.off, it.u[k]);
      }
      wave_append(first, it.u[k], wt, &c->n_pack, w.nlist, w.nwork);
    }
  });
  __syncthreads();
  if (threadIdx.x == 0 && s_atom) atomicAdd(&c->sum_atomics, (unsigned long long)s_atom);
}

// --------------------------------------------------------------- peel -----

__global__ void __launch_bounds__(BS) k_peel(Ws w) {
  Ctrl *c = w.ctrl;
  if (c->done) return;
  const unsigned long long np = c->n_pack;
  const bool cw = w.algo == ALGO_CW;
  __shared__ unsigned s_conf, s_atom;
  if (threadIdx.x == 0) s_conf = s_atom = 0;
  __syncthreads();
  lb_walk(w.nlist, w.nwork, pk_cnt(np), pk_work(np), w.off, w.col, nullptr, [&](Items &it) {
    unsigned conf = 0;
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      if (it.vert >> k & 1) {
        w.state[it.v[k]] = CLUST;
        if (cw && w.flag[it.v[k]]) {
          w.flag[it.v[k]] = 0;
          conf++;
        }
      }
    }
    if (cw && conf) atomicAdd(&s_conf, conf);
    int32_t lw[IPT];
#pragma unroll
    for (int k = 0; k < IPT; k++) lw[k] = (it.edge >> k & 1) ? w.lab[it.u[k]] : 0;
    unsigned dec = 0;
#pragma unroll
    for (int k = 0; k < IPT; k++)
      if (lw[k] == INF) {  // still unclustered after this round
        atomicSub(&w.resdeg[it.u[k]], 1);
        dec++;
      }
    if (dec) atomicAdd(&s_atom, dec);
  });
  __syncthreads();
  if (cw && threadIdx.x == 0 && s_conf) atomicAdd(&c->conflicts, (unsigned long long)s_conf);
  if (threadIdx.x == 0 && s_atom) atomicAdd(&c->sum_atomics, (unsigned long long)s_atom);
}

// -------------------------------------------------------------- delta -----

__global__ void __launch_bounds__(BS) k_delta(Ws w) {
  Ctrl *c = w.ctrl;
  if (c->done) return;
  const int64_t n = w.n;
  // forget this round's scan tiles
  const int64_t tiles = (int64_t)c->tile_counter + 1;
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < tiles && t < w.tstat_cap;
       t += (int64_t)gridDim.x * BS)
    w.tstat[t] = 0;
  int mx = 0;
  for (int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x; v < n; v += (int64_t)gridDim.x * BS)
    if (w.state[v] == UNCL) mx = max(mx, w.resdeg[v]);
  mx = wave_max(mx);
  __shared__ int s_mx[WAVES];
  if (lane_id() == 0) s_mx[wave_id()] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = 0;
    for (int i = 0; i < WAVES; i++) m = max(m, s_mx[i]);
    if (m > 0) atomicMax(&c->delta_next, m);
  }
  if (!last_block(&c->fin[FIN_DELTA])) return;
  if (threadIdx.x >= 64) return;
  // ---- close the round (wave 0 of the last workgroup; lane 0 updates the
  // control block, the other lanes get its values by shuffle) ----
  const long long now = (long long)wall_clock64();
  long long n_rem = 0, delta = 0, round = 0;
  int done = 0;
  float fconf = 0.f, fclaim = 0.f, feps = 0.f;
  if (threadIdx.x == 0) {
    if (c->has_round) {
      const bool c4 = w.algo == ALGO_C4;
      const long long centers = c4 ? pk_cnt(c->c_pack) : pk_cnt(c->a_pack);
      const long long newly = pk_cnt(c->n_pack);
      const long long conf = c4 ? (long long)c->n_blocked : (long long)c->conflicts;
      if (c->round < w.trace_cap) {
        RoundRec r;
        r.n_i = c->n_start;
        r.delta_i = c->delta;
        r.b_i = c->b;
        r.r_i = c->r_last;
        r.centers = centers;
        r.claimed = newly - centers;
        r.conflicts = conf;
        r.eps_used = c->eps_used;
        r.t_ns = now - c->t_start;
        w.trace[c->round] = r;
      }
      c->sum_elect += c4 ? (unsigned long long)pk_work(c->a_pack) : 0ull;
      c->sum_claim += c4 ? (unsigned long long)pk_work(c->c_pack) : (unsigned long long)pk_work(c->a_pack);
      c->sum_peel += (unsigned long long)pk_work(c->n_pack);
      c->sum_blocked += (unsigned long long)conf;
      c->feat_conf = c->b > 0 ? (float)conf / (float)c->b : 0.f;
      c->feat_claim = c->n_start > 0 ? (float)(newly - centers) / (float)c->n_start : 0.f;
      c->feat_eps = (float)c->eps_used;
      c->cursor = c->r_last + 1;
      c->n_rem = c->n_start - newly;
      c->round += 1;
      if (c->round > w.n + 1) set_error(c, ERR_NO_PROGRESS);
    }
    c->delta = c->delta_next;
    c->delta_next = 0;
    c->has_round = 1;
    c->a_pack = c->c_pack = c->n_pack = 0;
    c->tile_counter = 0;
    c->select_done = 0;
    c->n_blocked = 0;
    c->n_cedges = 0;
    c->conflicts = 0;
    if (c->n_rem <= 0 || c->error) c->done = 1;
    n_rem = c->n_rem;
    delta = c->delta;
    round = c->round;
    done = c->done;
    fconf = c->feat_conf;
    fclaim = c->feat_claim;
    feps = c->feat_eps;
  }
  n_rem = __shfl(n_rem, 0, 64);
  delta = __shfl(delta, 0, 64);
  round = __shfl(round, 0, 64);
  done = __shfl(done, 0, 64);
  fconf = __shfl(fconf, 0, 64);
  fclaim = __shfl(fclaim, 0, 64);
  feps = __shfl(feps, 0, 64);
  if (!done) {
    long long b = 0;
    double eps_used = 0.0;
    int fb = 0;
    next_batch(w, n_rem, delta, round, fconf, fclaim, feps, &b, &eps_used, &fb);
    if (threadIdx.x == 0) {
      c->b = b;
      c->eps_used = eps_used;
      if (fb) c->fallback = 1;
      c->n_start = n_rem;
      c->t_start = now;
    }
  }
  if (threadIdx.x == 0) c->fin[FIN_DELTA] = 0;
}

// ----------------------------------------------------------- finalize -----

__global__ void __launch_bounds__(BS) k_finalize(Ws w, int32_t *labels) {
  const int64_t n = w.n;
  for (int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x; v < n; v += (int64_t)gridDim.x * BS) {
    const int32_t l = w.lab[v];
    if (l < 0 || (int64_t)l >= n) {
      set_error(w.ctrl, ERR_LABEL);
      labels[v] = -1;
    } else {
      labels[v] = w.order[l];
    }
  }
}

// -------------------------------------------------------------- launch ----

static inline unsigned grid_for(int64_t items, unsigned cap) {
  int64_t g = (items + BS - 1) / BS;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_init(const Ws &w, hipStream_t s) {
  hipLaunchKernelGGL(k_invert, dim3(grid_for(w.n, 4096)), dim3(BS), 0, s, w);
  hipLaunchKernelGGL(k_init, dim3(grid_for(w.n, 4096)), dim3(BS), 0, s, w);
  hipLaunchKernelGGL(k_delta, dim3(grid_for(w.n, 2048)), dim3(BS), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_round(const Ws &w, hipStream_t s, const LaunchShape &ls) {
  hipLaunchKernelGGL(k_select, dim3(ls.select_grid), dim3(BS), 0, s, w);
  if (w.algo == ALGO_C4) {
    hipLaunchKernelGGL(k_elect, dim3(ls.edge_grid), dim3(BS), 0, s, w);
    hipLaunchKernelGGL(k_classify, dim3(ls.vertex_grid), dim3(BS), 0, s, w);
  }
  hipLaunchKernelGGL(k_claim, dim3(ls.edge_grid), dim3(BS), 0, s, w);
  hipLaunchKernelGGL(k_peel, dim3(ls.edge_grid), dim3(BS), 0, s, w);
  hipLaunchKernelGGL(k_delta, dim3(grid_for(w.n, ls.scan_grid)), dim3(BS), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_finalize(const Ws &w, int32_t *labels, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(grid_for(w.n, 4096)), dim3(BS), 0, s, w, labels);
  return hipGetLastError();
}

}  // namespace ccd
