// cc_rounds.hip -- the bulk-synchronous round loop of C4 and ClusterWild!
// (arXiv 1507.05086, Algorithm 2) as a fixed sequence of gfx950 kernels per
// round.  Kernel boundaries are the round's barriers (cheaper on this GPU than
// a software grid barrier); every kernel returns at once when its part of the
// round has nothing to do, so the host can queue rounds in groups and look at
// the done flag once per group.
//
//   select    next B_i unclustered vertices of pi (lazy deletion: a cursor
//             walks pi once); one pass with decoupled look-back
//   elect     C4: does an active vertex have an earlier-ranked active
//             neighbour?  (concurrency rule 1; edge-balanced)
//   classify  C4: roots become centers, the others are blocked
//   resolve   C4: one workgroup settles the blocked vertices as a fixed point
//             over the conflict edges (the greedy MIS of G[A] in pi order)
//   claim     every center claims its unclustered neighbours with atomicMin on
//             the center rank (concurrency rule 2, createCluster)
//   clear     the newly clustered leave the unclustered bitmap
//   peel      exact phase only: neighbours of the newly clustered lose one
//             remaining degree each (degree histogram kept per workgroup)
//   dscan / rescan (x3)   lazy phase: the next Delta from stale upper bounds,
//             rescanning only candidates in a band below the current Delta
//   xlist / xcount        switch to exact degrees when the band gets low
//   close     one workgroup: round record, Delta_{i+1}, B_{i+1}, counters
//
// The paper deletes lazily (clustered vertices are skipped, the graph is never
// changed); here that extends to the remaining degrees: while Delta is large
// they are upper bounds refreshed only where the maximum could be, and the
// edge-by-edge peeling starts only when little of the graph is left.
#include "cc_device.h"
#include "cc_launch.h"
#include "cc_walk.h"

namespace ccd {

// Per-row partial counts of rows split across tiles: one 64-bit atomic adds
// (items covered << 32 | count); the contributor that completes the row
// (covered == degree) owns the total.
__device__ inline bool row_combine(unsigned long long *acc, int64_t slot, int cnt, int64_t covered, int32_t deg,
                                   int *total) {
  const unsigned long long add = ((unsigned long long)covered << 32) | (unsigned)cnt;
  const unsigned long long tot = atomicAdd(&acc[slot], add) + add;
  if ((int64_t)(tot >> 32) != (int64_t)deg) return false;
  *total = (int)(tot & 0xFFFFFFFFu);
  return true;
}

// ------------------------------------------------------------------ init --

// pi moves to internal ids (one gather, written in pi order) and must be a
// permutation: n entries, each in range and none repeated.  Each entry marks
// its vertex in the (zeroed) state bytes with a plain store; n entries in
// range mark all n vertices exactly when none repeats, which k_init checks.
// pi is not inverted: the rank of a vertex is recorded when it becomes
// active, the only time anyone asks for it.
__global__ void __launch_bounds__(BS) k_check_order(Ws w) {
  const int64_t n = w.n;
  for (int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x; k < n; k += (int64_t)gridDim.x * BS) {
    const int32_t v = w.order_in[k];
    if (v < 0 || (int64_t)v >= n) {
      set_error(w.ctrl, ERR_PERM);
      w.iorder[k] = 0;
    } else {
      const int32_t vi = w.perm[v];
      w.iorder[k] = vi;
      w.state[vi] = ORDER_SEEN;
    }
  }
}

// An isolated vertex (id >= iso_start) has no neighbour to read its state,
// flag or bound, and k_select settles it by its id alone, so only a partial
// run (whose k_finalize reads its label) and the direct check of pi (which
// reads its mark) visit those ids.
__global__ void __launch_bounds__(BS) k_init(Ws w, const unsigned *lvl_init_cnt) {
  const int64_t n = w.n;
  const int64_t end = (w.order_mapped && w.max_rounds == 0) ? w.iso_start : n;
  for (int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x; v < end; v += (int64_t)gridDim.x * BS) {
    if (!w.order_mapped && w.state[v] != ORDER_SEEN) set_error(w.ctrl, ERR_PERM);  // no entry of pi names v
    w.lab[v] = INF;
    if (v >= w.iso_start) continue;
    w.state[v] = UNCL;
    w.flag[v] = 0;
    w.ub[v] = (int32_t)(w.off[v + 1] - w.off[v]);
  }
  const int64_t nw = (n + 31) / 32;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < nw; i += (int64_t)gridDim.x * BS) {
    const int64_t rem = n - i * 32;
    w.unc[i] = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
  }
  Ctrl *c = w.ctrl;
  if (blockIdx.x == 0) {
    if (threadIdx.x < NLVL) c->lvl_cnt[threadIdx.x] = lvl_init_cnt[threadIdx.x];
    if (threadIdx.x == 0) {
      c->n_rem = n;
      c->n_start = n;
      c->done = (n == 0);
      c->phase = PHASE_LAZY;
      c->feat_eps = (float)w.eps;
    }
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

// Delta-hat of round i under the practical schedule: Delta_0 halved every
// bin_period rounds (rounded down, as the trace records it).
__device__ inline long long delta_hat(const Ws &w, long long round) {
  const long long h = round / w.bin_period;
  return h >= 63 ? 0 : (long long)w.max_deg >> h;
}

// Sizes the next round; called by all lanes of wave 0 with the same values.
__device__ void next_batch(const Ws &w, long long n_rem, long long delta, long long round, float fconf,
                           float fclaim, float feps, long long *b_out, double *eps_out, int *fallback) {
  long long b = 0;
  double eps_used = w.eps;
  bool have = false;
  if (w.policy == POL_BINOMIAL) {  // round < sched_len: checked by the caller
    b = w.sched[round];
    eps_used = w.eps;
    have = true;
  } else if (w.policy == POL_TRACE && round < w.sched_len) {
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

// ------------------------------------------------- lazy Delta search -----
// Pass j rescans every candidate whose bound is >= L_j = ceil(f_j * T_j)
// (T_0 = Delta_i; f = 0.7, 0.3, 0.05).  Every other vertex has a bound below
// L_j, so if the largest exact degree found is >= L_j it is Delta_{i+1};
// otherwise T_{j+1} = L_j - 1.  When a band floor would fall below SWL, or all
// passes fail, the run switches to exact remaining degrees.

struct DSearch {
  int pending;      // 1 while the search still needs the next pass
  int switching;    // 1 when the run moves to exact degrees
  long long delta;  // resolved Delta (when neither pending nor switching)
  long long T, L;   // bounds of the pending pass
};

__device__ inline long long band_floor(int pass, long long T) {
  return (long long)ceilf(band_factor(pass) * (float)T);
}

// State of the search after `done` passes (every thread computes the same);
// C is Ctrl or a CtrlHead snapshot of it.
template <class C>
__device__ inline DSearch dsearch(const C *c, int done) {
  DSearch s{0, 0, -1, 0, 0};
  if (c->phase != PHASE_LAZY) return s;
  long long T = c->delta;
  for (int j = 0; j < done; j++) {
    const long long L = band_floor(j, T);
    if (L < SWL) {  // pass j never ran: the search switched before it
      s.switching = 1;
      return s;
    }
    const long long M = c->d_max[j];
    if (M >= L) {
      s.delta = M;
      return s;
    }
    T = L - 1;
  }
  if (done >= DITER || band_floor(done, T) < SWL) {
    s.switching = 1;
    return s;
  }
  s.pending = 1;
  s.T = T;
  s.L = band_floor(done, T);
  return s;
}

// Candidates of pass IT: live entries with bound >= L, found in the levels
// level(L) .. top (a bound can be stale above the current Delta).
template <int IT>
__global__ void __launch_bounds__(BS) k_dscan(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done) return;
  const DSearch s = dsearch(&h, IT);
  if (!s.pending) return;
  const int kL = level_of(s.L < DSW ? DSW : s.L), kT = NLVL - 1;
  int64_t base[NLVL + 1];
  int64_t tot = 0;
  for (int k = kL; k <= kT; k++) {
    base[k] = tot;
    const int64_t cap = w.lvl_off[k + 1] - w.lvl_off[k];
    const int64_t cnt = c->lvl_cnt[k];
    tot += cnt < cap ? cnt : cap;
  }
  base[kT + 1] = tot;
  __shared__ StageBuf<2 * BS> sb;
  stage_init(sb);
  // a contiguous share of the entries per workgroup
  const int64_t per = ((tot + gridDim.x - 1) / gridDim.x + BS - 1) / BS * BS;
  const int64_t e0 = (int64_t)blockIdx.x * per, e1 = e0 + per < tot ? e0 + per : tot;
  for (int64_t i0 = e0; i0 < e1; i0 += BS) {
    const int64_t i = i0 + threadIdx.x;
    if (i < e1) {
      int k = kL;
      while (k < kT && i >= base[k + 1]) k++;
      const int32_t v = w.lvl[w.lvl_off[k] + (i - base[k])];
      const int32_t x = w.ub[v];
      if (x >= s.L && level_of(x) == k && unc_bit(w.unc, v))  // live entry, inside the band
        stage_push(sb, v, (int32_t)(w.rend[v] - w.off[v]));
    }
    __syncthreads();
    if (sb.cnt > BS) stage_flush(sb, &c->r_pack[IT], w.rlist + IT * w.rcap, w.rwork + IT * w.rcap, w.racc + IT * w.rcap);
  }
  stage_flush(sb, &c->r_pack[IT], w.rlist + IT * w.rcap, w.rwork + IT * w.rcap, w.racc + IT * w.rcap);
}

// Exact remaining degrees of the pass's candidates; the new bounds move
// entries down the levels; the pass maximum goes to d_max.
template <int IT>
__global__ void __launch_bounds__(BS) k_rescan(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done) return;
  const DSearch s = dsearch(&h, IT);
  if (!s.pending) return;
  __shared__ int lcnt[TW];
  __shared__ int s_max, s_nmv;
  __shared__ int s_mvn[NLVL], s_mvbase[NLVL];
  __shared__ int32_t s_mv[TW];
  __shared__ int8_t s_mvk[TW];
  for (int i = threadIdx.x; i < TW; i += BS) lcnt[i] = 0;
  if (threadIdx.x < NLVL) s_mvn[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    s_max = 0;
    s_nmv = 0;
  }
  __syncthreads();
  const unsigned long long rp = h.r_pack[IT];
  const int64_t cnt = pk_cnt(rp) < w.rcap ? pk_cnt(rp) : w.rcap;
  unsigned long long *ra = w.racc + IT * w.rcap;
  auto finalize = [&](int32_t v, int r) {
    const int32_t old = w.ub[v];
    w.ub[v] = r;
    atomicMax(&s_max, r);
    const int kn = r >= DSW ? level_of(r) : -1;
    if (kn >= 0 && kn != level_of(old)) {
      const int p = atomicAdd(&s_nmv, 1);
      s_mv[p] = v;
      s_mvk[p] = (int8_t)kn;
      atomicAdd(&s_mvn[kn], 1);
    }
  };
  lb_walk(
      w.rlist + IT * w.rcap, w.rwork + IT * w.rcap, cnt, pk_work(rp), w.off, w.rend, w.col, nullptr, nullptr,
      [&](Items &it) {
#pragma unroll
        for (int k = 0; k < IPT; k++)
          if ((it.edge >> k & 1) && unc_bit(w.unc, it.u[k])) atomicAdd(&lcnt[it.ent[k]], 1);
      },
      [&](int j, int64_t slot, int32_t v, int32_t deg, int64_t covered) {
        const int cj = lcnt[j];
        lcnt[j] = 0;
        int total = cj;
        if (covered == deg || row_combine(ra, slot, cj, covered, deg, &total)) finalize(v, total);
      },
      [&]() {
        // this tile's level moves: one reservation per level, then the writes
        __syncthreads();
        if (threadIdx.x < NLVL && s_mvn[threadIdx.x]) {
          const int k = threadIdx.x;
          s_mvbase[k] = (int)atomicAdd(&c->lvl_cnt[k], (unsigned)s_mvn[k]);
        }
        __syncthreads();
        const int nmv = s_nmv;
        for (int p = threadIdx.x; p < nmv; p += BS) {
          const int k = s_mvk[p];
          int q = 0;  // rank among this tile's earlier moves to the same level
          for (int x = 0; x < p; x++) q += (s_mvk[x] == k);
          const int64_t pos = (int64_t)s_mvbase[k] + q;
          if (pos < w.lvl_off[k + 1] - w.lvl_off[k]) w.lvl[w.lvl_off[k] + pos] = s_mv[p];
          else set_error(c, ERR_OVERFLOW);
        }
        __syncthreads();
        if (threadIdx.x < NLVL) s_mvn[threadIdx.x] = 0;
        if (threadIdx.x == 0) s_nmv = 0;
      });
  __syncthreads();
  if (threadIdx.x == 0 && s_max > 0) atomicMax(&c->d_max[IT], s_max);
}

// Switch to exact degrees: list the unclustered rows of degree >= DSW (their
// accumulators live in the active-list weights, free at this point of the
// round) ...
__global__ void __launch_bounds__(BS) k_xlist(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done) return;
  const DSearch s = dsearch(&h, DITER);
  if (!s.switching) return;
  unsigned long long *xacc = (unsigned long long *)w.awork;
  __shared__ StageBuf<2 * BS> sb;
  stage_init(sb);
  const int64_t n = w.low_start;  // lower-degree rows are counted by id in k_xcount
  const int64_t per = ((n + gridDim.x - 1) / gridDim.x + BS - 1) / BS * BS;
  const int64_t v0 = (int64_t)blockIdx.x * per, v1 = v0 + per < n ? v0 + per : n;
  for (int64_t vb = v0; vb < v1; vb += BS) {
    const int64_t v = vb + threadIdx.x;
    if (v < v1 && unc_bit(w.unc, (int32_t)v)) {
      const int64_t d = w.off[v + 1] - w.off[v];
      w.xend[v] = w.off[v];  // k_xcount appends the row's unclustered neighbours
      if (d > 0) stage_push(sb, (int32_t)v, (int32_t)d);
    }
    __syncthreads();
    if (sb.cnt > BS) stage_flush(sb, &c->x_pack, w.xlist, w.xwork, xacc);
  }
  stage_flush(sb, &c->x_pack, w.xlist, w.xwork, xacc);
}

// ... and count their unclustered neighbours into ub and the histogram: the
// listed rows edge-balanced, the rows of degree below DSW (ids low_start ..
// iso_start, by falling level) one lane per row, so a wave's rows are of
// about one length and no search or barrier is needed.  The unclustered
// neighbours found are also written to the compacted rows (xcol, from the
// start of each row's slot; xend = where the row ends): every vertex the
// exact rounds walk is unclustered now, and its neighbours clustered before
// now can never count again.  A listed row's tiles reserve their shares of
// the slot with one atomic each, so its entries are in no particular order.
__global__ void __launch_bounds__(BS) k_xcount(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done) return;
  const DSearch s = dsearch(&h, DITER);
  if (!s.switching) return;
  __shared__ int lcnt[TW];
  __shared__ int64_t lbase[TW];  // where this tile's share of its row j goes in xcol
  __shared__ int s_hist[HLDS];
  for (int i = threadIdx.x; i < TW; i += BS) lcnt[i] = 0;
  for (int i = threadIdx.x; i < HLDS; i += BS) s_hist[i] = 0;
  __syncthreads();
  unsigned long long *xacc = (unsigned long long *)w.awork;
  const unsigned long long xp = h.x_pack;
  auto finalize = [&](int32_t v, int r) {
    w.ub[v] = r;
    if (r > 0 && r < HLDS) atomicAdd(&s_hist[r], 1);
    else if (r >= HLDS) atomicAdd(&w.hist[r], 1);
  };
  // this thread's unclustered neighbours in the current tile: the neighbour,
  // its row's slot in the tile, and its index in the tile's share of the row
  int32_t pu[IPT];
  int pj[IPT], pl[IPT];
  unsigned pending = 0;
  lb_walk(
      w.xlist, w.xwork, pk_cnt(xp), pk_work(xp), w.off, w.off + 1, w.col, nullptr, nullptr,
      [&](Items &it) {
        pending = 0;
#pragma unroll
        for (int k = 0; k < IPT; k++)
          if ((it.edge >> k & 1) && unc_bit(w.unc, it.u[k])) {
            pu[k] = it.u[k];
            pj[k] = it.ent[k];
            pl[k] = atomicAdd(&lcnt[it.ent[k]], 1);
            pending |= 1u << k;
          }
      },
      [&](int j, int64_t slot, int32_t v, int32_t deg, int64_t covered) {
        const int cj = lcnt[j];
        lcnt[j] = 0;
        lbase[j] = cj > 0 ? (int64_t)atomicAdd((unsigned long long *)&w.xend[v], (unsigned long long)cj) : 0;
        int total = cj;
        if (covered == deg || row_combine(xacc, slot, cj, covered, deg, &total)) finalize(v, total);
      },
      [&]() {
        __syncthreads();  // every row of the tile has its share reserved
#pragma unroll
        for (int k = 0; k < IPT; k++)
          if (pending >> k & 1) w.xcol[lbase[pj[k]] + pl[k]] = pu[k];
      });
  static_assert(DSW <= HLDS, "a lower-degree row's count fits the LDS histogram");
  int64_t scanned = 0;
  for (int64_t v = w.low_start + (int64_t)blockIdx.x * BS + threadIdx.x; v < w.iso_start;
       v += (int64_t)gridDim.x * BS) {
    if (!unc_bit(w.unc, (int32_t)v)) continue;
    const int64_t s0 = w.off[v];
    const int d = (int)(w.off[v + 1] - s0);
    int r = 0;
    for (int j = 0; j < d; j += 4) {
      int32_t u[4];
#pragma unroll
      for (int q = 0; q < 4; q++) u[q] = j + q < d ? w.col[s0 + j + q] : -1;
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (u[q] >= 0 && unc_bit(w.unc, u[q])) w.xcol[s0 + r++] = u[q];
    }
    scanned += d;
    w.ub[v] = r;
    w.xend[v] = s0 + r;
    if (r > 0) atomicAdd(&s_hist[r], 1);
  }
  const int64_t wsc = wave_sum(scanned);
  if (lane_id() == 0 && wsc) atomicAdd(&c->x_low[(blockIdx.x * (BS / 64) + wave_id()) & 63], (unsigned long long)wsc);
  __syncthreads();
  for (int i = threadIdx.x; i < HLDS; i += BS)
    if (s_hist[i]) atomicAdd(&w.hist[i], s_hist[i]);
}

// ------------------------------------------------------------- select -----
// Tile status word: bits 63..62 = 1 (aggregate) or 2 (inclusive prefix),
// bits 61..0 = value.  Tiles are handed out in order by an atomic counter, so
// a tile only ever waits for tiles that are already being processed.  The
// word carries its value with its flag, so it is read and written with
// relaxed device-scope atomics: nothing else needs ordering against it.  (A
// release or acquire at device scope would write back or invalidate the
// whole L2 of the XCD each time; the select_done flag is relaxed for the
// same reason, and r_last, written before it, is read after the kernel.)

// Decoupled look-back by one wave: lane l reads the status of tile j - l, so
// each step covers 64 predecessors; the walk stops at the nearest inclusive
// prefix.  Called by all 64 lanes of a wave; returns the exclusive prefix.
__device__ inline long long lookback(const Ws &w, unsigned t) {
  long long excl = 0;
  long long j = (long long)t - 1;
  unsigned spins = 0;
  const int l = lane_id();
  while (j >= 0) {
    const long long idx = j - l;
    const unsigned long long s = idx >= 0 ? ld_rlx(&w.tstat[idx]) : (2ull << 62);
    const unsigned flag = (unsigned)(s >> 62);
    const unsigned long long incl = __ballot(flag == 2);
    const unsigned long long notready = __ballot(flag == 0);
    const int first = incl ? __ffsll((long long)incl) - 1 : 64;  // nearest inclusive prefix
    const unsigned long long need = first < 63 ? ((2ull << first) - 1) : ~0ull;
    if (notready & need) {  // a nearer predecessor has not published yet
      if (++spins > (1u << 22)) {
        if (l == 0) set_error(w.ctrl, ERR_NO_PROGRESS);
        return excl;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    const long long val = (l <= first) ? (long long)(s & ((1ull << 62) - 1)) : 0;
    excl += wave_sum(val);
    if (first < 64) break;
    j -= 64;
  }
  return excl;
}

// The rows a round walks: the full rows until the run switches to exact
// degrees, the rows the switch compacted after it (the phase is read at the
// start of each kernel and changes only at the end of a round, in k_close).
__device__ inline const int64_t *round_end(const Ws &w, int phase) { return phase == PHASE_EXACT ? w.xend : w.rend; }
__device__ inline const int32_t *round_col(const Ws &w, int phase) { return phase == PHASE_EXACT ? w.xcol : w.col; }

// The positions of this thread's slots marked in `act` hold this round's
// active vertices (vv[k] at position base + k).  An active vertex with no
// unclustered neighbour (degree 0, or an exact remaining degree of 0) is a
// center that claims nobody and that no other active vertex can see: it is
// settled here and never listed.  Its label stays unset; k_finalize makes it
// its own center (an isolated vertex once the run is complete -- a partial
// run labels the isolated vertices it reaches -- or a vertex with its bit
// cleared and no label).  The others go to the active list with their row
// info.  Collective: every thread of the workgroup calls it.
__device__ inline void activate(const Ws &w, Ctrl *c, const int32_t vv[SIPT], unsigned act, int64_t base, bool exact,
                                const int64_t *rend,
                                int64_t *sh, unsigned long long *s_base) {
  int64_t wsum = 0;
  int cnt = 0, lone = 0;
  unsigned clears = 0;
  unsigned listed = 0;
  int32_t wt[SIPT];
  int64_t rs[SIPT];
#pragma unroll
  for (int k = 0; k < SIPT; k++) {
    wt[k] = 0;
    rs[k] = 0;
    if (act & (1u << k)) {
      const int32_t v = vv[k];
      if (v >= w.iso_start) {
        if (w.max_rounds > 0) w.lab[v] = (int32_t)(base + k);  // a partial run must tell it apart
        lone++;
      } else if (exact && w.ub[v] == 0) {
        atomicAnd(&w.unc[v >> 5], ~(1u << (v & 31)));
        lone++;
        clears++;
      } else {
        rs[k] = w.off[v];
        wt[k] = (int32_t)(rend[v] - rs[k]);
        listed |= 1u << k;
        cnt++;
        wsum += wt[k];
      }
    }
  }
  int64_t wtot, ctot;
  const int64_t wpre = wg_excl_scan<SEL_BS>(wsum, &wtot, sh);
  // listed count in the low 32 bits, settled count above (a tile holds < 2^32)
  const int64_t cpre = wg_excl_scan<SEL_BS>((int64_t)cnt | ((int64_t)lone << 32), &ctot, sh) & 0xFFFFFFFFll;
  const int64_t ltot = ctot >> 32;
  ctot &= 0xFFFFFFFFll;
  if (threadIdx.x == 0 && ctot > 0) *s_base = atomicAdd(&c->a_pack, pk(wtot, ctot));
  if (threadIdx.x == 0 && ltot > 0) atomicAdd(&c->spread_lone[blockIdx.x & 63], (unsigned long long)ltot);
  const int64_t wc = wave_sum((int64_t)clears);  // every lane takes part in the sum
  if (lane_id() == 0 && wc) atomicAdd(&c->spread_atom[blockIdx.x & 63], (unsigned long long)wc);
  __syncthreads();
  if (ctot > 0) {
    int64_t slot = pk_cnt(*s_base) + cpre, wpos = pk_work(*s_base) + wpre;
#pragma unroll
    for (int k = 0; k < SIPT; k++) {
      if (listed & (1u << k)) {
        const int32_t v = vv[k];
        w.state[v] = ACTIVE;
        // the rank of an active vertex, as its neighbours will ask for it:
        // ClusterWild! keeps it as the label (every active vertex is a center)
        if (w.algo == ALGO_CW) w.lab[v] = (int32_t)(base + k);
        else w.rank[v] = (int32_t)(base + k);
        w.alist[slot] = v;
        w.awork[slot] = wpos;
        w.ainfo[slot] = RowInfo{rs[k], wt[k], (int32_t)(base + k)};
        slot++;
        wpos += wt[k];
      }
    }
  }
}

// An unclustered-or-isolated mask of this thread's slots from base on (an
// isolated vertex's bit is never cleared: only its own position, which the
// cursor passes once, asks whether it is clustered).
__device__ inline unsigned load_slots(const Ws &w, int64_t base, int64_t end, int32_t vv[SIPT]) {
  unsigned un = 0;
#pragma unroll
  for (int k = 0; k < SIPT; k++) {
    const int64_t p = base + k;
    vv[k] = p < end ? w.order[p] : 0;
  }
#pragma unroll
  for (int k = 0; k < SIPT; k++) {
    const int64_t p = base + k;
    if (p < end && (vv[k] >= w.iso_start || unc_bit(w.unc, vv[k]))) un |= 1u << k;
  }
  return un;
}

// The next B_i unclustered vertices of pi (Algorithm 2's active set).
__global__ void __launch_bounds__(SEL_BS) k_select(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done) return;
  __shared__ unsigned s_tile;
  __shared__ int s_stop;
  __shared__ long long s_excl;
  __shared__ int64_t sh[SEL_BS / 64 + 1];
  __shared__ unsigned long long s_base;
  const long long B = h.b, cur0 = h.cursor;
  const bool exact = h.phase == PHASE_EXACT;
  const int64_t n = w.n;
  // Workgroups this round can use: B_i unclustered are spread over the
  // positions ahead with density n_i / (n - cursor); extra groups would only
  // grab tiles past the end of the active set.
  const long long ahead = n - cur0, n_i = h.n_rem > 0 ? h.n_rem : 1;
  const long long need_pos = (long long)((double)B * (double)ahead / (double)n_i) + TSEL;
  if ((long long)blockIdx.x > need_pos / TSEL) return;
  for (;;) {
    if (threadIdx.x == 0) {
      s_stop = ld_rlx(&c->select_done);
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
    const unsigned un = load_slots(w, base, n, vv);
    int64_t agg;
    const int64_t mine = wg_excl_scan<SEL_BS>(__popc(un), &agg, sh);
    if (threadIdx.x < 64) {  // wave 0 publishes and looks back
      long long excl = 0;
      if (t == 0) {
        if (threadIdx.x == 0) st_rlx(&w.tstat[0], (2ull << 62) | (unsigned long long)agg);
      } else {
        if (threadIdx.x == 0) st_rlx(&w.tstat[t], (1ull << 62) | (unsigned long long)agg);
        excl = lookback(w, t);
        if (threadIdx.x == 0) st_rlx(&w.tstat[t], (2ull << 62) | (unsigned long long)(excl + agg));
      }
      if (threadIdx.x == 0) s_excl = excl;
    }
    __syncthreads();
    const long long excl = s_excl;
    // the first (B - excl) unclustered positions of this tile are active
    unsigned act = 0;
    long long r = excl + mine;
#pragma unroll
    for (int k = 0; k < SIPT; k++) {
      if (un & (1u << k)) {
        if (r < B) {
          act |= 1u << k;
          if (r == B - 1) {
            c->r_last = base + k;
            st_rlx(&c->select_done, 1);
          }
        }
        r++;
      }
    }
    activate(w, c, vv, act, base, exact, round_end(w, h.phase), sh, &s_base);
    if (excl + agg >= B) break;
    __syncthreads();
  }
}

// The practical schedule's active set: the unclustered vertices among the
// next B_i positions of pi (Binomial batches over the unprocessed suffix).
// No prefix count is needed, so tiles are dealt statically.
__global__ void __launch_bounds__(SEL_BS) k_select_range(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done) return;
  __shared__ int64_t sh[SEL_BS / 64 + 1];
  __shared__ unsigned long long s_base;
  const int64_t cur0 = h.cursor;
  const int64_t end = cur0 + h.b < w.n ? cur0 + h.b : w.n;
  for (int64_t t = blockIdx.x; cur0 + t * TSEL < end; t += gridDim.x) {
    const int64_t base = cur0 + t * TSEL + (int64_t)threadIdx.x * SIPT;
    int32_t vv[SIPT];
    const unsigned un = load_slots(w, base, end, vv);
    activate(w, c, vv, un, base, false, round_end(w, h.phase), sh, &s_base);
    __syncthreads();
  }
}

// -------------------------------------------------------------- elect -----

__global__ void __launch_bounds__(BS) k_elect(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done) return;
  const unsigned long long ap = h.a_pack;
  lb_walk(w.alist, w.awork, pk_cnt(ap), pk_work(ap), w.off, round_end(w, h.phase), round_col(w, h.phase), nullptr,
          w.ainfo, [&](Items &it) {
    uint8_t su[IPT];
#pragma unroll
    for (int k = 0; k < IPT; k++) su[k] = (it.edge >> k & 1) ? w.state[it.u[k]] : (uint8_t)UNCL;
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      bool conf = false;
      // an ACTIVE mark is always this round's: C4 settles every active vertex
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

// Roots (no earlier active neighbour) are centers at once; the rest wait.
__global__ void __launch_bounds__(BS) k_classify(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done) return;
  __shared__ StageBufI<2 * BS> sb;
  stage_init(sb);
  const int64_t na = pk_cnt(h.a_pack);
  const int64_t per = ((na + gridDim.x - 1) / gridDim.x + BS - 1) / BS * BS;
  const int64_t a0 = (int64_t)blockIdx.x * per, a1 = a0 + per < na ? a0 + per : na;
  for (int64_t ib = a0; ib < a1; ib += BS) {
    const int64_t i = ib + threadIdx.x;
    int32_t a = 0;
    bool blocked = false;
    if (i < a1) {
      a = w.alist[i];
      blocked = w.flag[a] != 0;
      if (!blocked) {
        const RowInfo ri = w.ainfo[i];
        w.state[a] = CENTER;
        w.lab[a] = ri.rank;
        stage_push_info(sb, a, ri);
      }
    }
    const unsigned long long m = __ballot(blocked);  // blocked vertices are rare
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      unsigned base = 0;
      if (lane_id() == leader) base = atomicAdd(&c->n_blocked, (unsigned)__popcll(m));
      base = __shfl(base, leader, 64);
      if (blocked) w.blist[base + __popcll(m & lanemask_lt())] = a;
    }
    __syncthreads();
    if (sb.cnt > BS) stage_flush(sb, &c->c_pack, w.clist, w.cwork, nullptr, w.cinfo, sb.info);
  }
  stage_flush(sb, &c->c_pack, w.clist, w.cwork, nullptr, w.cinfo, sb.info);
}

// One workgroup settles the blocked vertices: the greedy MIS of G[A] in pi
// order restricted to them (rule 1).  A blocked vertex is a non-center as soon
// as an earlier active neighbour is a center, and a center once every earlier
// active neighbour is a non-center.
constexpr int RBS = 1024;

__device__ inline void mark_decided(Ws &w, int32_t i, unsigned *tail) {
  const unsigned q = atomicAdd(tail, 1u);
  w.bq[q] = i;
}

// The conflict edges are listed: build the dependence graph among the blocked
// vertices (edge (a, u): a waits for u) and settle it from the vertices whose
// earlier neighbours are all decided, level by level.  Every blocked vertex
// enters the queue once, when it is decided, and then walks its later
// neighbours once: O(blocked + conflict edges) work, one barrier per level.
__device__ void resolve_listed(Ws &w, Ctrl *c, int64_t nb, int64_t ne, const int64_t *rend) {
  __shared__ unsigned s_tail;
  __shared__ int64_t sh[RBS / 64 + 1];
  __shared__ int64_t s_carry;
  const int64_t total_dep = ne;  // upper bound of the dependence edges
  if (threadIdx.x == 0) {
    s_tail = 0;
    s_carry = 0;
  }
  for (int64_t i = threadIdx.x; i < nb; i += RBS) {
    w.bpos[w.blist[i]] = (int32_t)i;
    w.bpend[i] = 0;
    w.bdec[i] = 0;
    w.bdep[i] = 0;
  }
  __syncthreads();
  // an earlier neighbour that is a center already (a root) decides a at
  // once; an earlier blocked one is a dependence
  for (int64_t e = threadIdx.x; e < ne; e += RBS) {
    const int2 ed = w.cedge[e];
    const int32_t ia = w.bpos[ed.x];
    if (w.state[ed.y] == CENTER) {
      w.bdec[ia] = 2;
    } else {
      atomicAdd(&w.bpend[ia], 1);
      atomicAdd(&w.bdep[w.bpos[ed.y]], 1);
    }
  }
  __syncthreads();
  // inclusive prefix of the dependents' counts: bdep[i] = end of i's range
  for (int64_t i0 = 0; i0 < nb; i0 += RBS) {
    const int64_t i = i0 + threadIdx.x;
    const int64_t x = i < nb ? w.bdep[i] : 0;
    int64_t tot;
    const int64_t pre = wg_excl_scan<RBS>(x, &tot, sh) + s_carry;
    if (i < nb) w.bdep[i] = (int32_t)(pre + x);
    __syncthreads();
    if (threadIdx.x == 0) s_carry += tot;
    __syncthreads();
  }
  if (s_carry > total_dep) {  // cannot happen: every dependence is a listed edge
    if (threadIdx.x == 0) set_error(c, ERR_OVERFLOW);
    return;
  }
  const int64_t ndep = s_carry;
  // fill from the ends down: afterwards bdep[i] = start of i's range
  for (int64_t e = threadIdx.x; e < ne; e += RBS) {
    const int2 ed = w.cedge[e];
    if (w.state[ed.y] != CENTER) {
      const int32_t slot = atomicSub(&w.bdep[w.bpos[ed.y]], 1) - 1;
      w.bradj[slot] = w.bpos[ed.x];
    }
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < nb; i += RBS) {
    if (w.bdec[i] == 2) {
      mark_decided(w, (int32_t)i, &s_tail);
    } else if (w.bpend[i] == 0) {
      w.bdec[i] = 1;
      mark_decided(w, (int32_t)i, &s_tail);
    }
  }
  __syncthreads();
  int64_t h0 = 0;
  for (int64_t level = 0; level <= nb; level++) {
    const int64_t h1 = s_tail;  // the decided indices this level walks
    __syncthreads();            // every thread has read it before any appends
    if (h0 >= h1) break;
    for (int64_t q = h0 + threadIdx.x; q < h1; q += RBS) {
      const int32_t x = w.bq[q];
      const bool center = w.bdec[x] == 1;
      const int64_t d0 = w.bdep[x], d1 = x + 1 < nb ? w.bdep[x + 1] : ndep;
      for (int64_t d = d0; d < d1; d++) {
        const int32_t y = w.bradj[d];
        if (center) {
          if (atomicCAS(&w.bdec[y], 0, 2) == 0) mark_decided(w, y, &s_tail);
        } else if (atomicSub(&w.bpend[y], 1) == 1) {
          if (atomicCAS(&w.bdec[y], 0, 1) == 0) mark_decided(w, y, &s_tail);
        }
      }
    }
    __syncthreads();
    h0 = h1;
  }
  for (int64_t i0 = 0; i0 < nb; i0 += RBS) {
    const int64_t i = i0 + threadIdx.x;
    int32_t a = 0;
    bool promote = false;
    if (i < nb) {
      a = w.blist[i];
      const int d = w.bdec[i];
      if (d == 1) promote = true;
      else w.state[a] = NONCENTER;
      if (d == 0) set_error(c, ERR_NO_PROGRESS);  // every blocked vertex is decided by now
    }
    RowInfo ri{0, 0, 0};
    if (promote) {
      ri = RowInfo{w.off[a], (int32_t)(rend[a] - w.off[a]), w.rank[a]};
      w.state[a] = CENTER;
      w.lab[a] = ri.rank;
    }
    wave_append_info(promote, a, ri, &c->c_pack, w.clist, w.cwork, w.cinfo);
  }
}

// Too many conflict edges to list: sweep the rows of the blocked vertices
// until nothing changes (every earlier-ranked unclustered neighbour of an
// active vertex is active).  Each sweep settles at least the lowest-ranked
// undecided vertex.
__device__ void resolve_rows(Ws &w, Ctrl *c, int64_t nb, const int64_t *rend, const int32_t *col) {
  __shared__ int s_any;
  for (int64_t iter = 0; iter <= nb; iter++) {
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    for (int64_t i0 = 0; i0 < nb; i0 += RBS) {
      const int64_t i = i0 + threadIdx.x;
      int32_t a = 0;
      bool promote = false;
      if (i < nb) {
        a = w.blist[i];
        if (w.state[a] == ACTIVE) {
          const int32_t ra = w.rank[a];
          bool center_before = false, undecided_before = false;
          for (int64_t e = w.off[a]; e < rend[a] && !center_before; e++) {
            const int32_t u = col[e];
            if (!unc_bit(w.unc, u)) continue;
            const uint8_t su = w.state[u];
            if ((su == CENTER || su == ACTIVE) && w.rank[u] < ra) {
              if (su == CENTER) center_before = true;
              else undecided_before = true;
            }
          }
          if (center_before) w.state[a] = NONCENTER;
          else if (!undecided_before) promote = true;
          else s_any = 1;
        }
      }
      RowInfo ri{0, 0, 0};
      if (promote) {
        ri = RowInfo{w.off[a], (int32_t)(rend[a] - w.off[a]), w.rank[a]};
        w.state[a] = CENTER;
        w.lab[a] = ri.rank;
      }
      wave_append_info(promote, a, ri, &c->c_pack, w.clist, w.cwork, w.cinfo);
    }
    __syncthreads();
    if (!s_any) break;
  }
}

__global__ void __launch_bounds__(RBS) k_resolve(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done) return;
  const int64_t nb = h.n_blocked;
  if (nb == 0) return;
  const int64_t ne = h.n_cedges;
  if (ne <= w.cedge_cap) resolve_listed(w, c, nb, ne, round_end(w, h.phase));
  else resolve_rows(w, c, nb, round_end(w, h.phase), round_col(w, h.phase));
  __syncthreads();
  for (int64_t i = threadIdx.x; i < nb; i += RBS) w.flag[w.blist[i]] = 0;
}

// -------------------------------------------------------------- claim -----

constexpr int CLAIM_CAP = 2 * TW;  // staged newly claimed vertices (a tile adds <= TW)

__global__ void __launch_bounds__(BS) k_claim(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done) return;
  const bool c4 = w.algo == ALGO_C4;
  const unsigned long long lp = c4 ? h.c_pack : h.a_pack;
  const int32_t *list = c4 ? w.clist : w.alist;
  const int64_t *work = c4 ? w.cwork : w.awork;
  const RowInfo *info = c4 ? w.cinfo : w.ainfo;
  __shared__ unsigned s_atom;
  __shared__ IdBuf<CLAIM_CAP> sb;
  if (threadIdx.x == 0) s_atom = 0;
  id_init(sb);
  lb_walk(
      list, work, pk_cnt(lp), pk_work(lp), w.off, round_end(w, h.phase), round_col(w, h.phase), nullptr, info,
      [&](Items &it) {
        bool un[IPT];
#pragma unroll
        for (int k = 0; k < IPT; k++) un[k] = (it.edge >> k & 1) && unc_bit(w.unc, it.u[k]);
        bool elig[IPT];
        int32_t cur[IPT];
#pragma unroll
        for (int k = 0; k < IPT; k++) {
          elig[k] = un[k];
          if (!c4 && un[k] && w.state[it.u[k]] == ACTIVE) {  // ClusterWild! claims Gamma(c) \ A
            elig[k] = false;
            if (w.lab[it.u[k]] < it.val[k]) w.flag[it.v[k]] = 1;  // rule 1 broken (lab = rank here)
          }
          cur[k] = elig[k] ? w.lab[it.u[k]] : 0;  // stale reads are safe: labels only decrease
        }
        unsigned atom = 0;
#pragma unroll
        for (int k = 0; k < IPT; k++) {
          if (elig[k] && it.val[k] < cur[k]) {
            const int32_t old = atomicMin(&w.lab[it.u[k]], it.val[k]);
            atom++;
            if (old == INF) id_push(sb, it.u[k]);  // the newly claimed list
          }
        }
        if (atom) atomicAdd(&s_atom, atom);
      },
      NoEpilogue(),
      [&]() {
        __syncthreads();
        if (sb.cnt > CLAIM_CAP - TW) id_flush(sb, &c->n_pack, w.nlist);
      });
  id_flush(sb, &c->n_pack, w.nlist);
  if (threadIdx.x == 0 && s_atom) atomicAdd(&c->spread_atom[blockIdx.x & 63], (unsigned long long)s_atom);
}

__device__ inline void hist_add(int *s_hist, int *g_hist, int d, int x) {
  if (d <= 0) return;
  if (d < HLDS) atomicAdd(&s_hist[d], x);
  else atomicAdd(&g_hist[d], x);
}

// The newly clustered -- the listed centers (C4's center list, ClusterWild!'s
// active list) and the newly claimed -- leave the unclustered bitmap;
// ClusterWild! conflict marks are counted; the scan tiles of this round are
// forgotten.  In the exact phase the claimed vertices that still had
// unclustered neighbours go to the peel list.  Centers do not: every
// unclustered neighbour of a center is claimed in the same round (C4 claims
// all of them and no two centers are adjacent; ClusterWild!'s active
// neighbours are centers themselves), so a center's row has nobody left to
// peel; it only leaves the degree histogram.
__global__ void __launch_bounds__(BS) k_clear(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done) return;
  __shared__ StageBuf<2 * BS> sp;
  __shared__ int s_hist[HLDS];
  for (int i = threadIdx.x; i < HLDS; i += BS) s_hist[i] = 0;
  stage_init(sp);
  const bool cw = w.algo == ALGO_CW, exact = h.phase == PHASE_EXACT;
  const int64_t *rend = round_end(w, h.phase);
  const int64_t nc = pk_cnt(cw ? h.a_pack : h.c_pack);
  const int32_t *centers = cw ? w.alist : w.clist;
  const int64_t nn = nc + pk_cnt(h.n_pack);
  unsigned conf = 0;
  const int64_t per = ((nn + gridDim.x - 1) / gridDim.x + BS - 1) / BS * BS;
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = i0 + per < nn ? i0 + per : nn;
  for (int64_t ib = i0; ib < i1; ib += BS) {
    const int64_t i = ib + threadIdx.x;
    if (i < i1) {
      const bool center = i < nc;
      const int32_t u = center ? centers[i] : w.nlist[i - nc];
      atomicAnd(&w.unc[u >> 5], ~(1u << (u & 31)));
      if (cw && w.flag[u]) {
        w.flag[u] = 0;
        conf++;
      }
      if (exact) {
        const int32_t d = w.ub[u];
        if (center) hist_add(s_hist, w.hist, d, -1);
        else if (d > 0) stage_push(sp, u, (int32_t)(rend[u] - w.off[u]));
      }
    }
    __syncthreads();
    if (sp.cnt > BS) stage_flush(sp, &c->p_pack, w.plist, w.pwork);
  }
  stage_flush(sp, &c->p_pack, w.plist, w.pwork);
  const int64_t tiles = (int64_t)h.tile_counter + 1;
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < tiles && t < w.tstat_cap;
       t += (int64_t)gridDim.x * BS)
    w.tstat[t] = 0;
  if (cw) {
    const int64_t s = wave_sum((int64_t)conf);
    if (lane_id() == 0 && s) atomicAdd(&c->spread_conf[blockIdx.x & 63], (unsigned long long)s);
  }
  if (exact) {
    __syncthreads();
    for (int i = threadIdx.x; i < HLDS; i += BS)
      if (s_hist[i]) atomicAdd(&w.hist[i], s_hist[i]);
  }
}

// --------------------------------------------------------------- peel -----
// Exact phase: every unclustered neighbour of a newly clustered vertex loses
// one remaining degree; the degree histogram follows (low bins per workgroup).

__global__ void __launch_bounds__(BS) k_peel(Ws w) {
  Ctrl *c = w.ctrl;
  const CtrlHead h = ctrl_head(c);
  if (h.done || h.phase != PHASE_EXACT) return;
  __shared__ int s_hist[HLDS];
  __shared__ unsigned s_atom;
  for (int i = threadIdx.x; i < HLDS; i += BS) s_hist[i] = 0;
  if (threadIdx.x == 0) s_atom = 0;
  __syncthreads();
  const unsigned long long pp = h.p_pack;
  lb_walk(w.plist, w.pwork, pk_cnt(pp), pk_work(pp), w.off, round_end(w, h.phase), round_col(w, h.phase), nullptr,
          nullptr, [&](Items &it) {
#pragma unroll
    for (int k = 0; k < IPT; k++)
      if (it.vert >> k & 1) hist_add(s_hist, w.hist, w.ub[it.v[k]], -1);  // the vertex leaves
    bool un[IPT];
#pragma unroll
    for (int k = 0; k < IPT; k++) un[k] = (it.edge >> k & 1) && unc_bit(w.unc, it.u[k]);
    unsigned dec = 0;
#pragma unroll
    for (int k = 0; k < IPT; k++)
      if (un[k]) {
        const int32_t old = atomicSub(&w.ub[it.u[k]], 1);
        hist_add(s_hist, w.hist, old, -1);
        hist_add(s_hist, w.hist, old - 1, 1);
        dec++;
      }
    if (dec) atomicAdd(&s_atom, dec);
  });
  __syncthreads();
  for (int i = threadIdx.x; i < HLDS; i += BS)
    if (s_hist[i]) atomicAdd(&w.hist[i], s_hist[i]);
  if (threadIdx.x == 0 && s_atom) atomicAdd(&c->spread_atom[blockIdx.x & 63], (unsigned long long)s_atom);
}

// -------------------------------------------------------------- close -----
// One wave: record the finished round, find Delta_{i+1}, size the next round.

__global__ void __launch_bounds__(64) k_close(Ws w) {
  Ctrl *c = w.ctrl;
  if (c->done) return;
  const long long now = (long long)wall_clock64();
  long long lone = 0;  // centers settled by k_select
  long long xlow = 0;  // entries of lower-degree rows recounted at the switch
  {  // fold the spread statistics of the round
    const int l = lane_id();
    const unsigned long long sa = (unsigned long long)wave_sum((int64_t)c->spread_atom[l]);
    const unsigned long long sc = (unsigned long long)wave_sum((int64_t)c->spread_conf[l]);
    lone = wave_sum((int64_t)c->spread_lone[l]);
    xlow = wave_sum((int64_t)c->x_low[l]);
    c->spread_atom[l] = 0;
    c->spread_conf[l] = 0;
    c->spread_lone[l] = 0;
    c->x_low[l] = 0;
    if (l == 0) {
      c->sum_atomics += sa;
      c->conflicts += sc;
    }
  }
  long long n_rem = 0, delta = 0, round = 0;
  int done = 0;
  float fconf = 0.f, fclaim = 0.f, feps = 0.f;
  long long prev_delta = 0;
  if (threadIdx.x == 0) {
    prev_delta = c->delta;
    if (c->has_round) {
      const int phase_run = c->phase;  // phase the finished round ran in
      const bool c4 = w.algo == ALGO_C4;
      const long long listed = c4 ? pk_cnt(c->c_pack) : pk_cnt(c->a_pack);  // centers in a list
      const long long centers = listed + lone;
      const long long newly = pk_cnt(c->n_pack) + listed + lone;
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
      unsigned long long resc = pk_work(c->x_pack) + (unsigned long long)xlow;
      for (int j = 0; j < DITER; j++) resc += pk_work(c->r_pack[j]);
      c->sum_elect += c4 ? (unsigned long long)pk_work(c->a_pack) : 0ull;
      c->sum_claim += c4 ? (unsigned long long)pk_work(c->c_pack) : (unsigned long long)pk_work(c->a_pack);
      c->sum_rescan += resc;
      c->sum_peel += phase_run == PHASE_EXACT ? (unsigned long long)pk_work(c->p_pack) : 0ull;
      c->sum_atomics += (unsigned long long)(pk_cnt(c->n_pack) + listed);  // bitmap clears of the listed
      c->sum_blocked += (unsigned long long)conf;
      c->feat_conf = c->b > 0 ? (float)conf / (float)c->b : 0.f;
      c->feat_claim = c->n_start > 0 ? (float)(newly - centers) / (float)c->n_start : 0.f;
      c->feat_eps = (float)c->eps_used;
      c->cursor = c->r_last + 1;
      c->n_rem = c->n_start - newly;
      c->round += 1;
      // every round of the fixed rule clusters a vertex; the practical
      // schedule can have empty rounds and is bounded by its length instead
      if (w.policy != POL_BINOMIAL && c->round > w.n + 1) set_error(c, ERR_NO_PROGRESS);
      if (w.fault_round > 0 && c->round == w.fault_round) set_error(c, ERR_INJECTED);
      long long d = 0;
      if (w.policy == POL_BINOMIAL) {
        d = delta_hat(w, c->round);  // Delta-hat_{i+1}: no remaining degree is kept
      } else if (phase_run == PHASE_LAZY) {  // Delta_{i+1} (lazy search, or the exact histogram below)
        const DSearch s = dsearch(c, DITER);
        if (s.switching) c->phase = PHASE_EXACT;
        else d = s.delta;
      }
      c->delta = d;
    } else {
      c->delta = w.max_deg;  // Delta_0 (= Delta-hat_0)
    }
    c->has_round = 1;
    c->a_pack = c->c_pack = c->n_pack = c->p_pack = 0;
    c->tile_counter = 0;
    c->select_done = 0;
    c->n_blocked = 0;
    c->n_cedges = 0;
    c->conflicts = 0;
    for (int j = 0; j < DITER; j++) {
      c->r_pack[j] = 0;
      c->d_max[j] = 0;
    }
    c->x_pack = 0;
    if (c->n_rem <= 0 || c->error || (w.max_rounds > 0 && c->round >= w.max_rounds)) c->done = 1;
    // the practical schedule ends by taking every remaining position, so it
    // cannot run out while vertices are left
    if (!c->done && w.policy == POL_BINOMIAL && c->round >= w.sched_len) {
      set_error(c, ERR_NO_PROGRESS);
      c->done = 1;
    }
    n_rem = c->n_rem;
    delta = c->delta;
    round = c->round;
    done = c->done;
    fconf = c->feat_conf;
    fclaim = c->feat_claim;
    feps = c->feat_eps;
  }
  // exact phase: Delta = highest non-empty histogram bin, at most Delta_i
  int exact = 0;
  long long dprev = 0;
  if (threadIdx.x == 0) {
    exact = c->phase == PHASE_EXACT && c->has_round && !c->done;
    dprev = prev_delta;
  }
  exact = __shfl(exact, 0, 64);
  dprev = __shfl(dprev, 0, 64);
  if (exact) {
    long long found = 0;
    for (long long top = (dprev < w.max_deg ? dprev : w.max_deg); top >= 1 && !found; top -= 64) {
      const long long x = top - lane_id();
      const bool nz = x >= 1 && w.hist[x] > 0;
      const unsigned long long m = __ballot(nz);
      if (m) found = top - (__ffsll((long long)m) - 1);
    }
    if (threadIdx.x == 0) {
      c->delta = found;
      delta = found;
    }
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
      if (w.policy == POL_BINOMIAL) {  // positions: the last one taken is known now
        const long long left = w.n - c->cursor;
        if (b > left) b = left;
        c->r_last = c->cursor + b - 1;
      }
      c->b = b;
      c->eps_used = eps_used;
      if (fb) c->fallback = 1;
      c->n_start = n_rem;
      c->t_start = now;
    }
  }
  if (threadIdx.x == 0 && w.progress) {
    const unsigned long long p = (unsigned long long)(unsigned)round | (unsigned long long)(done != 0) << PROGRESS_DONE |
                                 (unsigned long long)(c->phase == PHASE_EXACT) << PROGRESS_EXACT |
                                 (unsigned long long)(c->error != 0) << PROGRESS_ERROR;
    // relaxed: the host acts on this word alone and reads the rest of the
    // state only after the stream has drained
    __hip_atomic_store(w.progress, p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// ----------------------------------------------------------- finalize -----

__global__ void __launch_bounds__(BS) k_finalize(Ws w, int32_t *labels) {
  const int64_t n = w.n;
  // by input id, so the labels are written in order; only the ids that are
  // not isolated look at their internal state
  for (int64_t vin = (int64_t)blockIdx.x * BS + threadIdx.x; vin < n; vin += (int64_t)gridDim.x * BS) {
    const int32_t v = w.perm[vin];
    if (v >= w.iso_start && w.max_rounds == 0) {  // a complete run settled every isolated vertex alone
      labels[vin] = (int32_t)vin;
      continue;
    }
    const int32_t l = w.lab[v];
    // no label: a center k_select settled (an isolated vertex -- a partial
    // run labels those it reached -- or a vertex whose bit it cleared), or
    // still unclustered
    const bool lone = l == INF && v < w.iso_start && !unc_bit(w.unc, v);
    if (lone) {
      labels[vin] = (int32_t)vin;
    } else if (l == INF && w.max_rounds > 0) {
      labels[vin] = -1;  // a partial run left v unclustered
    } else if (l < 0 || (int64_t)l >= n) {
      set_error(w.ctrl, ERR_LABEL);
      labels[vin] = -1;
    } else {
      labels[vin] = w.order_in[l];  // the input id at the center's position (a center's own)
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

hipError_t launch_init(const Ws &w, const unsigned *lvl_init_cnt, hipStream_t s) {
  if (!w.order_mapped) hipLaunchKernelGGL(k_check_order, dim3(grid_for(w.n, 4096)), dim3(BS), 0, s, w);
  hipLaunchKernelGGL(k_init, dim3(grid_for(w.n, 4096)), dim3(BS), 0, s, w, lvl_init_cnt);
  hipLaunchKernelGGL(k_close, dim3(1), dim3(64), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_round(const Ws &w, hipStream_t s, const LaunchShape &ls) {
  const bool binomial = w.policy == POL_BINOMIAL;
  if (binomial) hipLaunchKernelGGL(k_select_range, dim3(ls.select_grid), dim3(SEL_BS), 0, s, w);
  else hipLaunchKernelGGL(k_select, dim3(ls.select_grid), dim3(SEL_BS), 0, s, w);
  if (w.algo == ALGO_C4) {
    hipLaunchKernelGGL(k_elect, dim3(ls.edge_grid), dim3(BS), 0, s, w);
    hipLaunchKernelGGL(k_classify, dim3(ls.vertex_grid), dim3(BS), 0, s, w);
    hipLaunchKernelGGL(k_resolve, dim3(1), dim3(RBS), 0, s, w);
  }
  hipLaunchKernelGGL(k_claim, dim3(ls.edge_grid), dim3(BS), 0, s, w);
  hipLaunchKernelGGL(k_clear, dim3(ls.vertex_grid), dim3(BS), 0, s, w);
  if (binomial) {
    // Delta-hat needs no remaining degrees: no peel, no Delta search
  } else if (ls.exact_seen) {
    // the run has switched to exact degrees for good: no lazy search
    hipLaunchKernelGGL(k_peel, dim3(ls.edge_grid), dim3(BS), 0, s, w);
  } else {
    hipLaunchKernelGGL(k_peel, dim3(ls.edge_grid), dim3(BS), 0, s, w);
    hipLaunchKernelGGL(k_dscan<0>, dim3(ls.vertex_grid), dim3(BS), 0, s, w);
    hipLaunchKernelGGL(k_rescan<0>, dim3(ls.edge_grid), dim3(BS), 0, s, w);
    hipLaunchKernelGGL(k_dscan<1>, dim3(ls.vertex_grid), dim3(BS), 0, s, w);
    hipLaunchKernelGGL(k_rescan<1>, dim3(ls.edge_grid), dim3(BS), 0, s, w);
    hipLaunchKernelGGL(k_dscan<2>, dim3(ls.vertex_grid), dim3(BS), 0, s, w);
    hipLaunchKernelGGL(k_rescan<2>, dim3(ls.edge_grid), dim3(BS), 0, s, w);
    hipLaunchKernelGGL(k_xlist, dim3(grid_for(w.n, ls.vertex_grid)), dim3(BS), 0, s, w);
    hipLaunchKernelGGL(k_xcount, dim3(ls.edge_grid), dim3(BS), 0, s, w);
  }
  hipLaunchKernelGGL(k_close, dim3(1), dim3(64), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_finalize(const Ws &w, int32_t *labels, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(grid_for(w.n, 4096)), dim3(BS), 0, s, w, labels);
  return hipGetLastError();
}

}  // namespace ccd
