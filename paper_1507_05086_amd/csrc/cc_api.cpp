// cc_api.cpp -- the C ABI of include/cc.h: argument checks, device buffers,
// the host side of the round loop, statistics and traces.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cc.h"
#include "cc_device.h"
#include "cc_launch.h"

using namespace ccd;

namespace {

thread_local std::string g_last_error;

int32_t fail(int32_t code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? CC_ERR_OUT_OF_MEMORY : CC_ERR_DEVICE,    \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

template <class T>
hipError_t dalloc(T **p, size_t count) {
  return hipMalloc((void **)p, sizeof(T) * (count > 0 ? count : 1));
}

struct Policy {
  int32_t kind = CC_EPS_FIXED;
  std::vector<float> mlp;
  std::vector<int64_t> sched;
  double eps_min = 1.0 / 16, eps_max = 16.0;
};
Policy g_policy;
std::mutex g_policy_mu;

// Device workspace of a run (allocated on the first run of a graph).
struct Workspace {
  bool ready = false;
  int32_t *rank = nullptr, *lab = nullptr, *ub = nullptr;
  uint32_t *unc = nullptr;
  uint8_t *state = nullptr, *flag = nullptr;
  int32_t *alist = nullptr, *clist = nullptr, *nlist = nullptr, *blist = nullptr;
  int64_t *awork = nullptr, *cwork = nullptr, *nwork = nullptr;
  int32_t *rlist = nullptr, *xlist = nullptr, *plist = nullptr;
  int64_t *rwork = nullptr, *xwork = nullptr, *pwork = nullptr;
  unsigned long long *racc = nullptr;
  int64_t rcap = 0;
  int32_t *lvl = nullptr;
  int *hist = nullptr;
  int64_t hist_len = 0;
  int2 *cedge = nullptr;
  int64_t cedge_cap = 0;
  unsigned long long *tstat = nullptr;
  int64_t tstat_cap = 0;
  Ctrl *ctrl = nullptr;
  RoundRec *trace = nullptr;
  int64_t trace_cap = 0;
  int32_t *order_buf = nullptr, *label_buf = nullptr;
  int64_t *sched = nullptr;
  int64_t sched_cap = 0;
  float *mlp = nullptr;
  int *host_flags = nullptr;  // pinned: done, error, has_round, fallback, phase
  int32_t *cost_size = nullptr;
  long long *cost_acc = nullptr;
  int *dev_err = nullptr;
};

}  // namespace

struct cc_graph {
  int64_t n = 0, nnz = 0;
  int32_t num_graphs = 1;
  bool borrowed = false;
  int64_t *off = nullptr;
  int32_t *col = nullptr;
  int64_t *vtx_ptr = nullptr;  // device, batches only
  int32_t *gid = nullptr;      // device, batches only
  int64_t *wall = nullptr;     // device [n+1]
  int64_t max_deg = 0;
  int64_t n_hi = 0;            // vertices with degree >= DSW
  int32_t *lvl_init = nullptr; // device: initial bound buckets
  int64_t *lvl_off = nullptr;  // device [NLVL+1]
  unsigned *lvl_cnt0 = nullptr;  // device [NLVL]: initial entries per level
  int64_t lvl_total = 0;
  std::vector<int64_t> h_vtx_ptr;
  std::vector<int64_t> m_per_graph;
  Workspace ws;
};

namespace {

void free_ws(Workspace &w) {
  void *ptrs[] = {w.rank, w.lab, w.ub, w.unc, w.state, w.flag, w.alist, w.clist, w.nlist, w.blist,
                  w.awork, w.cwork, w.nwork, w.rlist, w.xlist, w.rwork, w.xwork, w.racc, w.lvl, w.hist, w.plist, w.pwork,
                  w.cedge, w.tstat, w.ctrl, w.trace, w.order_buf, w.label_buf, w.sched, w.mlp,
                  w.cost_size, w.cost_acc, w.dev_err};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (w.host_flags) (void)hipHostFree(w.host_flags);
  w = Workspace();
}

void free_graph(cc_graph *g) {
  if (!g) return;
  free_ws(g->ws);
  if (!g->borrowed) {
    if (g->off) (void)hipFree(g->off);
    if (g->col) (void)hipFree(g->col);
  }
  if (g->vtx_ptr) (void)hipFree(g->vtx_ptr);
  if (g->gid) (void)hipFree(g->gid);
  if (g->wall) (void)hipFree(g->wall);
  if (g->lvl_init) (void)hipFree(g->lvl_init);
  if (g->lvl_off) (void)hipFree(g->lvl_off);
  if (g->lvl_cnt0) (void)hipFree(g->lvl_cnt0);
  delete g;
}

int32_t ensure_ws(cc_graph *g) {
  Workspace &w = g->ws;
  if (w.ready) return CC_OK;
  const int64_t n = g->n > 0 ? g->n : 1;
  HIP_TRY(dalloc(&w.rank, n));
  HIP_TRY(dalloc(&w.lab, n));
  HIP_TRY(dalloc(&w.ub, n));
  HIP_TRY(dalloc(&w.unc, (size_t)(n + 31) / 32));
  HIP_TRY(dalloc(&w.state, n));
  HIP_TRY(dalloc(&w.flag, n));
  HIP_TRY(dalloc(&w.alist, n));
  HIP_TRY(dalloc(&w.clist, n));
  HIP_TRY(dalloc(&w.nlist, n));
  HIP_TRY(dalloc(&w.blist, n));
  HIP_TRY(dalloc(&w.awork, n));
  HIP_TRY(dalloc(&w.cwork, n));
  HIP_TRY(dalloc(&w.nwork, n));
  w.rcap = g->n_hi + 1;
  HIP_TRY(dalloc(&w.rlist, (size_t)(DITER * w.rcap)));
  HIP_TRY(dalloc(&w.rwork, (size_t)(DITER * w.rcap)));
  HIP_TRY(dalloc(&w.racc, (size_t)(DITER * w.rcap)));
  HIP_TRY(dalloc(&w.xlist, n));
  HIP_TRY(dalloc(&w.xwork, n));
  HIP_TRY(dalloc(&w.plist, n));
  HIP_TRY(dalloc(&w.pwork, n));
  HIP_TRY(dalloc(&w.lvl, (size_t)(g->lvl_total > 0 ? g->lvl_total : 1)));
  w.hist_len = g->max_deg + 2;
  HIP_TRY(dalloc(&w.hist, (size_t)w.hist_len));
  w.cedge_cap = n > (1 << 20) ? n : (1 << 20);
  HIP_TRY(dalloc(&w.cedge, (size_t)w.cedge_cap));
  w.tstat_cap = n / TSEL + 4096 + 2;
  HIP_TRY(dalloc(&w.tstat, (size_t)w.tstat_cap));
  HIP_TRY(hipMemset(w.tstat, 0, sizeof(unsigned long long) * (size_t)w.tstat_cap));
  HIP_TRY(dalloc(&w.ctrl, 1));
  w.trace_cap = 1 << 16;
  HIP_TRY(dalloc(&w.trace, (size_t)w.trace_cap));
  HIP_TRY(dalloc(&w.order_buf, n));
  HIP_TRY(dalloc(&w.label_buf, n));
  HIP_TRY(dalloc(&w.mlp, CC_MLP_PARAMS));
  HIP_TRY(dalloc(&w.cost_size, n));
  HIP_TRY(dalloc(&w.cost_acc, 2 * (size_t)g->num_graphs));
  HIP_TRY(dalloc(&w.dev_err, 1));
  HIP_TRY(hipHostMalloc((void **)&w.host_flags, 8 * sizeof(int), hipHostMallocDefault));
  w.ready = true;
  return CC_OK;
}

int32_t wall_clock_khz(int *khz) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(khz, hipDeviceAttributeWallClockRate, dev));
  if (*khz <= 0) *khz = 100000;
  return CC_OK;
}

int32_t run_loop(cc_graph *g, int algo, const int32_t *order, double eps, int32_t *labels,
                 cc_run_stats *stats, uint32_t flags, hipStream_t s) {
  if (!g) return fail(CC_ERR_INVALID_ARG, "graph handle is NULL");
  if (!order || !labels) return fail(CC_ERR_INVALID_ARG, "order and labels must not be NULL");
  if (!(eps > 0.0) || !(eps <= 1000.0) || !std::isfinite(eps))
    return fail(CC_ERR_INVALID_ARG, "eps must lie in (0, 1000]");
  if (flags & ~(uint32_t)(CC_INPUT_ON_DEVICE | CC_OUTPUT_ON_DEVICE))
    return fail(CC_ERR_INVALID_ARG, "unknown flag for a run");
  if (stats && stats->trace_capacity > 0 && !stats->trace)
    return fail(CC_ERR_INVALID_ARG, "stats->trace is NULL but trace_capacity > 0");
  if (g->num_graphs != 1)
    return fail(CC_ERR_INVALID_ARG, "batched graphs are clustered by the batched entry points");
  Policy pol;
  {
    std::lock_guard<std::mutex> lk(g_policy_mu);
    pol = g_policy;
  }
  if (int32_t rc = ensure_ws(g)) return rc;
  Workspace &ws = g->ws;
  const int64_t n = g->n;
  if (n == 0) {
    if (stats) {
      std::memset(stats, 0, offsetof(cc_run_stats, trace));
      stats->truncated = 0;
    }
    return CC_OK;
  }

  const int32_t *d_order = order;
  if (!(flags & CC_INPUT_ON_DEVICE)) {
    HIP_TRY(hipMemcpyAsync(ws.order_buf, order, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    d_order = ws.order_buf;
  }
  if (pol.kind == CC_EPS_TRACE && !pol.sched.empty()) {
    if ((int64_t)pol.sched.size() > ws.sched_cap) {
      if (ws.sched) HIP_TRY(hipFree(ws.sched));
      ws.sched = nullptr;
      HIP_TRY(dalloc(&ws.sched, pol.sched.size()));
      ws.sched_cap = (int64_t)pol.sched.size();
    }
    HIP_TRY(hipMemcpyAsync(ws.sched, pol.sched.data(), sizeof(int64_t) * pol.sched.size(),
                           hipMemcpyHostToDevice, s));
  }
  if (pol.kind == CC_EPS_LEARNED)
    HIP_TRY(hipMemcpyAsync(ws.mlp, pol.mlp.data(), sizeof(float) * CC_MLP_PARAMS, hipMemcpyHostToDevice, s));

  Ws w{};
  w.off = g->off;
  w.col = g->col;
  w.n = n;
  w.order = d_order;
  w.max_deg = g->max_deg;
  w.rank = ws.rank;
  w.lab = ws.lab;
  w.ub = ws.ub;
  w.unc = ws.unc;
  w.state = ws.state;
  w.flag = ws.flag;
  w.alist = ws.alist;
  w.clist = ws.clist;
  w.nlist = ws.nlist;
  w.blist = ws.blist;
  w.awork = ws.awork;
  w.cwork = ws.cwork;
  w.nwork = ws.nwork;
  w.rlist = ws.rlist;
  w.rwork = ws.rwork;
  w.racc = ws.racc;
  w.rcap = ws.rcap;
  w.xlist = ws.xlist;
  w.xwork = ws.xwork;
  w.plist = ws.plist;
  w.pwork = ws.pwork;
  w.lvl = ws.lvl;
  w.lvl_off = g->lvl_off;
  w.hist = ws.hist;
  w.cedge = ws.cedge;
  w.cedge_cap = ws.cedge_cap;
  w.tstat = ws.tstat;
  w.tstat_cap = ws.tstat_cap;
  w.ctrl = ws.ctrl;
  w.trace = ws.trace;
  w.trace_cap = ws.trace_cap;
  w.policy = pol.kind;
  w.algo = algo;
  w.eps = eps;
  w.eps_q = (int64_t)(eps * 1e6 + 0.5);
  w.sched = ws.sched;
  w.sched_len = pol.kind == CC_EPS_TRACE ? (int64_t)pol.sched.size() : 0;
  w.mlp = ws.mlp;
  w.eps_min = (float)pol.eps_min;
  w.eps_max = (float)pol.eps_max;

  // init: the permutation is checked before any kernel indexes with it
  HIP_TRY(hipMemsetAsync(ws.ctrl, 0, sizeof(Ctrl), s));
  HIP_TRY(hipMemsetAsync(ws.rank, 0xFF, sizeof(int32_t) * (size_t)n, s));
  HIP_TRY(hipMemsetAsync(ws.hist, 0, sizeof(int) * (size_t)ws.hist_len, s));
  if (g->lvl_total > 0)
    HIP_TRY(hipMemcpyAsync(ws.lvl, g->lvl_init, sizeof(int32_t) * (size_t)g->lvl_total, hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_init(w, g->lvl_cnt0, s));
  HIP_TRY(hipMemcpyAsync(ws.host_flags, &ws.ctrl->done, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (ws.host_flags[1] == ERR_PERM)
    return fail(CC_ERR_NOT_PERMUTATION, "order is not a permutation of 0..n-1");
  if (ws.host_flags[1]) return fail(CC_ERR_DEVICE, "device error during initialisation");

  LaunchShape ls{256, 2048, 1024, 0, 0};
  int64_t launched = 0, group = 4;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  HIP_TRY(hipEventCreate(&ev0));
  HIP_TRY(hipEventCreate(&ev1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evg{ev0, ev1};
  HIP_TRY(hipEventRecord(ev0, s));
  for (;;) {
    for (int64_t r = 0; r < group; r++) HIP_TRY(launch_round(w, s, ls));
    launched += group;
    HIP_TRY(hipMemcpyAsync(ws.host_flags, &ws.ctrl->done, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (ws.host_flags[0] || ws.host_flags[1]) break;
    if (ws.host_flags[4] == PHASE_EXACT) ls.exact_seen = 1;
    if (launched > n + 2) return fail(CC_ERR_NO_PROGRESS, "round loop exceeded n+1 rounds");
    group = group < 64 ? group * 2 : 64;
  }
  HIP_TRY(hipEventRecord(ev1, s));
  if (ws.host_flags[1]) {
    const int e = ws.host_flags[1];
    if (e == ERR_NO_PROGRESS) return fail(CC_ERR_NO_PROGRESS, "round loop made no progress");
    if (e == ERR_OVERFLOW) return fail(CC_ERR_DEVICE, "a device work list overflowed");
    return fail(CC_ERR_DEVICE, "device error " + std::to_string(e) + " in the round loop");
  }
  int32_t *d_labels = (flags & CC_OUTPUT_ON_DEVICE) ? labels : ws.label_buf;
  HIP_TRY(launch_finalize(w, d_labels, s));
  Ctrl hc;
  HIP_TRY(hipMemcpyAsync(&hc, ws.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hc.error) return fail(CC_ERR_DEVICE, "device error " + std::to_string(hc.error) + " while finishing");
  if (!(flags & CC_OUTPUT_ON_DEVICE)) {
    HIP_TRY(hipMemcpyAsync(labels, ws.label_buf, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (stats) {
    stats->rounds = hc.round;
    stats->scanned_elect = (int64_t)hc.sum_elect;
    stats->scanned_claim = (int64_t)hc.sum_claim;
    stats->scanned_peel = (int64_t)hc.sum_peel;
    stats->scanned_delta = (int64_t)hc.sum_rescan;
    stats->blocked = (int64_t)hc.sum_blocked;
    stats->atomics = (int64_t)hc.sum_atomics;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
    stats->loop_ms = ms;
    stats->policy_fallback = hc.fallback;
    const int64_t have = hc.round < ws.trace_cap ? hc.round : ws.trace_cap;
    stats->truncated = (hc.round > stats->trace_capacity || hc.round > ws.trace_cap) ? 1 : 0;
    const int64_t ncopy = stats->trace_capacity < have ? stats->trace_capacity : have;
    if (ncopy > 0) {
      std::vector<RoundRec> rr((size_t)ncopy);
      HIP_TRY(hipMemcpy(rr.data(), ws.trace, sizeof(RoundRec) * (size_t)ncopy, hipMemcpyDeviceToHost));
      int khz = 100000;
      if (int32_t rc = wall_clock_khz(&khz)) return rc;
      for (int64_t i = 0; i < ncopy; i++) {
        cc_round_record &o = stats->trace[i];
        const RoundRec &r = rr[(size_t)i];
        o.n_i = r.n_i;
        o.delta_i = r.delta_i;
        o.b_i = r.b_i;
        o.r_i = r.r_i;
        o.centers = r.centers;
        o.claimed = r.claimed;
        o.conflicts = r.conflicts;
        o.eps_used = r.eps_used;
        o.t_ns = (int64_t)((double)r.t_ns * 1e6 / (double)khz);
      }
    }
  }
  return CC_OK;
}

}  // namespace

extern "C" {

const char *cc_last_error(void) { return g_last_error.c_str(); }

int32_t cc_graph_from_csr(int32_t num_graphs, const int64_t *vtx_ptr, int64_t n_total, const int64_t *offsets,
                          const int32_t *cols, uint32_t flags, void *stream, cc_graph **out) {
  g_last_error.clear();
  hipStream_t s = (hipStream_t)stream;
  if (!out) return fail(CC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (flags & ~(uint32_t)(CC_VALIDATE | CC_INPUT_ON_DEVICE | CC_BORROW))
    return fail(CC_ERR_INVALID_ARG, "unknown flag for a graph");
  if (num_graphs < 1) return fail(CC_ERR_INVALID_ARG, "num_graphs must be >= 1");
  if (n_total < 0 || n_total >= ((int64_t)1 << 31)) return fail(CC_ERR_INVALID_ARG, "n_total must lie in [0, 2^31)");
  if (!offsets) return fail(CC_ERR_INVALID_ARG, "offsets is NULL");
  const bool on_dev = (flags & (CC_INPUT_ON_DEVICE | CC_BORROW)) != 0;
  std::vector<int64_t> hv;
  if (num_graphs > 1) {
    if (!vtx_ptr) return fail(CC_ERR_INVALID_ARG, "vtx_ptr is required for a batch");
    hv.assign(vtx_ptr, vtx_ptr + num_graphs + 1);
    if (hv[0] != 0 || hv[(size_t)num_graphs] != n_total)
      return fail(CC_ERR_INVALID_ARG, "vtx_ptr must start at 0 and end at n_total");
    for (int32_t i = 0; i < num_graphs; i++)
      if (hv[(size_t)i + 1] < hv[(size_t)i]) return fail(CC_ERR_INVALID_ARG, "vtx_ptr must not decrease");
  } else {
    hv = {0, n_total};
  }
  int64_t nnz = 0;
  if (on_dev) HIP_TRY(hipMemcpy(&nnz, offsets + n_total, sizeof(int64_t), hipMemcpyDeviceToHost));
  else nnz = offsets[n_total];
  if (nnz < 0 || nnz >= ((int64_t)1 << 33)) return fail(CC_ERR_INVALID_ARG, "offsets[n] must lie in [0, 2^33)");
  if (nnz > 0 && !cols) return fail(CC_ERR_INVALID_ARG, "cols is NULL");

  cc_graph *g = new cc_graph();
  g->n = n_total;
  g->nnz = nnz;
  g->num_graphs = num_graphs;
  g->h_vtx_ptr = hv;
  auto bail = [&](int32_t rc) {
    free_graph(g);
    return rc;
  };
#define G_TRY(expr)                                                                    \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return bail(fail(e_ == hipErrorOutOfMemory ? CC_ERR_OUT_OF_MEMORY : CC_ERR_DEVICE, \
                       std::string(#expr) + ": " + hipGetErrorString(e_)));            \
  } while (0)

  if (flags & CC_BORROW) {
    g->borrowed = true;
    g->off = const_cast<int64_t *>(offsets);
    g->col = const_cast<int32_t *>(cols);
  } else {
    G_TRY(dalloc(&g->off, (size_t)n_total + 1));
    G_TRY(dalloc(&g->col, (size_t)nnz));
    const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    G_TRY(hipMemcpyAsync(g->off, offsets, sizeof(int64_t) * ((size_t)n_total + 1), kind, s));
    if (nnz > 0) G_TRY(hipMemcpyAsync(g->col, cols, sizeof(int32_t) * (size_t)nnz, kind, s));
  }
  // offsets must start at 0 and never decrease (checked on the host copy)
  {
    std::vector<int64_t> ho;
    const int64_t *po = offsets;
    if (on_dev) {
      ho.resize((size_t)n_total + 1);
      G_TRY(hipMemcpyAsync(ho.data(), g->off, sizeof(int64_t) * ho.size(), hipMemcpyDeviceToHost, s));
      G_TRY(hipStreamSynchronize(s));
      po = ho.data();
    }
    if (po[0] != 0) return bail(fail(CC_ERR_INVALID_ARG, "offsets[0] must be 0"));
    for (int64_t v = 0; v < n_total; v++)
      if (po[v + 1] < po[v]) return bail(fail(CC_ERR_INVALID_ARG, "offsets must not decrease"));
    g->m_per_graph.resize((size_t)num_graphs);
    for (int32_t i = 0; i < num_graphs; i++)
      g->m_per_graph[(size_t)i] = (po[hv[(size_t)i + 1]] - po[hv[(size_t)i]]) / 2;
  }
  if (num_graphs > 1) {
    G_TRY(dalloc(&g->vtx_ptr, (size_t)num_graphs + 1));
    G_TRY(hipMemcpyAsync(g->vtx_ptr, hv.data(), sizeof(int64_t) * hv.size(), hipMemcpyHostToDevice, s));
    G_TRY(dalloc(&g->gid, (size_t)n_total));
  }
  G_TRY(dalloc(&g->wall, (size_t)n_total + 1));
  int64_t *blocksum = nullptr;
  int *derr = nullptr;
  const int64_t nb = (n_total + (int64_t)BS * 4 - 1) / ((int64_t)BS * 4);
  G_TRY(dalloc(&blocksum, (size_t)nb + 2));
  G_TRY(dalloc(&derr, 1));
  const int none = 0x7fffffff;
  hipError_t e = hipMemcpyAsync(derr, &none, sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_graph_setup(g->off, g->col, n_total, g->vtx_ptr, num_graphs, g->gid, g->wall, blocksum,
                           (flags & CC_VALIDATE) ? 1 : 0, derr, s);
  int herr = none;
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(blocksum);
  (void)hipFree(derr);
  G_TRY(e);
  if (herr == none && n_total > 0) {
    // bound buckets: capacity of level k = vertices of degree >= 2^k
    unsigned *dcnt = nullptr;
    int *dmax = nullptr;
    G_TRY(dalloc(&dcnt, NLVL));
    G_TRY(dalloc(&dmax, 1));
    G_TRY(hipMemsetAsync(dcnt, 0, sizeof(unsigned) * NLVL, s));
    G_TRY(hipMemsetAsync(dmax, 0, sizeof(int), s));
    G_TRY(launch_level_count(g->off, n_total, dcnt, dmax, s));
    unsigned hcnt[NLVL];
    int hmax = 0;
    G_TRY(hipMemcpyAsync(hcnt, dcnt, sizeof(hcnt), hipMemcpyDeviceToHost, s));
    G_TRY(hipMemcpyAsync(&hmax, dmax, sizeof(int), hipMemcpyDeviceToHost, s));
    G_TRY(hipStreamSynchronize(s));
    g->max_deg = hmax;
    int64_t hoff[NLVL + 1];
    int64_t acc = 0, hi = 0;
    for (int k = 0; k < NLVL; k++) {
      int64_t cap = 0;
      if (k >= LVL_MIN)
        for (int j = k; j < NLVL; j++) cap += hcnt[j];
      hoff[k] = acc;
      acc += cap;
      hi += hcnt[k];
    }
    hoff[NLVL] = acc;
    g->lvl_total = acc;
    g->n_hi = hi;
    G_TRY(dalloc(&g->lvl_off, NLVL + 1));
    G_TRY(dalloc(&g->lvl_cnt0, NLVL));
    G_TRY(dalloc(&g->lvl_init, (size_t)(acc > 0 ? acc : 1)));
    G_TRY(hipMemcpyAsync(g->lvl_off, hoff, sizeof(hoff), hipMemcpyHostToDevice, s));
    G_TRY(hipMemcpyAsync(g->lvl_cnt0, hcnt, sizeof(hcnt), hipMemcpyHostToDevice, s));
    G_TRY(hipMemsetAsync(dcnt, 0, sizeof(unsigned) * NLVL, s));
    G_TRY(launch_level_fill(g->off, n_total, g->lvl_off, dcnt, g->lvl_init, s));
    G_TRY(hipStreamSynchronize(s));
    (void)hipFree(dcnt);
    (void)hipFree(dmax);
  }
  if (herr != none) {
    herr &= 0xFF;
    const char *what = herr == CC_ERR_OUT_OF_RANGE ? "a column index lies outside its graph"
                       : herr == CC_ERR_NOT_SYMMETRIC ? "edge (u,v) present without (v,u)"
                       : herr == CC_ERR_SELF_LOOP     ? "self-loop"
                       : herr == CC_ERR_DUPLICATE_EDGE ? "row not strictly ascending (duplicate entry)"
                                                       : "invalid graph";
    return bail(fail(herr, what));
  }
#undef G_TRY
  *out = g;
  return CC_OK;
}

int32_t cc_graph_destroy(cc_graph *g) {
  if (!g) return fail(CC_ERR_INVALID_ARG, "graph handle is NULL");
  free_graph(g);
  return CC_OK;
}

int32_t cc_graph_info(const cc_graph *g, int64_t *n_total, int64_t *nnz, int32_t *num_graphs) {
  if (!g) return fail(CC_ERR_INVALID_ARG, "graph handle is NULL");
  if (n_total) *n_total = g->n;
  if (nnz) *nnz = g->nnz;
  if (num_graphs) *num_graphs = g->num_graphs;
  return CC_OK;
}

int32_t cc_c4(const cc_graph *g, const int32_t *order, double eps, int32_t *labels, cc_run_stats *stats,
              uint32_t flags, void *stream) {
  g_last_error.clear();
  return run_loop(const_cast<cc_graph *>(g), ALGO_C4, order, eps, labels, stats, flags, (hipStream_t)stream);
}

int32_t cc_clusterwild(const cc_graph *g, const int32_t *order, double eps, int32_t *labels,
                       cc_run_stats *stats, uint32_t flags, void *stream) {
  g_last_error.clear();
  return run_loop(const_cast<cc_graph *>(g), ALGO_CW, order, eps, labels, stats, flags, (hipStream_t)stream);
}

int32_t cc_cost(const cc_graph *gc, const int32_t *labels, int64_t *cost, uint32_t flags, void *stream) {
  g_last_error.clear();
  cc_graph *g = const_cast<cc_graph *>(gc);
  hipStream_t s = (hipStream_t)stream;
  if (!g) return fail(CC_ERR_INVALID_ARG, "graph handle is NULL");
  if (!labels || !cost) return fail(CC_ERR_INVALID_ARG, "labels and cost must not be NULL");
  if (flags & ~(uint32_t)CC_INPUT_ON_DEVICE) return fail(CC_ERR_INVALID_ARG, "unknown flag for cc_cost");
  if (int32_t rc = ensure_ws(g)) return rc;
  Workspace &ws = g->ws;
  const int64_t n = g->n;
  const int32_t *d_lab = labels;
  if (!(flags & CC_INPUT_ON_DEVICE) && n > 0) {
    HIP_TRY(hipMemcpyAsync(ws.label_buf, labels, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    d_lab = ws.label_buf;
  }
  const int none = 0x7fffffff;
  HIP_TRY(hipMemcpyAsync(ws.dev_err, &none, sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_cost(g->off, g->col, g->wall, n, g->vtx_ptr, g->gid, d_lab, ws.cost_size, ws.cost_acc,
                      g->num_graphs, ws.dev_err, s));
  std::vector<long long> acc(2 * (size_t)g->num_graphs);
  int herr = none;
  HIP_TRY(hipMemcpyAsync(acc.data(), ws.cost_acc, sizeof(long long) * acc.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&herr, ws.dev_err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (herr != none) return fail(herr & 0xFF, "a label lies outside its graph");
  for (int32_t i = 0; i < g->num_graphs; i++)
    cost[i] = (int64_t)acc[2 * (size_t)i] + g->m_per_graph[(size_t)i] - (int64_t)acc[2 * (size_t)i + 1];
  return CC_OK;
}

int32_t cc_set_eps_policy(int32_t kind, const void *params, size_t nbytes, double eps_min, double eps_max) {
  g_last_error.clear();
  Policy p;
  p.kind = kind;
  if (kind == CC_EPS_FIXED) {
    // nothing else to read
  } else if (kind == CC_EPS_LEARNED) {
    if (!params || nbytes != sizeof(float) * CC_MLP_PARAMS)
      return fail(CC_ERR_POLICY, "learned policy needs CC_MLP_PARAMS float32 weights");
    if (!(eps_min > 0.0) || !(eps_max >= eps_min) || !(eps_max <= 1000.0))
      return fail(CC_ERR_POLICY, "need 0 < eps_min <= eps_max <= 1000");
    const float *f = (const float *)params;
    p.mlp.assign(f, f + CC_MLP_PARAMS);
    p.eps_min = eps_min;
    p.eps_max = eps_max;
  } else if (kind == CC_EPS_TRACE) {
    if (nbytes % sizeof(int64_t) != 0 || (nbytes > 0 && !params))
      return fail(CC_ERR_POLICY, "trace schedule must be an int64 array");
    const int64_t *b = (const int64_t *)params;
    p.sched.assign(b, b + nbytes / sizeof(int64_t));
    for (int64_t x : p.sched)
      if (x < 1) return fail(CC_ERR_POLICY, "every scheduled active-set size must be >= 1");
  } else {
    return fail(CC_ERR_POLICY, "unknown policy kind");
  }
  std::lock_guard<std::mutex> lk(g_policy_mu);
  g_policy = p;
  return CC_OK;
}

}  // extern "C"
