// cc_api.cpp -- the C ABI of include/cc.h: argument checks, device buffers,
// the host side of the round loop, statistics and traces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/cc.h"
#include "cc_device.h"
#include "cc_launch.h"
#include "cc_schedule.h"

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
  uint64_t bin_seed = 0;   // BINOMIAL
  double bin_delta = 0.1;  // BINOMIAL
};

// What the device schedule buffer of a workspace holds (a drawn practical
// schedule is kept for the next call with the same inputs).
struct SchedKey {
  bool binomial = false;
  int64_t n = 0, delta0 = 0;
  double eps = 0.0, delta = 0.0;
  uint64_t seed = 0;
  bool operator==(const SchedKey &o) const {
    return binomial == o.binomial && n == o.n && delta0 == o.delta0 && eps == o.eps && delta == o.delta &&
           seed == o.seed;
  }
};
Policy g_policy;
std::mutex g_policy_mu;

// A captured group of k rounds (kernels only), keyed by the bytes of the
// run's kernel arguments and the phase it was captured for.
struct RoundGraph {
  unsigned char key[sizeof(Ws)];
  int exact = -1;
  int64_t k = 0;
  hipGraphExec_t exec = nullptr;
};

// Device workspace of a run (allocated on the first run of a graph).
struct Workspace {
  bool ready = false;
  int32_t *rank = nullptr, *lab = nullptr, *ub = nullptr;
  uint32_t *unc = nullptr;
  uint8_t *state = nullptr, *flag = nullptr;
  int32_t *alist = nullptr, *clist = nullptr, *nlist = nullptr, *blist = nullptr;
  int64_t *awork = nullptr, *cwork = nullptr;
  int32_t *rlist = nullptr, *xlist = nullptr, *plist = nullptr;
  int64_t *rwork = nullptr, *xwork = nullptr, *pwork = nullptr;
  RowInfo *ainfo = nullptr, *cinfo = nullptr;
  unsigned long long *racc = nullptr;
  int64_t rcap = 0;
  int32_t *lvl = nullptr;
  int *hist = nullptr;
  int64_t hist_len = 0;
  int2 *cedge = nullptr;
  int64_t cedge_cap = 0;
  int32_t *bpos = nullptr, *bpend = nullptr, *bdec = nullptr, *bdep = nullptr, *bq = nullptr, *bradj = nullptr;
  unsigned long long *tstat = nullptr;
  int64_t tstat_cap = 0;
  Ctrl *ctrl = nullptr;
  RoundRec *trace = nullptr;
  int64_t trace_cap = 0;
  int32_t *order_buf = nullptr, *label_buf = nullptr, *iorder = nullptr;
  uint8_t *omap_buf = nullptr;  // bucketed order mapping scratch (large n only)
  int32_t *ccol = nullptr;       // rows compacted at the switch to exact degrees (single graphs; col-sized)
  int64_t *cend = nullptr;       // their ends
  OrderMap omap{};
  int64_t *sched = nullptr;
  int64_t sched_cap = 0;
  SchedKey sched_key;      // the practical schedule the sched buffer holds, if any
  int64_t sched_len = 0;   // its length
  float *mlp = nullptr;
  int *host_flags = nullptr;  // pinned: the device error word, read after the labels are finalized
  unsigned long long *progress = nullptr;  // pinned, coherent: k_close's progress word
  unsigned long long *progress_dev = nullptr;  // the same word as the device addresses it
  int32_t *cost_size = nullptr;
  long long *cost_acc = nullptr;
  int *dev_err = nullptr;
  hipStream_t cap = nullptr;  // private stream the round groups are captured on
  std::vector<RoundGraph> graphs;
};

// Device buffers and launch shape of a batch.
struct BatchState {
  int32_t *queue = nullptr;
  unsigned *heads = nullptr;
  int32_t *rounds = nullptr;
  unsigned long long *stat = nullptr;
  int *err = nullptr;
  int q_block = 0, q_wave = -1, q_quad = -1;  // shape the uploaded queue was built for
  int n_big = 0, n_quad = 0, cap_big = 0, cap_quad = 0, cap_wave = 0;
  bool has_cfg = false;          // shape fixed by cc_batch_set_config / cc_batch_autotune
  cc_batch_config cfg{};
};

// Size class of a batch: log2 buckets of (graphs, largest graph, median graph).
using SizeClass = std::tuple<int, int, int, int>;
std::map<SizeClass, cc_batch_config> g_tuned;
std::mutex g_tuned_mu;

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
  // single graphs: internal renumbering (hubs first) and the renumbered CSR
  int32_t *perm = nullptr, *iperm = nullptr, *rcol = nullptr;
  int64_t *roff = nullptr;
  int64_t max_deg = 0;
  int64_t low_start = 0;       // single graphs: internal ids >= low_start have degree < DSW,
  int64_t iso_start = 0;       // and those >= iso_start degree 0
  int64_t n_hi = 0;            // vertices with degree >= DSW
  int32_t *lvl_init = nullptr; // device: initial bound buckets
  int64_t *lvl_off = nullptr;  // device [NLVL+1]
  unsigned *lvl_cnt0 = nullptr;  // device [NLVL]: initial entries per level
  int64_t lvl_total = 0;
  std::vector<int64_t> h_vtx_ptr;
  std::vector<int64_t> m_per_graph;
  Workspace ws;
  BatchState bs;
};

namespace {

void free_ws(Workspace &w) {
  void *ptrs[] = {w.rank, w.lab, w.ub, w.unc, w.state, w.flag, w.alist, w.clist, w.nlist, w.blist,
                  w.awork, w.cwork, w.rlist, w.xlist, w.rwork, w.xwork, w.racc, w.lvl, w.hist, w.plist, w.pwork,
                  w.cedge, w.tstat, w.ctrl, w.trace, w.order_buf, w.label_buf, w.sched, w.mlp, w.ainfo, w.cinfo,
                  w.iorder, w.cost_size, w.cost_acc, w.dev_err, w.bpos, w.bpend, w.bdec, w.bdep, w.bq, w.bradj, w.omap_buf, w.ccol, w.cend};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (w.host_flags) (void)hipHostFree(w.host_flags);
  if (w.progress) (void)hipHostFree(w.progress);
  for (RoundGraph &g : w.graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (w.cap) (void)hipStreamDestroy(w.cap);
  w = Workspace();
}

void free_graph(cc_graph *g) {
  if (!g) return;
  free_ws(g->ws);
  {
    BatchState &b = g->bs;
    void *ptrs[] = {b.queue, b.heads, b.rounds, b.stat, b.err};
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
  }
  if (!g->borrowed) {
    if (g->off) (void)hipFree(g->off);
    if (g->col) (void)hipFree(g->col);
  }
  if (g->vtx_ptr) (void)hipFree(g->vtx_ptr);
  if (g->gid) (void)hipFree(g->gid);
  if (g->wall) (void)hipFree(g->wall);
  {
    void *ptrs[] = {g->perm, g->iperm, g->rcol, g->roff};
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
  }
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
  HIP_TRY(dalloc(&w.ainfo, n));
  HIP_TRY(dalloc(&w.cinfo, n));
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
  HIP_TRY(dalloc(&w.bpos, n));
  HIP_TRY(dalloc(&w.bpend, n));
  HIP_TRY(dalloc(&w.bdec, n));
  HIP_TRY(dalloc(&w.bdep, n + 1));
  HIP_TRY(dalloc(&w.bq, n));
  HIP_TRY(dalloc(&w.bradj, (size_t)w.cedge_cap));
  w.tstat_cap = n / TSEL + 4096 + 2;
  HIP_TRY(dalloc(&w.tstat, (size_t)w.tstat_cap));
  HIP_TRY(hipMemset(w.tstat, 0, sizeof(unsigned long long) * (size_t)w.tstat_cap));
  HIP_TRY(dalloc(&w.ctrl, 1));
  w.trace_cap = 1 << 16;
  HIP_TRY(dalloc(&w.trace, (size_t)w.trace_cap));
  HIP_TRY(dalloc(&w.order_buf, n));
  HIP_TRY(dalloc(&w.label_buf, n));
  HIP_TRY(dalloc(&w.iorder, n));
  if (order_map_applies(n)) {
    HIP_TRY(dalloc(&w.omap_buf, order_map_bytes(n)));
    w.omap = order_map_layout(n, w.omap_buf);
  }
  if (g->num_graphs == 1) {  // the round loop's compacted rows (written at its switch to exact degrees)
    HIP_TRY(dalloc(&w.ccol, (size_t)(g->nnz > 0 ? g->nnz : 1)));
    HIP_TRY(dalloc(&w.cend, n));
  }
  HIP_TRY(dalloc(&w.mlp, CC_MLP_PARAMS));
  HIP_TRY(dalloc(&w.cost_size, n));
  HIP_TRY(dalloc(&w.cost_acc, 2 * (size_t)g->num_graphs));
  HIP_TRY(dalloc(&w.dev_err, 1));
  HIP_TRY(hipHostMalloc((void **)&w.host_flags, 8 * sizeof(int), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void **)&w.progress, sizeof(unsigned long long), hipHostMallocCoherent | hipHostMallocMapped));
  HIP_TRY(hipHostGetDevicePointer((void **)&w.progress_dev, w.progress, 0));
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

int32_t run_batch(cc_graph *g, int algo, const int32_t *order, double eps, int32_t *labels, cc_run_stats *stats,
                  uint32_t flags, hipStream_t s);

// Rounds per queued group.  Small enough that a finished run leaves little
// behind it, large enough that the host stays ahead of the device.
constexpr int64_t kRoundGroup = 4;

// Queues k rounds on s as one graph launch: the round's kernels are captured
// once per (arguments, phase, k) and replayed; the host then issues one call
// per group instead of ~16 launches per round.
int32_t launch_rounds(Workspace &ws, const Ws &w, const LaunchShape &ls, int64_t k, hipStream_t s) {
  for (RoundGraph &g : ws.graphs)
    if (g.k == k && g.exact == ls.exact_seen && std::memcmp(g.key, &w, sizeof(Ws)) == 0) {
      HIP_TRY(hipGraphLaunch(g.exec, s));
      return CC_OK;
    }
  if (!ws.cap) HIP_TRY(hipStreamCreateWithFlags(&ws.cap, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(ws.cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int64_t r = 0; r < k && e == hipSuccess; r++) e = launch_round(w, ws.cap, ls);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(ws.cap, &graph);
  if (e == hipSuccess) e = e2;
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  HIP_TRY(e);
  if (ws.graphs.size() >= 24) {  // keep the cache small: drop the oldest
    (void)hipGraphExecDestroy(ws.graphs.front().exec);
    ws.graphs.erase(ws.graphs.begin());
  }
  RoundGraph rg;
  std::memcpy(rg.key, &w, sizeof(Ws));
  rg.exact = ls.exact_seen;
  rg.k = k;
  rg.exec = exec;
  ws.graphs.push_back(rg);
  HIP_TRY(hipGraphLaunch(exec, s));
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
  if (stats && stats->max_rounds < 0) return fail(CC_ERR_INVALID_ARG, "stats->max_rounds must be >= 0");
  if (stats && stats->fault_round < 0) return fail(CC_ERR_INVALID_ARG, "stats->fault_round must be >= 0");
  if (stats && stats->max_rounds > 0 && g->num_graphs != 1)
    return fail(CC_ERR_INVALID_ARG, "max_rounds applies to single graphs only");
  if (stats && stats->fault_round > 0 && g->num_graphs != 1)
    return fail(CC_ERR_INVALID_ARG, "fault_round applies to single graphs only");
  if (g->num_graphs != 1) return run_batch(g, algo, order, eps, labels, stats, flags, s);
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
      if (stats->graph_rounds) stats->graph_rounds[0] = 0;
    }
    return CC_OK;
  }

  const int32_t *d_order = order;
  if (!(flags & CC_INPUT_ON_DEVICE)) {
    HIP_TRY(hipMemcpyAsync(ws.order_buf, order, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    d_order = ws.order_buf;
  }
  auto upload_sched = [&](const std::vector<int64_t> &v) -> int32_t {
    if ((int64_t)v.size() > ws.sched_cap) {
      if (ws.sched) HIP_TRY(hipFree(ws.sched));
      ws.sched = nullptr;
      ws.sched_cap = 0;
      HIP_TRY(dalloc(&ws.sched, v.size()));
      ws.sched_cap = (int64_t)v.size();
    }
    HIP_TRY(hipMemcpyAsync(ws.sched, v.data(), sizeof(int64_t) * v.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // v is pageable host memory the caller may free
    return CC_OK;
  };
  int64_t bin_period = 1;
  if (pol.kind == CC_EPS_TRACE && !pol.sched.empty()) {
    ws.sched_key = SchedKey();
    if (int32_t rc = upload_sched(pol.sched)) return rc;
  } else if (pol.kind == CC_EPS_BINOMIAL) {
    // the practical schedule depends on (n, Delta_0, eps, delta, seed) only
    SchedKey key{true, n, g->max_deg, eps, pol.bin_delta, pol.bin_seed};
    bin_period = halving_period(n, g->max_deg, eps, pol.bin_delta);
    if (!(ws.sched_key == key)) {
      std::vector<int64_t> bs;
      binomial_schedule(n, g->max_deg, eps, pol.bin_delta, pol.bin_seed, &bs);
      ws.sched_key = SchedKey();
      if (int32_t rc = upload_sched(bs)) return rc;
      ws.sched_key = key;
      ws.sched_len = (int64_t)bs.size();
    }
  }
  if (pol.kind == CC_EPS_LEARNED)
    HIP_TRY(hipMemcpyAsync(ws.mlp, pol.mlp.data(), sizeof(float) * CC_MLP_PARAMS, hipMemcpyHostToDevice, s));

  Ws w;
  std::memset(&w, 0, sizeof(w));  // the bytes (padding included) key the captured round graphs
  w.off = g->roff;
  w.rend = g->roff + 1;
  w.col = g->rcol;
  w.xcol = ws.ccol;
  w.xend = ws.cend;
  w.n = n;
  w.order = ws.iorder;
  w.iorder = ws.iorder;
  w.order_in = d_order;
  w.perm = g->perm;
  w.iperm = g->iperm;
  w.order_mapped = ws.omap_buf != nullptr;
  w.max_deg = g->max_deg;
  w.low_start = g->low_start;
  w.iso_start = g->iso_start;
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
  w.ainfo = ws.ainfo;
  w.cinfo = ws.cinfo;
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
  w.bpos = ws.bpos;
  w.bpend = ws.bpend;
  w.bdec = ws.bdec;
  w.bdep = ws.bdep;
  w.bq = ws.bq;
  w.bradj = ws.bradj;
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
  w.sched_len = pol.kind == CC_EPS_TRACE ? (int64_t)pol.sched.size() : pol.kind == CC_EPS_BINOMIAL ? ws.sched_len : 0;
  w.bin_period = bin_period;
  w.mlp = ws.mlp;
  w.eps_min = (float)pol.eps_min;
  w.eps_max = (float)pol.eps_max;
  w.max_rounds = stats ? stats->max_rounds : 0;
  w.fault_round = stats ? stats->fault_round : 0;
  w.progress = ws.progress_dev;

  // init.  The permutation check needs no host round trip: an entry out of
  // range is never used as an index, and a failed check sets the device
  // error, which ends the run in its first k_close; every later kernel of
  // the call then returns at once.
  __atomic_store_n(ws.progress, 0ull, __ATOMIC_RELEASE);  // nothing of this handle is in flight
  HIP_TRY(hipMemsetAsync(ws.ctrl, 0, sizeof(Ctrl), s));
  if (w.order_mapped) {
    HIP_TRY(launch_order_map(ws.omap, d_order, g->perm, n, ws.iorder, ws.ctrl, s));
  } else {
    HIP_TRY(hipMemsetAsync(ws.state, 0, (size_t)n, s));  // k_check_order marks the vertices pi names
  }
  HIP_TRY(hipMemsetAsync(ws.hist, 0, sizeof(int) * (size_t)ws.hist_len, s));
  if (g->lvl_total > 0)
    HIP_TRY(hipMemcpyAsync(ws.lvl, g->lvl_init, sizeof(int32_t) * (size_t)g->lvl_total, hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_init(w, g->lvl_cnt0, s));

  LaunchShape ls{512, 1024, 512, 0, 0};
  int64_t launched = 0;
  // the fixed rule clusters a vertex every round; the practical schedule's
  // rounds may be empty, and it has as many as it drew
  const int64_t round_limit = pol.kind == CC_EPS_BINOMIAL ? std::max<int64_t>(n, w.sched_len) : n;
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
  // Two groups of rounds stay queued: while one runs, the host waits on the
  // progress word for the older one and queues the next.  The device never
  // idles on the host, and a finished run leaves at most one group and the
  // rest of the current one (all kernels return at once) behind it.
  if (int32_t rc = launch_rounds(ws, w, ls, kRoundGroup, s)) return rc;
  launched = kRoundGroup;
  for (;;) {
    const int64_t older = launched;
    if (int32_t rc = launch_rounds(ws, w, ls, kRoundGroup, s)) {
      (void)hipStreamSynchronize(s);  // nothing of this call may still write the progress word
      return rc;
    }
    launched += kRoundGroup;
    bool done = false;
    for (unsigned spin = 1;; spin++) {
      const unsigned long long p = __atomic_load_n(ws.progress, __ATOMIC_ACQUIRE);
      done = (p >> PROGRESS_DONE & 1) || (p >> PROGRESS_ERROR & 1);
      if (p >> PROGRESS_EXACT & 1) ls.exact_seen = 1;
      if (done || (int64_t)(p & 0xFFFFFFFFull) >= older) break;
      if (spin % 64 == 0) {
        const hipError_t q = hipStreamQuery(s);
        if (q != hipErrorNotReady) {  // drained: read the state itself
          HIP_TRY(q);
          Ctrl now;
          HIP_TRY(hipMemcpyAsync(&now, ws.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
          HIP_TRY(hipStreamSynchronize(s));
          done = now.done || now.error;
          if (now.phase == PHASE_EXACT) ls.exact_seen = 1;
          break;
        }
      }
      std::this_thread::yield();
    }
    if (done) break;
    if (launched > round_limit + 4 * kRoundGroup) {  // a backstop: the device stops a runaway loop itself
      (void)hipStreamSynchronize(s);
      return fail(CC_ERR_NO_PROGRESS, "round loop exceeded its round limit");
    }
  }
  HIP_TRY(hipEventRecord(ev1, s));
  Ctrl hc;
  HIP_TRY(hipMemcpyAsync(&hc, ws.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  // labels go to the workspace first and reach the caller only on success,
  // so a failed run leaves the caller's buffer untouched
  HIP_TRY(launch_finalize(w, ws.label_buf, s));
  HIP_TRY(hipMemcpyAsync(ws.host_flags, &ws.ctrl->error, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hc.error) {
    const int e = hc.error;
    if (e == ERR_PERM) return fail(CC_ERR_NOT_PERMUTATION, "order is not a permutation of 0..n-1");
    if (e == ERR_NO_PROGRESS) return fail(CC_ERR_NO_PROGRESS, "round loop made no progress");
    if (e == ERR_OVERFLOW) return fail(CC_ERR_DEVICE, "a device work list overflowed");
    if (e == ERR_INJECTED) return fail(CC_ERR_DEVICE, "device error injected by stats->fault_round");
    return fail(CC_ERR_DEVICE, "device error " + std::to_string(e) + " in the round loop");
  }
  if (ws.host_flags[0]) return fail(CC_ERR_DEVICE, "device error " + std::to_string(ws.host_flags[0]) + " while finishing");
  HIP_TRY(hipMemcpyAsync(labels, ws.label_buf, sizeof(int32_t) * (size_t)n,
                         (flags & CC_OUTPUT_ON_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (stats) {
    stats->rounds = hc.round;
    if (stats->graph_rounds) stats->graph_rounds[0] = (int32_t)hc.round;
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

// ------------------------------------------------------- asynchronous runs

int32_t run_async(cc_graph *g, int algo, const int32_t *order, int32_t *labels, cc_run_stats *stats, uint32_t flags,
                  hipStream_t s) {
  if (!g) return fail(CC_ERR_INVALID_ARG, "graph handle is NULL");
  if (!order || !labels) return fail(CC_ERR_INVALID_ARG, "order and labels must not be NULL");
  if (flags & ~(uint32_t)(CC_INPUT_ON_DEVICE | CC_OUTPUT_ON_DEVICE))
    return fail(CC_ERR_INVALID_ARG, "unknown flag for a run");
  if (g->num_graphs != 1) return fail(CC_ERR_INVALID_ARG, "the asynchronous variants take single graphs");
  if (stats && (stats->max_rounds != 0 || stats->fault_round != 0))
    return fail(CC_ERR_INVALID_ARG, "max_rounds and fault_round apply to the round loop only");
  if (stats && (stats->async_waves < 0 || stats->async_waves > (1 << 20)))
    return fail(CC_ERR_INVALID_ARG, "stats->async_waves must lie in [0, 2^20]");
  if (int32_t rc = ensure_ws(g)) return rc;
  Workspace &ws = g->ws;
  const int64_t n = g->n;
  if (n == 0) {
    if (stats) std::memset(stats, 0, offsetof(cc_run_stats, trace));
    return CC_OK;
  }
  const int32_t *d_order = order;
  if (!(flags & CC_INPUT_ON_DEVICE)) {
    HIP_TRY(hipMemcpyAsync(ws.order_buf, order, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    d_order = ws.order_buf;
  }
  HIP_TRY(hipMemsetAsync(ws.ctrl, 0, sizeof(Ctrl), s));
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
  // the long-row claim list borrows two vertex lists of the round loop
  AsyncArgs a{g->roff, g->rcol, n, g->iso_start, ws.iorder, ws.rank, ws.lab, ws.ctrl, ws.xlist, ws.plist, n};
  // labels reach the caller only on success
  HIP_TRY(launch_async(a, algo, d_order, g->perm, ws.iorder, ws.label_buf, stats ? (int)stats->async_waves : 0, s,
                       ev0, ev1, ws.omap_buf ? &ws.omap : nullptr));
  Ctrl hc;
  HIP_TRY(hipMemcpyAsync(&hc, ws.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hc.error == ERR_PERM) return fail(CC_ERR_NOT_PERMUTATION, "order is not a permutation of 0..n-1");
  if (hc.error == ERR_NO_PROGRESS) return fail(CC_ERR_NO_PROGRESS, "a bounded wait for an earlier vertex expired");
  if (hc.error) return fail(CC_ERR_DEVICE, "device error " + std::to_string(hc.error) + " in the asynchronous run");
  HIP_TRY(hipMemcpyAsync(labels, ws.label_buf, sizeof(int32_t) * (size_t)n,
                         (flags & CC_OUTPUT_ON_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (stats) {
    unsigned long long walked = 0, claimed = 0, atoms = 0;
    for (int i = 0; i < 64; i++) {
      walked += hc.spread_lone[i];
      claimed += hc.x_low[i];
      atoms += hc.spread_atom[i];
    }
    stats->rounds = 0;
    stats->scanned_elect = (int64_t)walked;
    stats->scanned_claim = (int64_t)claimed;
    stats->scanned_peel = 0;
    stats->scanned_delta = 0;
    stats->blocked = 0;
    stats->atomics = (int64_t)atoms;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
    stats->loop_ms = ms;
    stats->policy_fallback = 0;
    stats->truncated = 0;
    if (stats->graph_rounds) stats->graph_rounds[0] = 0;
  }
  return CC_OK;
}

// ------------------------------------------------------------------ batches

int ilog2_ceil(int64_t x) {
  int k = 0;
  while (((int64_t)1 << k) < x) k++;
  return k;
}

int64_t graph_n(const cc_graph *g, int32_t i) { return g->h_vtx_ptr[(size_t)i + 1] - g->h_vtx_ptr[(size_t)i]; }

int32_t device_arch(int *arch_id, int *max_lds) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t p;
  HIP_TRY(hipGetDeviceProperties(&p, dev));
  *arch_id = p.major * 100 + p.minor * 10;
  *max_lds = (int)p.sharedMemPerBlock;
  return CC_OK;
}

SizeClass size_class(const cc_graph *g, int arch) {
  std::vector<int64_t> ns((size_t)g->num_graphs);
  for (int32_t i = 0; i < g->num_graphs; i++) ns[(size_t)i] = graph_n(g, i);
  std::sort(ns.begin(), ns.end());
  const int64_t mx = ns.empty() ? 0 : ns.back(), med = ns.empty() ? 0 : ns[ns.size() / 2];
  return SizeClass{arch, ilog2_ceil(g->num_graphs), ilog2_ceil(mx + 1), ilog2_ceil(med + 1)};
}

// Tier of a graph under a shape: 0 workgroup, 1 sub-group of 4 waves, 2 wave.
int tier_of(int64_t n, const cc_batch_config &c) {
  if (n <= c.wave_max_n) return 2;
  if (c.block > 256 && n <= c.quad_max_n) return 1;
  return 0;
}

// LDS (bytes of dynamic shared memory) a shape needs for this batch; sets the
// slot capacities: the largest graph of each tier.
size_t shape_lds(const cc_graph *g, const cc_batch_config &c, int *cap_big, int *cap_quad, int *cap_wave, int *n_big,
                 int *n_quad) {
  int cap[3] = {0, 0, 0}, cnt[3] = {0, 0, 0};
  for (int32_t i = 0; i < g->num_graphs; i++) {
    const int n = (int)graph_n(g, i);
    const int t = tier_of(n, c);
    cap[t] = std::max(cap[t], n);
    cnt[t]++;
  }
  if (cap_big) *cap_big = cap[0];
  if (cap_quad) *cap_quad = cap[1];
  if (cap_wave) *cap_wave = cap[2];
  if (n_big) *n_big = cnt[0];
  if (n_quad) *n_quad = cnt[1];
  return batched_lds_bytes(c.block, cap[0], cap[1], cap[2]);
}

// Static LDS of the batched kernel (graph id, scan scratch, 256 B of window
// scratch per wave), with slack.
constexpr int kBatchStaticLds = 4608;

int32_t check_shape(const cc_graph *g, const cc_batch_config &c) {
  if (c.block != 256 && c.block != 512 && c.block != 1024)
    return fail(CC_ERR_INVALID_ARG, "batch block must be 256, 512 or 1024");
  if (c.wave_max_n < 0 || c.quad_max_n < 0) return fail(CC_ERR_INVALID_ARG, "wave_max_n and quad_max_n must be >= 0");
  if (c.reserved != 0) return fail(CC_ERR_INVALID_ARG, "cc_batch_config.reserved must be 0");
  int arch = 0, max_lds = 0;
  if (int32_t rc = device_arch(&arch, &max_lds)) return rc;
  const size_t lds = shape_lds(g, c, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (lds + kBatchStaticLds > (size_t)max_lds)
    return fail(CC_ERR_INVALID_ARG, "batch shape needs " + std::to_string(lds) + " B of LDS per workgroup; the device has " +
                                        std::to_string(max_lds));
  return CC_OK;
}

cc_batch_config default_shape(const cc_graph *g) {
  // one wave per graph while four wave slots fit beside the largest graph's slot
  cc_batch_config c{256, 0, 0, 0, 0.0};
  int64_t mx = 0;
  for (int32_t i = 0; i < g->num_graphs; i++) mx = std::max(mx, graph_n(g, i));
  c.wave_max_n = (int)std::min<int64_t>(512, std::max<int64_t>(64, mx / 4));
  return c;
}

int32_t ensure_batch(cc_graph *g) {
  BatchState &b = g->bs;
  if (b.queue) return CC_OK;
  HIP_TRY(dalloc(&b.queue, (size_t)g->num_graphs));
  HIP_TRY(dalloc(&b.heads, 3));
  HIP_TRY(dalloc(&b.rounds, (size_t)g->num_graphs));
  HIP_TRY(dalloc(&b.stat, 4));
  HIP_TRY(dalloc(&b.err, 1));
  return CC_OK;
}

// Queue of graph ids: the workgroup tier, then the sub-group tier, then the
// wave tier; each part in decreasing order of work (entries + vertices), so
// the persistent groups finish together (longest-processing-time-first).
int32_t build_queue(cc_graph *g, const cc_batch_config &c, hipStream_t s) {
  BatchState &b = g->bs;
  if (b.q_block == c.block && b.q_wave == c.wave_max_n && b.q_quad == c.quad_max_n) return CC_OK;
  std::vector<int32_t> part[3];
  for (int32_t i = 0; i < g->num_graphs; i++) part[tier_of(graph_n(g, i), c)].push_back(i);
  auto work = [&](int32_t i) { return 2 * g->m_per_graph[(size_t)i] + graph_n(g, i); };
  auto by_work = [&](int32_t x, int32_t y) { return work(x) != work(y) ? work(x) > work(y) : x < y; };
  std::vector<int32_t> q;
  for (auto &p : part) {
    std::sort(p.begin(), p.end(), by_work);
    q.insert(q.end(), p.begin(), p.end());
  }
  HIP_TRY(hipMemcpyAsync(b.queue, q.data(), sizeof(int32_t) * q.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  shape_lds(g, c, &b.cap_big, &b.cap_quad, &b.cap_wave, &b.n_big, &b.n_quad);
  b.q_block = c.block;
  b.q_wave = c.wave_max_n;
  b.q_quad = c.quad_max_n;
  return CC_OK;
}

// One launch over the whole batch; d_order and d_labels are device buffers.
int32_t launch_batch(cc_graph *g, int algo, const int32_t *d_order, int64_t eps_q, int32_t *d_labels,
                     const cc_batch_config &c, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  BatchState &b = g->bs;
  if (int32_t rc = build_queue(g, c, s)) return rc;
  const size_t lds = batched_lds_bytes(c.block, b.cap_big, b.cap_quad, b.cap_wave);
  int grid = 0;
  HIP_TRY(batched_max_grid(c.block, lds, &grid));
  if (grid < 1) return fail(CC_ERR_DEVICE, "batched kernel does not fit on a compute unit");
  const int waves = c.block / 64, quads = c.block / 256;
  const int64_t nsmall = g->num_graphs - b.n_big - b.n_quad;
  const int64_t need =
      std::max<int64_t>(1, b.n_big + (b.n_quad + quads - 1) / quads + (nsmall + waves - 1) / waves);
  if (need < grid) grid = (int)need;
  HIP_TRY(hipMemsetAsync(b.heads, 0, 3 * sizeof(unsigned), s));
  HIP_TRY(hipMemsetAsync(b.stat, 0, 4 * sizeof(unsigned long long), s));
  HIP_TRY(hipMemsetAsync(b.err, 0, sizeof(int), s));
  BatchLaunch bl{g->off, g->col, g->vtx_ptr, d_order, d_labels, b.queue, b.n_big, b.n_quad, g->num_graphs,
                 b.cap_big, b.cap_quad, b.cap_wave, b.heads, b.rounds, b.stat, b.err, algo, eps_q, c.block, grid};
  if (ev0) HIP_TRY(hipEventRecord(ev0, s));
  HIP_TRY(launch_batched(bl, s));
  if (ev1) HIP_TRY(hipEventRecord(ev1, s));
  return CC_OK;
}

int32_t batch_error(int e) {
  if (e == ERR_PERM) return fail(CC_ERR_NOT_PERMUTATION, "order of a graph is not a permutation of 0..n_g-1");
  if (e == ERR_NO_PROGRESS) return fail(CC_ERR_NO_PROGRESS, "a graph's round loop made no progress");
  return fail(CC_ERR_DEVICE, "device error " + std::to_string(e) + " in the batched loop");
}

int32_t batch_prepare(cc_graph *g, const int32_t *order, double eps, uint32_t flags, hipStream_t s,
                      const int32_t **d_order, int64_t *eps_q) {
  if (!(eps > 0.0) || !(eps <= 1000.0) || !std::isfinite(eps))
    return fail(CC_ERR_INVALID_ARG, "eps must lie in (0, 1000]");
  {
    std::lock_guard<std::mutex> lk(g_policy_mu);
    if (g_policy.kind != CC_EPS_FIXED)
      return fail(CC_ERR_POLICY, "batches use the fixed eps rule; set CC_EPS_FIXED first");
  }
  for (int32_t i = 0; i < g->num_graphs; i++)
    if (graph_n(g, i) > CC_BATCH_MAX_N)
      return fail(CC_ERR_INVALID_ARG, "graph " + std::to_string(i) + " of the batch has more than CC_BATCH_MAX_N vertices");
  if (int32_t rc = ensure_ws(g)) return rc;
  if (int32_t rc = ensure_batch(g)) return rc;
  *d_order = order;
  if (!(flags & CC_INPUT_ON_DEVICE)) {
    HIP_TRY(hipMemcpyAsync(g->ws.order_buf, order, sizeof(int32_t) * (size_t)g->n, hipMemcpyHostToDevice, s));
    *d_order = g->ws.order_buf;
  }
  *eps_q = (int64_t)(eps * 1e6 + 0.5);
  return CC_OK;
}

int32_t run_batch(cc_graph *g, int algo, const int32_t *order, double eps, int32_t *labels, cc_run_stats *stats,
                  uint32_t flags, hipStream_t s) {
  const int32_t *d_order = nullptr;
  int64_t eps_q = 0;
  if (int32_t rc = batch_prepare(g, order, eps, flags, s, &d_order, &eps_q)) return rc;
  BatchState &b = g->bs;
  cc_batch_config c = b.cfg;
  if (!b.has_cfg) {
    int arch = 0, max_lds = 0;
    if (int32_t rc = device_arch(&arch, &max_lds)) return rc;
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    auto it = g_tuned.find(size_class(g, arch));
    c = it != g_tuned.end() ? it->second : default_shape(g);
  }
  if (int32_t rc = check_shape(g, c)) return rc;
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
  // labels go to the workspace first, so a failing graph leaves the caller's untouched
  if (int32_t rc = launch_batch(g, algo, d_order, eps_q, g->ws.label_buf, c, s, ev0, ev1)) return rc;
  int herr = 0;
  unsigned long long hst[4];
  HIP_TRY(hipMemcpyAsync(&herr, b.err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hst, b.stat, sizeof(hst), hipMemcpyDeviceToHost, s));
  std::vector<int32_t> rounds((size_t)g->num_graphs);
  HIP_TRY(hipMemcpyAsync(rounds.data(), b.rounds, sizeof(int32_t) * rounds.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (herr) return batch_error(herr);
  HIP_TRY(hipMemcpyAsync(labels, g->ws.label_buf, sizeof(int32_t) * (size_t)g->n,
                         (flags & CC_OUTPUT_ON_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (stats) {
    int64_t mx = 0;
    for (int32_t r : rounds) mx = std::max<int64_t>(mx, r);
    stats->rounds = mx;
    stats->scanned_elect = (int64_t)hst[0];
    stats->scanned_claim = (int64_t)hst[1];
    stats->scanned_peel = (int64_t)hst[2];
    stats->scanned_delta = 0;
    stats->blocked = 0;
    stats->atomics = (int64_t)hst[3];
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
    stats->loop_ms = ms;
    stats->policy_fallback = 0;
    stats->truncated = 0;
    if (stats->graph_rounds) std::memcpy(stats->graph_rounds, rounds.data(), sizeof(int32_t) * rounds.size());
  }
  return CC_OK;
}

int32_t autotune_batch(cc_graph *g, int algo, const int32_t *order, double eps, uint32_t flags, hipStream_t s,
                       cc_batch_config *best) {
  const int32_t *d_order = nullptr;
  int64_t eps_q = 0;
  if (int32_t rc = batch_prepare(g, order, eps, flags, s, &d_order, &eps_q)) return rc;
  int arch = 0, max_lds = 0;
  if (int32_t rc = device_arch(&arch, &max_lds)) return rc;
  int64_t mx = 0;
  for (int32_t i = 0; i < g->num_graphs; i++) mx = std::max(mx, graph_n(g, i));
  static const int kWave[] = {0, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096, 7168};
  static const int kQuad[] = {0, 512, 768, 1024, 1280, 1536, 1792, 2048, 3072, 4096};
  static const int kBlock[] = {256, 512, 1024};
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
  cc_batch_config top{0, 0, 0, 0, 1e300};
  for (int blk : kBlock) {
    int prev_split = -1;
    for (int wv : kWave) {
      if (wv > 0 && wv / 2 >= mx) break;  // every graph already runs on a wave
      for (int qd : kQuad) {
        if (qd != 0 && (blk == 256 || qd <= wv)) continue;
        if (qd > 0 && qd / 2 >= mx) break;
        cc_batch_config c{blk, wv, qd, 0, 0.0};
        int cb = 0, cq = 0, cw = 0, nb = 0, nq = 0;
        const size_t lds = shape_lds(g, c, &cb, &cq, &cw, &nb, &nq);
        if (lds + kBatchStaticLds > (size_t)max_lds) continue;
        const int split = cw * 65536 + nq;  // same tiers as the previous candidate: skip
        if (qd == 0 && split == prev_split) continue;
        if (qd == 0) prev_split = split;
        double t = 1e300;
        for (int rep = 0; rep < 3; rep++) {
          if (int32_t rc = launch_batch(g, algo, d_order, eps_q, g->ws.label_buf, c, s, ev0, ev1)) return rc;
          int herr = 0;
          HIP_TRY(hipMemcpyAsync(&herr, g->bs.err, sizeof(int), hipMemcpyDeviceToHost, s));
          HIP_TRY(hipStreamSynchronize(s));
          if (herr) return batch_error(herr);
          float ms = 0.f;
          HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
          if (rep > 0) t = std::min(t, (double)ms);  // first run warms caches
        }
        if (t < top.ms) top = cc_batch_config{blk, wv, qd, 0, t};
      }
    }
  }
  if (top.block == 0) return fail(CC_ERR_INVALID_ARG, "no batch shape fits the device's LDS");
  g->bs.cfg = top;
  g->bs.has_cfg = true;
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned[size_class(g, arch)] = top;
  }
  if (best) *best = top;
  return CC_OK;
}

}  // namespace

extern "C" {

const char *cc_last_error(void) { return g_last_error.c_str(); }

int32_t cc_binomial_schedule(int64_t n, int64_t delta0, double eps, uint64_t seed, double delta, int64_t *out,
                             int64_t capacity, int64_t *rounds, int64_t *period) {
  g_last_error.clear();
  if (n < 0 || delta0 < 0) return fail(CC_ERR_INVALID_ARG, "n and delta0 must be >= 0");
  if (!(eps > 0.0) || !(eps <= 1000.0) || !std::isfinite(eps)) return fail(CC_ERR_INVALID_ARG, "eps must lie in (0, 1000]");
  if (!(delta > 0.0 && delta < 1.0)) return fail(CC_ERR_INVALID_ARG, "delta must lie in (0, 1)");
  if (capacity < 0 || (capacity > 0 && !out)) return fail(CC_ERR_INVALID_ARG, "out is NULL but capacity > 0");
  std::vector<int64_t> bs;
  binomial_schedule(n, delta0, eps, delta, seed, &bs);
  const int64_t k = std::min<int64_t>(capacity, (int64_t)bs.size());
  if (k > 0) std::memcpy(out, bs.data(), sizeof(int64_t) * (size_t)k);
  if (rounds) *rounds = (int64_t)bs.size();
  if (period) *period = halving_period(n, delta0, eps, delta);
  return CC_OK;
}

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
  if (herr == none && n_total > 0 && num_graphs == 1) {
    G_TRY(dalloc(&g->perm, (size_t)n_total));
    G_TRY(dalloc(&g->iperm, (size_t)n_total));
    G_TRY(dalloc(&g->roff, (size_t)n_total + 1));
    G_TRY(dalloc(&g->rcol, (size_t)nnz));
    unsigned *cnt = nullptr;
    int64_t *binoff = nullptr, *rdeg = nullptr, *bsum = nullptr;
    hipError_t re = dalloc(&cnt, 2 * (NLVL + 1));
    if (re == hipSuccess) re = dalloc(&binoff, NLVL + 1);
    if (re == hipSuccess) re = dalloc(&rdeg, (size_t)n_total);
    if (re == hipSuccess) re = dalloc(&bsum, (size_t)(n_total / (4 * BS) + 4));
    if (re == hipSuccess)
      re = launch_relabel(g->off, g->col, g->wall, n_total, cnt, binoff, g->perm, g->iperm, rdeg, g->roff, bsum,
                          g->rcol, &g->low_start, &g->iso_start, s);
    if (re == hipSuccess) re = hipStreamSynchronize(s);
    void *tmp[] = {cnt, binoff, rdeg, bsum};
    for (void *p : tmp)
      if (p) (void)hipFree(p);
    G_TRY(re);
  }
  if (herr == none && n_total > 0) {
    // bound buckets: capacity of level k = vertices of degree >= 2^k (internal ids)
    const int64_t *xoff = g->roff ? g->roff : g->off;
    unsigned *dcnt = nullptr;
    int *dmax = nullptr;
    G_TRY(dalloc(&dcnt, NLVL));
    G_TRY(dalloc(&dmax, 1));
    G_TRY(hipMemsetAsync(dcnt, 0, sizeof(unsigned) * NLVL, s));
    G_TRY(hipMemsetAsync(dmax, 0, sizeof(int), s));
    G_TRY(launch_level_count(xoff, n_total, dcnt, dmax, s));
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
    G_TRY(launch_level_fill(xoff, n_total, g->lvl_off, dcnt, g->lvl_init, s));
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

int32_t cc_c4_async(const cc_graph *g, const int32_t *order, int32_t *labels, cc_run_stats *stats, uint32_t flags,
                    void *stream) {
  g_last_error.clear();
  return run_async(const_cast<cc_graph *>(g), ALGO_C4, order, labels, stats, flags, (hipStream_t)stream);
}

int32_t cc_clusterwild_async(const cc_graph *g, const int32_t *order, int32_t *labels, cc_run_stats *stats,
                             uint32_t flags, void *stream) {
  g_last_error.clear();
  return run_async(const_cast<cc_graph *>(g), ALGO_CW, order, labels, stats, flags, (hipStream_t)stream);
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

int32_t cc_batch_set_config(cc_graph *g, const cc_batch_config *cfg) {
  g_last_error.clear();
  if (!g || !cfg) return fail(CC_ERR_INVALID_ARG, "graph handle and cfg must not be NULL");
  if (g->num_graphs < 2) return fail(CC_ERR_INVALID_ARG, "not a batch (num_graphs < 2)");
  if (int32_t rc = check_shape(g, *cfg)) return rc;
  g->bs.cfg = *cfg;
  g->bs.cfg.ms = 0.0;
  g->bs.has_cfg = true;
  return CC_OK;
}

int32_t cc_batch_autotune(cc_graph *g, int32_t algo, const int32_t *order, double eps, uint32_t flags, void *stream,
                          cc_batch_config *best) {
  g_last_error.clear();
  if (!g || !order) return fail(CC_ERR_INVALID_ARG, "graph handle and order must not be NULL");
  if (g->num_graphs < 2) return fail(CC_ERR_INVALID_ARG, "not a batch (num_graphs < 2)");
  if (algo != CC_ALGO_C4 && algo != CC_ALGO_CLUSTERWILD) return fail(CC_ERR_INVALID_ARG, "unknown algorithm");
  if (flags & ~(uint32_t)CC_INPUT_ON_DEVICE) return fail(CC_ERR_INVALID_ARG, "unknown flag for cc_batch_autotune");
  return autotune_batch(g, algo, order, eps, flags, (hipStream_t)stream, best);
}

int32_t cc_mlp_forward(const float *params, const float *x, int64_t n, float *y, void *stream) {
  g_last_error.clear();
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(CC_ERR_INVALID_ARG, "n must lie in [0, 2^31)");
  if (!params || (n > 0 && (!x || !y))) return fail(CC_ERR_INVALID_ARG, "params, x and y must not be NULL");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_mlp_forward(params, x, (int)n, y, s));
  HIP_TRY(hipStreamSynchronize(s));
  return CC_OK;
}

int32_t cc_mlp_train_step(float *params, float *adam_m, float *adam_v, const float *x, const float *target, int64_t n,
                          int64_t step, float lr, float *grad, float *loss, void *stream) {
  g_last_error.clear();
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(CC_ERR_INVALID_ARG, "n must lie in [0, 2^31)");
  if (!params || (n > 0 && (!x || !target))) return fail(CC_ERR_INVALID_ARG, "params, x and target must not be NULL");
  if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(CC_ERR_INVALID_ARG, "lr must be finite and >= 0");
  if (lr > 0.f && (!adam_m || !adam_v || step < 1))
    return fail(CC_ERR_INVALID_ARG, "an Adam step needs adam_m, adam_v and step >= 1");
  hipStream_t s = (hipStream_t)stream;
  const int nblk = mlp_grad_blocks((int)n);
  // partial gradient rows, one per workgroup; one buffer per device, kept for later calls
  static std::mutex mu;
  static std::map<int, float *> partial;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  float *&rows = partial[dev];
  if (!rows) HIP_TRY(dalloc(&rows, (size_t)1024 * 514));
  HIP_TRY(launch_mlp_train_step(params, adam_m, adam_v, x, target, (int)n, (long long)step, lr, rows, nblk, grad,
                                loss, s));
  HIP_TRY(hipStreamSynchronize(s));
  return CC_OK;
}

int32_t cc_mlp_train_step_noalloc(float *params, float *adam_m, float *adam_v, const float *x, const float *target,
                                  int64_t n, int64_t step, float lr, float *grad, float *loss, void *stream) {
  g_last_error.clear();
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(CC_ERR_INVALID_ARG, "n must lie in [0, 2^31)");
  if (!params || (n > 0 && (!x || !target))) return fail(CC_ERR_INVALID_ARG, "params, x and target must not be NULL");
  if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(CC_ERR_INVALID_ARG, "lr must be finite and >= 0");
  if (lr > 0.f && (!adam_m || !adam_v || step < 1))
    return fail(CC_ERR_INVALID_ARG, "an Adam step needs adam_m, adam_v and step >= 1");
  hipStream_t s = (hipStream_t)stream;
  const int nblk = mlp_grad_blocks((int)n);
  float *rows = nullptr;
  int cap = 0;
  HIP_TRY(mlp_scratch(&rows, &cap));  // the device's static buffer: no allocation
  if (nblk > cap)
    return fail(CC_ERR_INVALID_ARG, "the gradient needs " + std::to_string(nblk) + " partial rows; the static buffer holds " +
                                        std::to_string(cap));
  HIP_TRY(launch_mlp_train_step(params, adam_m, adam_v, x, target, (int)n, (long long)step, lr, rows, nblk, grad,
                                loss, s));
  HIP_TRY(hipStreamSynchronize(s));
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
  } else if (kind == CC_EPS_BINOMIAL) {
    if (!params || nbytes != sizeof(cc_binomial_params))
      return fail(CC_ERR_POLICY, "the binomial schedule needs a cc_binomial_params");
    const cc_binomial_params *bp = (const cc_binomial_params *)params;
    if (!(bp->delta > 0.0 && bp->delta < 1.0)) return fail(CC_ERR_POLICY, "delta must lie in (0, 1)");
    p.bin_seed = bp->seed;
    p.bin_delta = bp->delta;
  } else {
    return fail(CC_ERR_POLICY, "unknown policy kind");
  }
  std::lock_guard<std::mutex> lk(g_policy_mu);
  g_policy = p;
  return CC_OK;
}

}  // extern "C"
