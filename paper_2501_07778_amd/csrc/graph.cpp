// The batched hot step as one HIP graph: the launches of n independent
// y_i = round(A_i x_i) captured once, split over branches that share
// nothing (each branch its own workspace, its cases in sequence), and
// replayed by one hipGraphLaunch.  The step holds no host synchronisation
// (device-side ranks, kernel-argument rank uploads, the capacity of y
// checked at capture against the bound its ranks can reach), so the whole
// batch is one launch and the host only reads back ranks and norms.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "step.h"

struct qtt_graph {
  int n = 0;
  // one graph (branches as parallel paths) or one graph per branch
  std::vector<hipGraph_t> graph;
  std::vector<hipGraphExec_t> exec;
  // per-branch mode: the streams the branch graphs are replayed on, forked
  // from and joined back into the caller's stream by events
  std::vector<hipStream_t> st;
  std::vector<hipEvent_t> ev;
  std::vector<qtt_tt *> y;  // outputs, for the host ranks at collect
  int32_t *aux_rk = nullptr;
  double *aux_scal = nullptr;
  ~qtt_graph() {
    for (auto x : exec)
      if (x) (void)hipGraphExecDestroy(x);
    for (auto x : graph)
      if (x) (void)hipGraphDestroy(x);
    for (auto x : ev)
      if (x) (void)hipEventDestroy(x);
    for (auto x : st)
      if (x) (void)hipStreamDestroy(x);
  }
};

namespace qtt {
namespace {

constexpr size_t kRkStride = QTT_MAXD + 1;  // int32 per case

size_t aux_bytes_of(int n) {
  return ((sizeof(int32_t) * kRkStride * n + 255) & ~size_t(255)) + sizeof(double) * 2 * n;
}

// packed elements of y at the largest ranks the rounding can leave: the
// product ranks, capped by rmax when it is positive
int64_t y_bound(const qtt_tt *A, const qtt_tt *x, int32_t rmax) {
  const int D = A->ncores;
  std::vector<int64_t> b(D + 1);
  for (int k = 0; k <= D; ++k) {
    int64_t r = (int64_t)A->ranks[k] * x->ranks[k];
    b[k] = (rmax > 0 && r > rmax) ? rmax : r;
  }
  int64_t e = 0;
  for (int k = 0; k < D; ++k) e += b[k] * A->nrow[k] * b[k + 1];
  return e;
}

// the rounded train's ranks and (norm, squared error) into the case's
// slots of aux, and the ranks into y's device mirror when it has one
__global__ void k_step_result(const int *rk, int D, const double *scal, int *out_rk,
                              double *out_scal, int *d_ranks) {
  const int i = threadIdx.x;
  if (i <= D) {
    out_rk[i] = rk[i];
    if (d_ranks) d_ranks[i] = rk[i];
  }
  if (i < 2) out_scal[i] = scal[i];
}

hipError_t launch_step_result(const TTView &t, const double *scal, int32_t *out_rk,
                              double *out_scal, int32_t *d_ranks, hipStream_t s) {
  hipLaunchKernelGGL(k_step_result, dim3(1), dim3(64), 0, s, t.rk, t.D, scal, out_rk,
                     out_scal, d_ranks);
  return hipGetLastError();
}


}  // namespace
}  // namespace qtt

using namespace qtt;

extern "C" {

qtt_status qtt_matvec_round_graph_aux_bytes(int32_t n, size_t *bytes) {
  if (n < 1) return fail(QTT_E_INVAL, "n must be >= 1");
  if (!bytes) return fail(QTT_E_INVAL, "bytes is NULL");
  *bytes = aux_bytes_of(n);
  return QTT_OK;
}

qtt_status qtt_matvec_round_graph_create(int32_t n, const qtt_matvec_round_case *cases,
                                         int32_t nbranch, void *const *ws,
                                         const size_t *ws_bytes, void *aux, size_t aux_bytes,
                                         int32_t per_branch, qtt_graph **out) {
  qtt::clear_stale_error();
  if (!out) return fail(QTT_E_INVAL, "out is NULL");
  *out = nullptr;
  if (per_branch != 0 && per_branch != 1) return fail(QTT_E_INVAL, "per_branch must be 0 or 1");
  if (n < 1 || !cases) return fail(QTT_E_INVAL, "need n >= 1 cases");
  if (nbranch < 1 || nbranch > 64 || !ws || !ws_bytes)
    return fail(QTT_E_INVAL, "nbranch must be in 1..64 with a workspace each");
  for (int b = 0; b < nbranch; ++b)
    if (!ws[b]) return fail(QTT_E_INVAL, "NULL branch workspace");
  if (!aux || aux_bytes < aux_bytes_of(n) || ((uintptr_t)aux & 255))
    return fail(QTT_E_CAPACITY, "aux: need " + std::to_string(aux_bytes_of(n)) +
                                    " bytes, 256-byte aligned");
  if (ktimer_active())
    return fail(QTT_E_INVAL, "kernel timing is on: its event records cannot be captured");
  // every check of the eager step, and y's capacity against the ranks the
  // rounding can reach (the replay cannot stop to look at them)
  std::vector<size_t> need(n);
  for (int i = 0; i < n; ++i) {
    const qtt_matvec_round_case &c = cases[i];
    qtt_status st = check_matvec_round_args(c.A, c.x, c.y, c.compute, c.ell, c.eps);
    if (st != QTT_OK)
      return fail(st, "case " + std::to_string(i) + ": " + std::string(qtt_last_error()));
    const int64_t yb = y_bound(c.A, c.x, c.rmax);
    if (yb > c.y->capacity)
      return fail(QTT_E_CAPACITY, "case " + std::to_string(i) + ": y capacity " +
                                      std::to_string(c.y->capacity) + " < " +
                                      std::to_string(yb) + " (ranks capped by rmax)");
    if ((st = qtt_matvec_round_workspace(c.A, c.x, c.ell, &need[i])) != QTT_OK) return st;
  }
  // longest case first onto the least loaded branch; a branch's workspace
  // must hold the largest of its cases
  std::vector<int> order(n), branch(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return need[a] > need[b]; });
  std::vector<double> load(nbranch, 0.0);
  for (int i : order) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    branch[i] = b;
    load[b] += (double)need[i];
    if (need[i] > ws_bytes[b])
      return fail(QTT_E_CAPACITY, "branch workspace " + std::to_string(b) + ": " +
                                      std::to_string(ws_bytes[b]) + " < " +
                                      std::to_string(need[i]) + " bytes for case " +
                                      std::to_string(i));
  }
  int32_t *aux_rk = (int32_t *)aux;
  double *aux_scal = (double *)((char *)aux + ((sizeof(int32_t) * kRkStride * n + 255) &
                                               ~size_t(255)));
  // the cases of branch b, in order, enqueued on sb
  auto enqueue_branch = [&](int b, hipStream_t sb) -> qtt_status {
    for (int i : order) {
      if (branch[i] != b) continue;
      const qtt_matvec_round_case &c = cases[i];
      MatvecRoundPlan p;
      qtt_status r = enqueue_matvec_round(c.A, c.x, c.compute, c.ell, c.seed, c.eps, c.rmax,
                                          ws[b], ws_bytes[b], sb, p);
      if (r != QTT_OK) return r;
      QTT_HIP(launch_pack(p.t.v, (double *)c.y->data, sb));
      QTT_HIP(launch_step_result(p.t.v, p.w.scal, aux_rk + kRkStride * i, aux_scal + 2 * i,
                                 c.y->d_ranks, sb));
    }
    return QTT_OK;
  };
  // captures what body enqueues on s into an instantiated graph
  auto capture_into = [&](hipStream_t s, auto body, hipGraph_t &graph,
                          hipGraphExec_t &exec) -> qtt_status {
    QTT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const qtt_status cst = body();
    graph = nullptr;
    hipError_t ec = hipStreamEndCapture(s, &graph);
    if (cst != QTT_OK || ec != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      graph = nullptr;
      if (cst != QTT_OK) return cst;
      return fail(QTT_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    }
    ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ec != hipSuccess) {
      (void)hipGraphDestroy(graph);
      graph = nullptr;
      return fail(QTT_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ec));
    }
    return QTT_OK;
  };
  qtt_graph *g = new qtt_graph;
  g->n = n;
  g->aux_rk = aux_rk;
  g->aux_scal = aux_scal;
  g->y.resize(n);
  for (int i = 0; i < n; ++i) g->y[i] = cases[i].y;
  auto bail = [&](qtt_status st) {
    delete g;
    return st;
  };
  // one stream and event per branch, and one more for the origin
  g->st.resize(nbranch + 1, nullptr);
  g->ev.resize(nbranch + 1, nullptr);
  for (int b = 0; b <= nbranch; ++b) {
    if (hipStreamCreateWithFlags(&g->st[b], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev[b], hipEventDisableTiming) != hipSuccess)
      return bail(fail(QTT_E_HIP, "stream or event creation failed"));
  }
  if (per_branch) {
    // graph j holds the j-th branch that has cases (more branches than
    // cases leave some empty) and is replayed on stream j
    for (int b = 0; b < nbranch; ++b) {
      if (std::find(branch.begin(), branch.end(), b) == branch.end()) continue;
      const int j = (int)g->exec.size();
      g->graph.push_back(nullptr);
      g->exec.push_back(nullptr);
      qtt_status r = capture_into(g->st[j], [&]() { return enqueue_branch(b, g->st[j]); },
                                  g->graph[j], g->exec[j]);
      if (r != QTT_OK) return bail(r);
    }
  } else {
    // the origin stream forks to one stream per branch and joins them
    hipStream_t s0 = g->st[nbranch];
    auto body = [&]() -> qtt_status {
      QTT_HIP(hipEventRecord(g->ev[nbranch], s0));
      for (int b = 0; b < nbranch; ++b) {
        QTT_HIP(hipStreamWaitEvent(g->st[b], g->ev[nbranch], 0));
        qtt_status r = enqueue_branch(b, g->st[b]);
        if (r != QTT_OK) return r;
        QTT_HIP(hipEventRecord(g->ev[b], g->st[b]));
        QTT_HIP(hipStreamWaitEvent(s0, g->ev[b], 0));
      }
      return QTT_OK;
    };
    g->graph.resize(1, nullptr);
    g->exec.resize(1, nullptr);
    qtt_status r = capture_into(s0, body, g->graph[0], g->exec[0]);
    if (r != QTT_OK) return bail(r);
  }
  *out = g;
  return QTT_OK;
}

qtt_status qtt_matvec_round_graph_launch(qtt_graph *g, void *stream) {
  qtt::clear_stale_error();
  if (!g || g->exec.empty()) return fail(QTT_E_INVAL, "graph is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (g->exec.size() == 1) {
    QTT_HIP(hipGraphLaunch(g->exec[0], s));
    return QTT_OK;
  }
  // per-branch graphs: fork from the caller's stream, replay, join back
  hipEvent_t fork = g->ev.back();
  QTT_HIP(hipEventRecord(fork, s));
  for (size_t j = 0; j < g->exec.size(); ++j) {
    QTT_HIP(hipStreamWaitEvent(g->st[j], fork, 0));
    QTT_HIP(hipGraphLaunch(g->exec[j], g->st[j]));
    QTT_HIP(hipEventRecord(g->ev[j], g->st[j]));
    QTT_HIP(hipStreamWaitEvent(s, g->ev[j], 0));
  }
  return QTT_OK;
}

qtt_status qtt_matvec_round_graph_collect(qtt_graph *g, qtt_matvec_round_case *cases,
                                          void *stream) {
  qtt::clear_stale_error();
  if (!g || g->exec.empty()) return fail(QTT_E_INVAL, "graph is NULL");
  if (!cases) return fail(QTT_E_INVAL, "cases is NULL");
  const int n = g->n;
  std::vector<int32_t> rk(kRkStride * n);
  std::vector<double> sc(2 * n);
  hipStream_t s = (hipStream_t)stream;
  QTT_HIP(hipMemcpyAsync(rk.data(), g->aux_rk, sizeof(int32_t) * rk.size(),
                         hipMemcpyDeviceToHost, s));
  QTT_HIP(hipMemcpyAsync(sc.data(), g->aux_scal, sizeof(double) * sc.size(),
                         hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i) {
    qtt_tt *y = g->y[i];
    for (int k = 0; k <= y->ncores; ++k) y->ranks[k] = rk[kRkStride * i + k];
    cases[i].norm = sc[2 * i];
    cases[i].err = std::sqrt(sc[2 * i + 1] > 0.0 ? sc[2 * i + 1] : 0.0);
    cases[i].status = QTT_OK;
  }
  return QTT_OK;
}

qtt_status qtt_matvec_round_graph_destroy(qtt_graph *g) {
  delete g;
  return QTT_OK;
}

}  // extern "C"
