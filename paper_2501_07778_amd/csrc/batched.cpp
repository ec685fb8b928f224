// batched.cpp — many independent solves at once (load cases of the batched
// configuration): host workers feed the cases to qtt_solve on the cases'
// own streams, so several solves' small kernels run side by side on the
// 256 compute units; a self-written autotuner picks the concurrency.
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

namespace {

std::mutex g_tune_mu;
std::map<int, int> g_tuned;  // largest level (cores) of a batch -> concurrency

int batch_key(int32_t n, const qtt_solve_case *cases) {
  int key = 0;
  for (int i = 0; i < n; ++i)
    if (cases[i].K && cases[i].K->ncores > key) key = cases[i].K->ncores;
  return key;
}

qtt_status run_batch(int32_t n, qtt_solve_case *cases, int conc) {
  std::atomic<int> next{0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return qtt::fail(QTT_E_HIP, "hipGetDevice failed");
  auto worker = [&]() {
    // workers inherit the caller's device
    (void)hipSetDevice(dev);
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= n) break;
      qtt_solve_case &c = cases[i];
      c.status = qtt_solve(c.K, c.f, c.x0, c.opts, c.u, c.report, c.ws, c.ws_bytes, c.stream);
    }
  };
  const int nw = conc < n ? conc : n;
  std::vector<std::thread> pool;
  pool.reserve(nw);
  for (int w = 0; w < nw; ++w) pool.emplace_back(worker);
  for (auto &t : pool) t.join();
  for (int i = 0; i < n; ++i)
    if (cases[i].status != QTT_OK)
      return qtt::fail((qtt_status)cases[i].status,
                       "case " + std::to_string(i) + " failed with status " +
                           std::to_string(cases[i].status));
  return QTT_OK;
}

qtt_status check_cases(int32_t n, const qtt_solve_case *cases) {
  if (n < 0 || (n > 0 && !cases)) return qtt::fail(QTT_E_INVAL, "bad case array");
  for (int i = 0; i < n; ++i)
    if (!cases[i].K || !cases[i].f || !cases[i].opts || !cases[i].u || !cases[i].ws)
      return qtt::fail(QTT_E_INVAL, "case " + std::to_string(i) + " has a NULL field");
  return QTT_OK;
}

}  // namespace

extern "C" qtt_status qtt_solve_batched(int32_t n, qtt_solve_case *cases, int32_t concurrency) {
  qtt_status st = check_cases(n, cases);
  if (st != QTT_OK) return st;
  if (n == 0) return QTT_OK;
  int conc = concurrency;
  if (conc <= 0) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tuned.find(batch_key(n, cases));
    conc = it != g_tuned.end() ? it->second : 8;
  }
  if (conc > 64) conc = 64;
  return run_batch(n, cases, conc);
}

extern "C" qtt_status qtt_autotune_batched(int32_t n, qtt_solve_case *cases, int32_t *best,
                                           double *rates) {
  qtt_status st = check_cases(n, cases);
  if (st != QTT_OK) return st;
  if (n == 0) return qtt::fail(QTT_E_INVAL, "no cases to tune on");
  const int cand[6] = {1, 2, 4, 8, 16, 32};
  double best_rate = -1.0;
  int best_c = 1;
  for (int j = 0; j < 6; ++j) {
    const auto t0 = std::chrono::steady_clock::now();
    st = run_batch(n, cases, cand[j]);
    const double dt =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    // a case that stops at its sweep limit (QTT_E_NOCONV) is a finished
    // run for timing; any other failure ends the tuning
    if (st != QTT_OK && st != QTT_E_NOCONV) return st;
    int converged = 0;
    for (int i = 0; i < n; ++i) converged += cases[i].status == QTT_OK ? 1 : 0;
    const double rate = converged / (dt > 0.0 ? dt : 1e-9);
    if (rates) rates[j] = rate;
    if (rate > best_rate) {
      best_rate = rate;
      best_c = cand[j];
    }
  }
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned[batch_key(n, cases)] = best_c;
  }
  if (best) *best = best_c;
  // the cases hold the last run's results; report their aggregate status
  for (int i = 0; i < n; ++i)
    if (cases[i].status != QTT_OK)
      return qtt::fail((qtt_status)cases[i].status,
                       "case " + std::to_string(i) + " ended with status " +
                           std::to_string(cases[i].status) + " (tuning completed)");
  return QTT_OK;
}

extern "C" qtt_status qtt_matvec_round_batched(int32_t n, qtt_matvec_round_case *cases,
                                               int32_t nworkers, void *const *ws,
                                               const size_t *ws_bytes, void *const *streams) {
  if (n < 0 || (n > 0 && !cases)) return qtt::fail(QTT_E_INVAL, "bad case array");
  if (nworkers < 1 || nworkers > 64 || !ws || !ws_bytes || !streams)
    return qtt::fail(QTT_E_INVAL, "nworkers must be in 1..64 with a workspace and stream each");
  for (int w = 0; w < nworkers; ++w)
    if (!ws[w]) return qtt::fail(QTT_E_INVAL, "NULL worker workspace");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return qtt::fail(QTT_E_HIP, "hipGetDevice failed");
  std::atomic<int> next{0};
  auto worker = [&](int w) {
    (void)hipSetDevice(dev);
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= n) break;
      qtt_matvec_round_case &c = cases[i];
      c.status = qtt_matvec_round(c.A, c.x, c.y, c.compute, c.ell, c.seed, c.eps, c.rmax,
                                  &c.norm, &c.err, ws[w], ws_bytes[w], streams[w]);
    }
  };
  const int nw = nworkers < n ? nworkers : n;
  std::vector<std::thread> pool;
  for (int w = 0; w < nw; ++w) pool.emplace_back(worker, w);
  for (auto &t : pool) t.join();
  for (int i = 0; i < n; ++i)
    if (cases[i].status != QTT_OK)
      return qtt::fail((qtt_status)cases[i].status,
                       "case " + std::to_string(i) + " failed with status " +
                           std::to_string(cases[i].status));
  return QTT_OK;
}
