// capi.cpp — the extern "C" entry points for the tensor-train operations:
// argument validation, workspace carving and dispatch to the kernels.
#include <cmath>
#include <cstring>
#include <string>

#include "step.h"

namespace qtt {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

qtt_status fail(qtt_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

int64_t layout(TTView &v, int D, const int32_t *n, const int32_t *m,
               const std::vector<int> &caps) {
  v.D = D;
  int64_t off = 0;
  for (int k = 0; k < D; ++k) {
    v.n[k] = n[k];
    v.m[k] = m ? m[k] : 1;
    v.off[k] = off;
    off += (int64_t)caps[k] * v.n[k] * v.m[k] * caps[k + 1];
    off = (off + 31) & ~int64_t(31);  // 256-byte aligned slots
  }
  for (int k = 0; k <= D; ++k) v.cap[k] = caps[k];
  for (int k = D; k < QTT_MAXD; ++k) {
    v.n[k] = 1;
    v.m[k] = 1;
    v.off[k] = off;
  }
  return off;
}

std::vector<int> bounded_caps(int D, const int32_t *n, const int32_t *m,
                              int r) {
  std::vector<int> c(D + 1, 1);
  double left = 1.0;
  for (int k = 1; k < D; ++k) {
    left *= (double)n[k - 1] * (m ? m[k - 1] : 1);
    double right = 1.0;
    for (int l = k; l < D; ++l) right *= (double)n[l] * (m ? m[l] : 1);
    double b = left < right ? left : right;
    c[k] = (int)(b < r ? b : r);
  }
  return c;
}

bool arena_tt(Arena &ar, TTDesc &t, int D, const int32_t *n,
              const int32_t *m, const std::vector<int> &caps) {
  t.elems = layout(t.v, D, n, m, caps);
  t.v.data = (double *)ar.take(sizeof(double) * (t.elems > 0 ? t.elems : 1));
  t.v.rk = (int32_t *)ar.take(sizeof(int32_t) * (D + 1));
  return ar.ok();
}

// ---------------------------------------------------------------- checks
qtt_status check_tt(const qtt_tt *t, const char *name, bool need_ranks) {
  if (!t) return fail(QTT_E_INVAL, std::string(name) + " is NULL");
  if (t->dtype != QTT_F64)
    return fail(QTT_E_UNSUPPORTED, std::string(name) + ": storage dtype must be QTT_F64");
  if (t->ncores < 1 || t->ncores > QTT_MAX_CORES)
    return fail(QTT_E_INVAL, std::string(name) + ": ncores out of range");
  if (!t->nrow || !t->ranks)
    return fail(QTT_E_INVAL, std::string(name) + ": NULL nrow or ranks");
  for (int k = 0; k < t->ncores; ++k) {
    if (t->nrow[k] < 1 || t->nrow[k] > 64 || (t->ncol && (t->ncol[k] < 1 || t->ncol[k] > 64)))
      return fail(QTT_E_INVAL, std::string(name) + ": mode out of range");
  }
  if (need_ranks) {
    if (t->ranks[0] != 1 || t->ranks[t->ncores] != 1)
      return fail(QTT_E_SHAPE, std::string(name) + ": boundary ranks must be 1");
    for (int k = 1; k < t->ncores; ++k)
      if (t->ranks[k] < 1 || t->ranks[k] > (1 << 20))
        return fail(QTT_E_SHAPE, std::string(name) + ": rank out of range");
    int64_t need = 0;
    for (int k = 0; k < t->ncores; ++k)
      need += (int64_t)t->ranks[k] * t->nrow[k] * (t->ncol ? t->ncol[k] : 1) *
              t->ranks[k + 1];
    if (need > t->capacity)
      return fail(QTT_E_CAPACITY, std::string(name) + ": capacity " +
                                      std::to_string(t->capacity) + " < " +
                                      std::to_string(need));
    if (!t->data) return fail(QTT_E_INVAL, std::string(name) + ": NULL data");
  }
  return QTT_OK;
}

// the device mirror of a producer's ranks, when the caller keeps one
hipError_t publish_ranks(const qtt_tt *t, hipStream_t s) {
  if (!t || !t->d_ranks) return hipSuccess;
  return hipMemcpyAsync(t->d_ranks, t->ranks, sizeof(int32_t) * (t->ncores + 1),
                        hipMemcpyHostToDevice, s);
}

int64_t packed_elems(const qtt_tt *t) {
  int64_t e = 0;
  for (int k = 0; k < t->ncores; ++k)
    e += (int64_t)t->ranks[k] * t->nrow[k] * (t->ncol ? t->ncol[k] : 1) *
         t->ranks[k + 1];
  return e;
}

// A packed TT is a slotted TT whose caps are its ranks and whose slots
// have no gaps.
static void packed_view(const qtt_tt *t, TTView &v, int32_t *rk_dev) {
  v.D = t->ncores;
  int64_t off = 0;
  for (int k = 0; k < t->ncores; ++k) {
    v.n[k] = t->nrow[k];
    v.m[k] = t->ncol ? t->ncol[k] : 1;
    v.off[k] = off;
    off += (int64_t)t->ranks[k] * v.n[k] * v.m[k] * t->ranks[k + 1];
  }
  for (int k = 0; k <= t->ncores; ++k) v.cap[k] = t->ranks[k];
  for (int k = t->ncores; k < QTT_MAXD; ++k) {
    v.n[k] = 1;
    v.m[k] = 1;
    v.off[k] = off;
  }
  v.rk = rk_dev;
  v.data = t->data;
}

}  // namespace qtt

using namespace qtt;

extern "C" {

const char *qtt_last_error(void) { return g_last_error.c_str(); }

const char *qtt_version(void) { return "qtt-mi355x 0.1 (gfx950)"; }

qtt_status qtt_matvec(const qtt_tt *A, const qtt_tt *x, qtt_tt *y,
                      qtt_dtype compute, void *ws, size_t ws_bytes,
                      void *stream) {
  qtt::clear_stale_error();
  qtt_status st;
  if ((st = check_tt(A, "A", true)) != QTT_OK) return st;
  if ((st = check_tt(x, "x", true)) != QTT_OK) return st;
  if (!y || !y->ranks || !y->nrow || !y->data)
    return fail(QTT_E_INVAL, "y: NULL field");
  if (!A->ncol) return fail(QTT_E_INVAL, "A must be a matrix (ncol != NULL)");
  if (x->ncol) return fail(QTT_E_INVAL, "x must be a vector");
  if (A->ncores != x->ncores || y->ncores != A->ncores)
    return fail(QTT_E_SHAPE, "core counts differ");
  for (int k = 0; k < A->ncores; ++k) {
    if (A->ncol[k] != x->nrow[k]) return fail(QTT_E_SHAPE, "A column mode != x mode");
    if (y->nrow[k] != A->nrow[k]) return fail(QTT_E_SHAPE, "y mode != A row mode");
  }
  if (compute != QTT_F64 && compute != QTT_F32 && compute != QTT_BF16)
    return fail(QTT_E_INVAL, "bad compute dtype");
  const int D = A->ncores;
  for (int k = 0; k <= D; ++k) y->ranks[k] = A->ranks[k] * x->ranks[k];
  int64_t need = packed_elems(y);
  if (need > y->capacity)
    return fail(QTT_E_CAPACITY, "y: capacity " + std::to_string(y->capacity) +
                                    " < " + std::to_string(need));
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  int32_t *rk = (int32_t *)ar.take(sizeof(int32_t) * 3 * (QTT_MAXD + 1));
  if (!ar.ok() || !ws) return fail(QTT_E_CAPACITY, "workspace too small for qtt_matvec");
  TTView va, vx, vy;
  packed_view(A, va, rk);
  packed_view(x, vx, rk + (QTT_MAXD + 1));
  packed_view(y, vy, rk + 2 * (QTT_MAXD + 1));
  hipStream_t s = (hipStream_t)stream;
  QTT_HIP(upload_ranks(va, A->ranks, s));
  QTT_HIP(upload_ranks(vx, x->ranks, s));
  QTT_HIP(launch_matvec(va, vx, vy, compute, s));
  QTT_HIP(publish_ranks(y, s));
  return QTT_OK;
}

qtt_status qtt_round_workspace(const qtt_tt *x, int32_t rmax, size_t *bytes) {
  qtt_status st;
  if ((st = check_tt(x, "x", false)) != QTT_OK) return st;
  if (!bytes) return fail(QTT_E_INVAL, "bytes is NULL");
  (void)rmax;
  TTView v;
  packed_view(x, v, nullptr);
  Arena ar;
  ar.dry = true;
  TTDesc t;
  std::vector<int> caps(x->ranks, x->ranks + x->ncores + 1);
  arena_tt(ar, t, x->ncores, x->nrow, x->ncol, caps);
  RoundWs w;
  round_ws_take(ar, t.v, w);
  *bytes = ar.used + 256;
  return QTT_OK;
}

qtt_status qtt_round(qtt_tt *x, double eps, int32_t rmax, double *norm,
                     double *err, void *ws, size_t ws_bytes, void *stream) {
  qtt::clear_stale_error();
  qtt_status st;
  if ((st = check_tt(x, "x", true)) != QTT_OK) return st;
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(QTT_E_INVAL, "eps must be >= 0");
  size_t need = 0;
  qtt_round_workspace(x, rmax, &need);
  if (!ws || ws_bytes < need)
    return fail(QTT_E_CAPACITY, "workspace too small for qtt_round: need " +
                                    std::to_string(need));
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  TTDesc t;
  std::vector<int> caps(x->ranks, x->ranks + x->ncores + 1);
  arena_tt(ar, t, x->ncores, x->nrow, x->ncol, caps);
  RoundWs w;
  round_ws_take(ar, t.v, w);
  if (!ar.ok()) return fail(QTT_E_CAPACITY, "workspace too small for qtt_round");
  hipStream_t s = (hipStream_t)stream;
  // the packed layout is the slotted layout with caps = ranks, up to the
  // 256-byte slot alignment: copy core by core
  TTView pv;
  packed_view(x, pv, t.v.rk);
  QTT_HIP(upload_ranks(t.v, x->ranks, s));
  QTT_HIP(launch_unpack(x->data, t.v, s));
  QTT_HIP(round_tt(t.v, eps, rmax, w, s));
  QTT_HIP(launch_pack(t.v, x->data, s));
  int32_t rk_host[QTT_MAXD + 1];
  double scal[2];
  QTT_HIP(hipMemcpyAsync(rk_host, t.v.rk, sizeof(int32_t) * (x->ncores + 1),
                         hipMemcpyDeviceToHost, s));
  QTT_HIP(hipMemcpyAsync(scal, w.scal, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));
  for (int k = 0; k <= x->ncores; ++k) x->ranks[k] = rk_host[k];
  QTT_HIP(publish_ranks(x, s));
  if (norm) *norm = scal[0];
  if (err) *err = std::sqrt(scal[1] > 0.0 ? scal[1] : 0.0);
  return QTT_OK;
}

qtt_status qtt_round_sketch_workspace(const qtt_tt *x, int32_t ell, size_t *bytes) {
  qtt_status st;
  if ((st = check_tt(x, "x", true)) != QTT_OK) return st;
  if (x->ncol) return fail(QTT_E_INVAL, "x must be a vector");
  if (ell < 1 || ell > 512) return fail(QTT_E_INVAL, "ell must be in 1..512");
  if (!bytes) return fail(QTT_E_INVAL, "bytes is NULL");
  Arena ar;
  ar.dry = true;
  TTDesc t;
  std::vector<int> caps(x->ranks, x->ranks + x->ncores + 1);
  arena_tt(ar, t, x->ncores, x->nrow, x->ncol, caps);
  RoundWs w;
  round_ws_take(ar, t.v, w);
  ar.take(sizeof(double) * sketch_ws_elems(t.v, ell));
  *bytes = ar.used + 256;
  return QTT_OK;
}

qtt_status qtt_round_sketch(qtt_tt *x, int32_t ell, uint64_t seed, double eps, int32_t rmax,
                            double *norm, double *err, void *ws, size_t ws_bytes,
                            void *stream) {
  qtt::clear_stale_error();
  qtt_status st;
  if ((st = check_tt(x, "x", true)) != QTT_OK) return st;
  if (x->ncol) return fail(QTT_E_INVAL, "x must be a vector");
  if (ell < 1 || ell > 512) return fail(QTT_E_INVAL, "ell must be in 1..512");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(QTT_E_INVAL, "eps must be >= 0");
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  TTDesc t;
  std::vector<int> caps(x->ranks, x->ranks + x->ncores + 1);
  arena_tt(ar, t, x->ncores, x->nrow, x->ncol, caps);
  RoundWs w;
  round_ws_take(ar, t.v, w);
  double *sk = (double *)ar.take(sizeof(double) * sketch_ws_elems(t.v, ell));
  if (!ws || !ar.ok())
    return fail(QTT_E_CAPACITY, "workspace too small for qtt_round_sketch: need " +
                                    std::to_string(ar.used));
  hipStream_t s = (hipStream_t)stream;
  QTT_HIP(upload_ranks(t.v, x->ranks, s));
  QTT_HIP(launch_unpack(x->data, t.v, s));
  QTT_HIP(sketch_tt(t.v, ell, seed, 0, sk, s));
  QTT_HIP(round_tt(t.v, eps, rmax, w, s, true, ell));
  QTT_HIP(launch_pack(t.v, x->data, s));
  int32_t rk_host[QTT_MAXD + 1];
  double scal[2];
  QTT_HIP(hipMemcpyAsync(rk_host, t.v.rk, sizeof(int32_t) * (x->ncores + 1),
                         hipMemcpyDeviceToHost, s));
  QTT_HIP(hipMemcpyAsync(scal, w.scal, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));
  for (int k = 0; k <= x->ncores; ++k) x->ranks[k] = rk_host[k];
  QTT_HIP(publish_ranks(x, s));
  if (norm) *norm = scal[0];
  if (err) *err = std::sqrt(scal[1] > 0.0 ? scal[1] : 0.0);
  return QTT_OK;
}

// ---------------------------------------------------------------- fused step
static qtt_status check_matvec_args(const qtt_tt *A, const qtt_tt *x, qtt_dtype compute) {
  qtt_status st;
  if ((st = check_tt(A, "A", true)) != QTT_OK) return st;
  if ((st = check_tt(x, "x", true)) != QTT_OK) return st;
  if (!A->ncol) return fail(QTT_E_INVAL, "A must be a matrix (ncol != NULL)");
  if (x->ncol) return fail(QTT_E_INVAL, "x must be a vector");
  if (A->ncores != x->ncores) return fail(QTT_E_SHAPE, "core counts differ");
  for (int k = 0; k < A->ncores; ++k) {
    if (A->ncol[k] != x->nrow[k]) return fail(QTT_E_SHAPE, "A column mode != x mode");
  }
  if (compute != QTT_F64 && compute != QTT_F32 && compute != QTT_BF16)
    return fail(QTT_E_INVAL, "bad compute dtype");
  return QTT_OK;
}

// carve the product train (caps = product ranks) and the rounding and
// sketch workspaces
static bool carve_matvec_round(Arena &ar, const qtt_tt *A, const qtt_tt *x, int32_t ell,
                               TTDesc &t, RoundWs &w, double *&sk, int32_t *&rk) {
  const int D = A->ncores;
  std::vector<int> caps(D + 1);
  for (int k = 0; k <= D; ++k) caps[k] = A->ranks[k] * x->ranks[k];
  arena_tt(ar, t, D, A->nrow, nullptr, caps);
  round_ws_take(ar, t.v, w);
  sk = ell > 0 ? (double *)ar.take(sizeof(double) * sketch_ws_elems(t.v, ell)) : nullptr;
  rk = (int32_t *)ar.take(sizeof(int32_t) * 2 * (QTT_MAXD + 1));
  return ar.ok();
}

}  // extern "C"

qtt_status qtt::check_matvec_round_args(const qtt_tt *A, const qtt_tt *x, const qtt_tt *y,
                                   qtt_dtype compute, int32_t ell, double eps) {
  qtt_status st;
  if ((st = check_matvec_args(A, x, compute)) != QTT_OK) return st;
  if (!y || !y->ranks || !y->nrow || !y->data) return fail(QTT_E_INVAL, "y: NULL field");
  if (y->ncores != A->ncores || y->ncol) return fail(QTT_E_SHAPE, "y must be a vector like x");
  for (int k = 0; k < A->ncores; ++k)
    if (y->nrow[k] != A->nrow[k]) return fail(QTT_E_SHAPE, "y mode != A row mode");
  if (ell < 0 || ell > 512) return fail(QTT_E_INVAL, "ell must be in 0..512");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(QTT_E_INVAL, "eps must be >= 0");
  return QTT_OK;
}

qtt_status qtt::enqueue_matvec_round(const qtt_tt *A, const qtt_tt *x, qtt_dtype compute,
                                int32_t ell, uint64_t seed, double eps, int32_t rmax, void *ws,
                                size_t ws_bytes, hipStream_t s, MatvecRoundPlan &p) {
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  double *sk;
  int32_t *rk;
  if (!carve_matvec_round(ar, A, x, ell, p.t, p.w, sk, rk))
    return fail(QTT_E_CAPACITY, "workspace too small for qtt_matvec_round: need " +
                                    std::to_string(ar.used));
  TTView va, vx;
  packed_view(A, va, rk);
  packed_view(x, vx, rk + (QTT_MAXD + 1));
  QTT_HIP(upload_ranks(va, A->ranks, s));
  QTT_HIP(upload_ranks(vx, x->ranks, s));
  // the product goes straight into the slotted train (the kernel writes its
  // device ranks), then sketch and rounding work on it in place
  QTT_HIP(launch_matvec(va, vx, p.t.v, compute, s));
  if (ell > 0) {
    QTT_HIP(sketch_tt(p.t.v, ell, seed, 0, sk, s));
    QTT_HIP(round_tt(p.t.v, eps, rmax, p.w, s, true, ell));
  } else {
    QTT_HIP(round_tt(p.t.v, eps, rmax, p.w, s));
  }
  return QTT_OK;
}

extern "C" {

qtt_status qtt_matvec_round_workspace(const qtt_tt *A, const qtt_tt *x, int32_t ell,
                                      size_t *bytes) {
  qtt_status st;
  if ((st = check_matvec_args(A, x, QTT_F64)) != QTT_OK) return st;
  if (ell < 0 || ell > 512) return fail(QTT_E_INVAL, "ell must be in 0..512");
  if (!bytes) return fail(QTT_E_INVAL, "bytes is NULL");
  Arena ar;
  ar.dry = true;
  TTDesc t;
  RoundWs w;
  double *sk;
  int32_t *rk;
  carve_matvec_round(ar, A, x, ell, t, w, sk, rk);
  *bytes = ar.used + 256;
  return QTT_OK;
}

qtt_status qtt_matvec_round(const qtt_tt *A, const qtt_tt *x, qtt_tt *y, qtt_dtype compute,
                            int32_t ell, uint64_t seed, double eps, int32_t rmax, double *norm,
                            double *err, void *ws, size_t ws_bytes, void *stream) {
  qtt::clear_stale_error();
  qtt_status st;
  if ((st = check_matvec_round_args(A, x, y, compute, ell, eps)) != QTT_OK) return st;
  if (!ws) return fail(QTT_E_CAPACITY, "workspace is NULL");
  const int D = A->ncores;
  hipStream_t s = (hipStream_t)stream;
  MatvecRoundPlan p;
  if ((st = enqueue_matvec_round(A, x, compute, ell, seed, eps, rmax, ws, ws_bytes, s, p)) !=
      QTT_OK)
    return st;
  int32_t rk_host[QTT_MAXD + 1];
  double scal[2];
  QTT_HIP(hipMemcpyAsync(rk_host, p.t.v.rk, sizeof(int32_t) * (D + 1), hipMemcpyDeviceToHost,
                         s));
  QTT_HIP(hipMemcpyAsync(scal, p.w.scal, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));
  int64_t need = 0;
  for (int k = 0; k < D; ++k) need += (int64_t)rk_host[k] * y->nrow[k] * rk_host[k + 1];
  if (need > y->capacity)
    return fail(QTT_E_CAPACITY, "y: capacity " + std::to_string(y->capacity) + " < " +
                                    std::to_string(need));
  QTT_HIP(launch_pack(p.t.v, (double *)y->data, s));
  QTT_HIP(hipStreamSynchronize(s));
  for (int k = 0; k <= D; ++k) y->ranks[k] = rk_host[k];
  QTT_HIP(publish_ranks(y, s));
  if (norm) *norm = scal[0];
  if (err) *err = std::sqrt(scal[1] > 0.0 ? scal[1] : 0.0);
  return QTT_OK;
}

qtt_status qtt_dot(const qtt_tt *x, const qtt_tt *y, double *out, void *ws,
                   size_t ws_bytes, void *stream) {
  qtt::clear_stale_error();
  qtt_status st;
  if ((st = check_tt(x, "x", true)) != QTT_OK) return st;
  if ((st = check_tt(y, "y", true)) != QTT_OK) return st;
  if (!out) return fail(QTT_E_INVAL, "out is NULL");
  if (x->ncores != y->ncores) return fail(QTT_E_SHAPE, "core counts differ");
  for (int k = 0; k < x->ncores; ++k) {
    const int nx = x->nrow[k] * (x->ncol ? x->ncol[k] : 1);
    const int ny = y->nrow[k] * (y->ncol ? y->ncol[k] : 1);
    if (nx != ny) return fail(QTT_E_SHAPE, "modes differ");
  }
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  int32_t *rk = (int32_t *)ar.take(sizeof(int32_t) * 2 * (QTT_MAXD + 1));
  double *res = (double *)ar.take(sizeof(double));
  TTView vx, vy;
  packed_view(x, vx, rk);
  packed_view(y, vy, rk + (QTT_MAXD + 1));
  const int64_t we = dot_ws_elems(vx, vy);
  double *dws = (double *)ar.take(sizeof(double) * we);
  if (!ws || !ar.ok())
    return fail(QTT_E_CAPACITY, "workspace too small for qtt_dot: need " +
                                    std::to_string(ar.used));
  hipStream_t s = (hipStream_t)stream;
  QTT_HIP(upload_ranks(vx, x->ranks, s));
  QTT_HIP(upload_ranks(vy, y->ranks, s));
  QTT_HIP(launch_dot(vx, vy, res, dws, we, s));
  QTT_HIP(hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));
  return QTT_OK;
}

qtt_status qtt_axpby(double a, const qtt_tt *x, double b, const qtt_tt *y,
                     qtt_tt *z, void *ws, size_t ws_bytes, void *stream) {
  qtt::clear_stale_error();
  qtt_status st;
  if ((st = check_tt(x, "x", true)) != QTT_OK) return st;
  if ((st = check_tt(y, "y", true)) != QTT_OK) return st;
  if (!z || !z->ranks || !z->data) return fail(QTT_E_INVAL, "z: NULL field");
  if (x->ncores != y->ncores || z->ncores != x->ncores)
    return fail(QTT_E_SHAPE, "core counts differ");
  for (int k = 0; k < x->ncores; ++k)
    if (x->nrow[k] != y->nrow[k] || (x->ncol ? x->ncol[k] : 1) != (y->ncol ? y->ncol[k] : 1))
      return fail(QTT_E_SHAPE, "modes differ");
  if (z->data == x->data || z->data == y->data)
    return fail(QTT_E_INVAL, "z must not alias x or y");
  const int D = x->ncores;
  for (int k = 0; k <= D; ++k)
    z->ranks[k] = (k == 0 || k == D) ? 1 : x->ranks[k] + y->ranks[k];
  if (packed_elems(z) > z->capacity) return fail(QTT_E_CAPACITY, "z: capacity too small");
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  int32_t *rk = (int32_t *)ar.take(sizeof(int32_t) * 3 * (QTT_MAXD + 1));
  if (!ws || !ar.ok()) return fail(QTT_E_CAPACITY, "workspace too small for qtt_axpby");
  TTView vx, vy, vz;
  packed_view(x, vx, rk);
  packed_view(y, vy, rk + (QTT_MAXD + 1));
  packed_view(z, vz, rk + 2 * (QTT_MAXD + 1));
  hipStream_t s = (hipStream_t)stream;
  QTT_HIP(upload_ranks(vx, x->ranks, s));
  QTT_HIP(upload_ranks(vy, y->ranks, s));
  QTT_HIP(launch_axpby(a, nullptr, vx, b, nullptr, vy, vz, s));
  QTT_HIP(publish_ranks(z, s));
  return QTT_OK;
}

}  // extern "C"
