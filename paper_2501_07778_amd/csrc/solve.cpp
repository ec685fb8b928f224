// solve.cpp — qtt_solve: iterative solvers on the QTT format driven by the
// QTT matrix-vector product and TT rounding.
//
// The paper solves K u = f with AMEn (Sec. 3, 3.7 and 4), which it cites but
// does not describe; these solves are built from the two operations of the
// format instead.
//
// CHEBYSHEV (for fine grids, with the BPX preconditioner C): Chebyshev
// semi-iteration on C K u = C f with the residual r = f - K u recomputed
// from the iterate at every step (exact product, then rounding relative to
// ||r||), z = round(C r), d = c1 d + c2 z, u = round(u + d).  No quantity is
// updated by a recurrence that rounding could corrupt, so truncation only
// perturbs each step; the coefficients depend only on the spectral bounds
// and are computed on the host.  Stop: sqrt(<r, C r>) <= tol sqrt(<f, C f>).
//
// CG_IR (small grids):
//   outer (FP64):  r = round(f - K u); stop when ||f - K u|| <= tol ||f||
//                  (the norm of the unrounded difference comes out of the
//                  rounding's QR sweep); e = CG(K, r); u = round(u + e)
//   inner:         truncated CG: the products K p and C r are formed
//                  exactly and used unrounded in <p, K p> and <r, C r>; the
//                  new residual r - alpha K p and direction z + beta p are
//                  rounded as sums to (eps_in, rmax_in), so each truncation
//                  error is relative to the vector CG continues with; the
//                  iterate is rounded to (eps, rmax) (its truncation error
//                  reaches the true residual multiplied by ||K||); ||r||^2 is
//                  read off the rounding of r.  With a preconditioner C
//                  (QTT matrix ~ K^-1) z = C r, otherwise z = r.
// All scalars and ranks stay on the device; the host synchronises only at
// the convergence checks (every check_every inner iterations and once per
// refinement step).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"

namespace qtt {
namespace {

struct SolveLayout {
  TTDesc U[2], Ku, R, X[2], Rr[2], Pp[2], Q;
  TTView Rin, Pin, Qin;  // R, Pp[0], Q with the caps of a rounded inner vector
  TTView Pin1;           // Pp[1] likewise
  TTView Uin[2];         // U[s] with the caps of a rounded iterate
  RoundWs rw;
  double *dot_ws = nullptr;
  int64_t dot_elems = 0;
  double *sc = nullptr;  // device scalars
  double *sk_ws = nullptr;    // randomised rounding
  double *dense = nullptr;    // dense residual (N doubles)
  double *full_ws = nullptr;  // dense contraction workspace
  int64_t N = 0;
};

enum {
  S_FNORM2 = 0, S_RHO, S_PQ, S_ALPHA, S_BETA, S_RHONEW, S_ONE, S_RES, S_PK, S_CR,
  S_FP, S_XKP, S_ZKP, S_PKP, S_COUNT = 16
};

std::vector<int> caps_for(const qtt_tt *K, int r) {
  return bounded_caps(K->ncores, K->nrow, nullptr, r);
}

bool carve(Arena &ar, const qtt_tt *K, const qtt_tt *f, const qtt_solve_opts *o,
           SolveLayout &L) {
  const int D = K->ncores;
  const int32_t *n = K->nrow;
  int Rk = 1;
  for (int k = 0; k <= D; ++k) Rk = K->ranks[k] > Rk ? K->ranks[k] : Rk;
  int rf = 1;
  for (int k = 0; k <= D; ++k) rf = f->ranks[k] > rf ? f->ranks[k] : rf;
  const int rmax = o->rmax, rin = o->rmax_in;
  // products have ranks R_k * r_k bond by bond
  auto prod_caps = [&](int r) {
    std::vector<int> c = caps_for(K, r);
    for (int k = 0; k <= D; ++k) c[k] *= K->ranks[k];
    return c;
  };
  // products with the preconditioner share the buffer of K p
  auto op_caps = [&](int r) {
    std::vector<int> c = caps_for(K, r);
    for (int k = 0; k <= D; ++k) {
      int R = K->ranks[k];
      if (o->precond) R = R > o->precond->ranks[k] ? R : o->precond->ranks[k];
      c[k] *= R;
    }
    return c;
  };
  auto sum_caps = [&](std::vector<int> a, const std::vector<int> &b) {
    for (size_t k = 0; k < a.size(); ++k) a[k] += b[k];
    a.front() = a.back() = 1;
    return a;
  };
  std::vector<int> cu = caps_for(K, rmax), ci = caps_for(K, rin);
  std::vector<int> cf(f->ranks, f->ranks + D + 1);
  bool ok = true;
  // u + e: both ranks are bounded by rmax (the correction keeps the outer
  // accuracy)
  for (int s = 0; s < 2; ++s) ok &= arena_tt(ar, L.U[s], D, n, nullptr, sum_caps(cu, cu));
  ok &= arena_tt(ar, L.Ku, D, n, nullptr, prod_caps(rmax));
  std::vector<int> cr = sum_caps(prod_caps(rmax), cf);
  ok &= arena_tt(ar, L.R, D, n, nullptr, sum_caps(cr, ci));
  std::vector<int> c2 = sum_caps(sum_caps(ci, ci), ci);
  for (int s = 0; s < 2; ++s) {
    ok &= arena_tt(ar, L.X[s], D, n, nullptr, sum_caps(sum_caps(cu, ci), ci));
    ok &= arena_tt(ar, L.Rr[s], D, n, nullptr, sum_caps(ci, op_caps(rin)));
    ok &= arena_tt(ar, L.Pp[s], D, n, nullptr, sum_caps(ci, op_caps(rin)));
  }
  ok &= arena_tt(ar, L.Q, D, n, nullptr, op_caps(rin));
  // the rounding workspace serves every operand: size it for the bondwise
  // largest caps
  TTView big = L.R.v;
  for (const TTDesc *t : {&L.U[0], &L.Ku, &L.X[0], &L.Rr[0], &L.Pp[0], &L.Q})
    for (int k = 0; k <= D; ++k) big.cap[k] = big.cap[k] > t->v.cap[k] ? big.cap[k] : t->v.cap[k];
  ok &= round_ws_take(ar, big, L.rw);
  TTView fv = L.R.v;
  for (int k = 0; k <= D; ++k) fv.cap[k] = cf[k];
  L.dot_elems = dot_ws_elems(L.R.v, L.R.v);
  for (int64_t e : {dot_ws_elems(fv, fv), dot_ws_elems(L.Pp[0].v, L.Q.v),
                    dot_ws_elems(L.R.v, L.Q.v), dot_ws_elems(L.Rr[0].v, L.Q.v),
                    dot_ws_elems(L.Pp[0].v, L.Ku.v)})
    L.dot_elems = e > L.dot_elems ? e : L.dot_elems;
  // <r, C r> and <v, K v> of the Chebyshev solve, without the products:
  // r and v are rounded to rmax_in first
  {
    L.Rin = L.R.v;
    L.Pin = L.Pp[0].v;
    L.Pin1 = L.Pp[1].v;
    L.Qin = L.Q.v;
    TTView Kc = L.R.v, Cc = L.R.v;
    for (int k = 0; k <= D; ++k) {
      L.Rin.cap[k] = L.Pin.cap[k] = L.Pin1.cap[k] = L.Qin.cap[k] = ci[k];
      Kc.cap[k] = K->ranks[k];
      Cc.cap[k] = o->precond ? o->precond->ranks[k] : 1;
    }
    L.Uin[0] = L.U[0].v;
    L.Uin[1] = L.U[1].v;
    for (int k = 0; k <= D; ++k) L.Uin[0].cap[k] = L.Uin[1].cap[k] = cu[k];
    const TTView &Uc = L.Uin[0];
    for (int64_t e : {dot3_ws_elems(L.Rin, Cc, L.Rin), dot3_ws_elems(L.Pin, Kc, L.Pin),
                      dot3_ws_elems(Uc, Kc, L.Pin), dot_ws_elems(fv, L.Pin)})
      L.dot_elems = e > L.dot_elems ? e : L.dot_elems;
  }
  L.dot_ws = (double *)ar.take(sizeof(double) * L.dot_elems);
  L.sc = (double *)ar.take(sizeof(double) * S_COUNT);
  if (o->sketch > 0) {
    const int ell = rin + o->sketch;
    int64_t e = sketch_ws_elems(L.R.v, ell);
    e = std::max<int64_t>(e, sketch_ws_elems(L.Rr[0].v, ell));
    e = std::max<int64_t>(e, sketch_ws_elems(L.Pp[0].v, ell));
    L.sk_ws = (double *)ar.take(sizeof(double) * e);
  }
  // FP64 residual check on the dense grid
  L.N = 1;
  for (int k = 0; k < D; ++k) L.N *= n[k];
  L.dense = (double *)ar.take(sizeof(double) * L.N);
  std::vector<int32_t> rc(L.R.v.cap, L.R.v.cap + D + 1);
  L.full_ws = (double *)ar.take(sizeof(double) * full_ws_elems(L.R.v, rc.data()));
  (void)Rk;
  (void)rf;
  return ok && ar.ok();
}

void packed_view_of(const qtt_tt *t, TTView &v, int32_t *rk) {
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
  v.rk = rk;
  v.data = t->data;
}

qtt_status check_opts(const qtt_solve_opts *o) {
  if (!o) return fail(QTT_E_INVAL, "opts is NULL");
  if (o->method == QTT_SOLVE_ALS || o->method == QTT_SOLVE_AMEN) return check_als_opts(o);
  if (!(o->tol > 0.0) || !(o->eps >= 0.0) || !(o->eps_in >= 0.0) || !(o->red_in > 0.0))
    return fail(QTT_E_INVAL, "tolerances must be positive");
  if (o->rmax < 1 || o->rmax_in < 1 || o->rmax > 4096 || o->rmax_in > 4096)
    return fail(QTT_E_INVAL, "rank caps must be in 1..4096");
  if (o->maxit_in < 1 || o->maxit_out < 0) return fail(QTT_E_INVAL, "bad iteration limits");
  if (o->compute != QTT_F64 && o->compute != QTT_F32 && o->compute != QTT_BF16)
    return fail(QTT_E_INVAL, "bad compute dtype");
  if (o->sketch < 0 || o->sketch > 256) return fail(QTT_E_INVAL, "sketch must be in 0..256");
  if (o->method != QTT_SOLVE_CG_IR && o->method != QTT_SOLVE_CHEBYSHEV &&
      o->method != QTT_SOLVE_FCG)
    return fail(QTT_E_INVAL, "unknown solve method");
  if (o->method != QTT_SOLVE_CG_IR) {
    if (!o->precond) return fail(QTT_E_INVAL, "this solve method needs a preconditioner");
    if (o->rmax_in > o->rmax) return fail(QTT_E_INVAL, "rmax_in must be <= rmax");
    if (o->check_every < 1) return fail(QTT_E_INVAL, "check_every must be >= 1");
    const double lmin = o->lmin > 0.0 ? o->lmin : 0.09;
    if (o->lmax > 0.0 && !(o->lmax > lmin))
      return fail(QTT_E_INVAL, "Chebyshev solve: lmax must exceed lmin");
  }
  return QTT_OK;
}

qtt_status check_precond(const qtt_tt *K, const qtt_tt *C) {
  if (!C) return QTT_OK;
  qtt_status st;
  if ((st = check_tt(C, "precond", true)) != QTT_OK) return st;
  if (!C->ncol || C->ncores != K->ncores)
    return fail(QTT_E_INVAL, "precond must be a QTT matrix with K's cores");
  for (int k = 0; k < K->ncores; ++k)
    if (C->nrow[k] != K->nrow[k] || C->ncol[k] != K->ncol[k])
      return fail(QTT_E_SHAPE, "precond modes differ from K's");
  if (C->ranks[0] != 1 || C->ranks[C->ncores] != 1)
    return fail(QTT_E_SHAPE, "precond boundary ranks must be 1");
  return QTT_OK;
}

qtt_status check_system(const qtt_tt *K, const qtt_tt *f) {
  qtt_status st;
  if ((st = check_tt(K, "K", true)) != QTT_OK) return st;
  if ((st = check_tt(f, "f", true)) != QTT_OK) return st;
  if (!K->ncol || f->ncol) return fail(QTT_E_INVAL, "K must be a matrix, f a vector");
  if (K->ncores != f->ncores || K->ncores < 1 || K->ncores > QTT_MAX_CORES)
    return fail(QTT_E_SHAPE, "core counts differ");
  for (int k = 0; k < K->ncores; ++k)
    if (K->nrow[k] != K->ncol[k] || K->nrow[k] != f->nrow[k])
      return fail(QTT_E_SHAPE, "K must be square with f's modes");
  if (K->ranks[0] != 1 || K->ranks[K->ncores] != 1 || f->ranks[0] != 1 || f->ranks[f->ncores] != 1)
    return fail(QTT_E_SHAPE, "boundary ranks must be 1");
  if (!K->data || !f->data) return fail(QTT_E_INVAL, "NULL data");
  return QTT_OK;
}

}  // namespace
}  // namespace qtt

using namespace qtt;

extern "C" qtt_status qtt_solve_workspace(const qtt_tt *K, const qtt_tt *f,
                                          const qtt_solve_opts *o, size_t *bytes) {
  qtt_status st;
  if ((st = check_system(K, f)) != QTT_OK) return st;
  if ((st = check_opts(o)) != QTT_OK) return st;
  if ((st = check_precond(K, o->precond)) != QTT_OK) return st;
  if (!bytes) return fail(QTT_E_INVAL, "bytes is NULL");
  if (o->method == QTT_SOLVE_ALS || o->method == QTT_SOLVE_AMEN) {
    *bytes = als_workspace_bytes(K, f, o);
    return QTT_OK;
  }
  Arena ar;
  ar.dry = true;
  SolveLayout L;
  carve(ar, K, f, o, L);
  ar.take(sizeof(int32_t) * 4 * (QTT_MAXD + 1));
  *bytes = ar.used + 4096;
  return QTT_OK;
}

extern "C" qtt_status qtt_solve(const qtt_tt *K, const qtt_tt *f, const qtt_tt *x0,
                                const qtt_solve_opts *o, qtt_tt *u, qtt_solve_report *rep,
                                void *ws, size_t ws_bytes, void *stream) {
  qtt::clear_stale_error();
  qtt_status st;
  if ((st = check_system(K, f)) != QTT_OK) return st;
  if ((st = check_opts(o)) != QTT_OK) return st;
  if ((st = check_precond(K, o->precond)) != QTT_OK) return st;
  if (!u || !u->data || !u->ranks || !u->nrow || u->ncores != K->ncores)
    return fail(QTT_E_INVAL, "bad u");
  for (int k = 0; k < K->ncores; ++k)
    if (u->nrow[k] != K->nrow[k]) return fail(QTT_E_SHAPE, "u modes differ from K's");
  if (x0) {
    if ((st = check_tt(x0, "x0", true)) != QTT_OK) return st;
    if (x0->ncores != K->ncores || x0->ncol) return fail(QTT_E_SHAPE, "bad x0");
    for (int k = 0; k < K->ncores; ++k)
      if (x0->nrow[k] != K->nrow[k]) return fail(QTT_E_SHAPE, "x0 modes differ from K's");
    std::vector<int> cu = bounded_caps(K->ncores, K->nrow, nullptr, o->rmax);
    for (int k = 0; k <= x0->ncores; ++k)
      if (x0->ranks[k] > cu[k])
        return fail(QTT_E_SHAPE, "x0 rank exceeds rmax or the mode-product bound");
  }
  if (!ws) return fail(QTT_E_CAPACITY, "workspace is NULL");
  if (o->method == QTT_SOLVE_ALS || o->method == QTT_SOLVE_AMEN)
    return solve_als(K, f, x0, o, u, rep, ws, ws_bytes, (hipStream_t)stream);
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  SolveLayout L;
  if (!carve(ar, K, f, o, L)) return fail(QTT_E_CAPACITY, "solve workspace too small");
  int32_t *rk = (int32_t *)ar.take(sizeof(int32_t) * 4 * (QTT_MAXD + 1));
  if (!ar.ok()) return fail(QTT_E_CAPACITY, "solve workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const int D = K->ncores;
  TTView Kv, fv, x0v;
  packed_view_of(K, Kv, rk);
  packed_view_of(f, fv, rk + (QTT_MAXD + 1));
  QTT_HIP(upload_ranks(Kv, K->ranks, s));
  QTT_HIP(upload_ranks(fv, f->ranks, s));
  const bool pre = o->precond != nullptr;
  TTView Cv;
  if (pre) {
    packed_view_of(o->precond, Cv, rk + 3 * (QTT_MAXD + 1));
    QTT_HIP(upload_ranks(Cv, o->precond->ranks, s));
  }
  double *sc = L.sc;
  const RoundWs &rw = L.rw;
  QTT_HIP(launch_scalar(SC_SET, sc + S_ONE, nullptr, nullptr, 1.0, s));
  QTT_HIP(tt_full(fv, f->ranks, L.dense, L.full_ws, s));
  QTT_HIP(launch_diff_norm2(L.dense, nullptr, L.N, sc + S_FNORM2, s));
  double fn2 = 0.0;
  QTT_HIP(hipMemcpyAsync(&fn2, sc + S_FNORM2, sizeof(double), hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));
  uint64_t call = 0;
  // QTT_SOLVE_TRACE=1 prints the refinement history to stderr
  const bool trace = std::getenv("QTT_SOLVE_TRACE") != nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  auto secs = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  const double fnorm = std::sqrt(fn2 > 0.0 ? fn2 : 0.0);
  qtt_solve_report R;
  std::memset(&R, 0, sizeof(R));
  int cur = 0;
  bool have_u = false;
  if (x0) {
    packed_view_of(x0, x0v, rk + 2 * (QTT_MAXD + 1));
    QTT_HIP(upload_ranks(x0v, x0->ranks, s));
    QTT_HIP(launch_copy_tt(x0v, L.U[0].v, s));
    have_u = true;
  }
  if (fnorm == 0.0) {
    // zero load: u = 0
    std::vector<int32_t> ones(D + 1, 1);
    QTT_HIP(upload_ranks(L.U[0].v, ones.data(), s));
    QTT_HIP(hipMemsetAsync(L.U[0].v.data, 0, sizeof(double) * L.U[0].elems, s));
    have_u = true;
  }
  const qtt_dtype lowp = (qtt_dtype)o->compute;
  bool converged = fnorm == 0.0;
  // sketch (if enabled) then exact rounding to (eps, r)
  auto round_sk = [&](const TTView &v, double eps, int r) -> hipError_t {
    hipError_t e = hipSuccess;
    if (o->sketch > 0) e = sketch_tt(v, r + o->sketch, o->seed, call++, L.sk_ws, s);
    if (e != hipSuccess) return e;
    return round_tt(v, eps, r, rw, s, o->sketch > 0, o->sketch > 0 ? r + o->sketch : 0);
  };
  auto read_scalar = [&](int idx, double &out) -> hipError_t {
    hipError_t e = hipMemcpyAsync(&out, sc + idx, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
  };
  if (o->method != QTT_SOLVE_CG_IR && fnorm > 0.0) {
    const bool cheb = o->method == QTT_SOLVE_CHEBYSHEV;
    const int rin = o->rmax_in;
    // <f, C f> with f rounded to the inner rank cap (exact when f's ranks fit)
    QTT_HIP(launch_copy_tt(fv, L.R.v, s));
    QTT_HIP(round_tt(L.R.v, 0.0, rin, rw, s));
    QTT_HIP(launch_dot3(L.Rin, Cv, L.Rin, sc + S_RHO, L.dot_ws, L.dot_elems, s));
    double fcf = 0.0;
    QTT_HIP(read_scalar(S_RHO, fcf));
    if (!(fcf > 0.0)) return fail(QTT_E_INVAL, "<f, C f> is not positive: C is not SPD");
    const double lmin = o->lmin > 0.0 ? o->lmin : 0.09;
    double lmax = o->lmax;
    if (cheb && !(lmax > 0.0)) {
      // power steps v <- round(C round(K v)); Rayleigh quotient
      // <K v, C K v> / <v, K v> (no normalisation: the rounding is relative
      // and 12 steps stay far inside the FP64 range)
      QTT_HIP(launch_copy_tt(L.R.v, L.Pp[0].v, s));
      for (int it = 0; it < 12; ++it) {
        QTT_HIP(launch_dot3(L.Pin, Kv, L.Pin, sc + S_PK, L.dot_ws, L.dot_elems, s));
        QTT_HIP(launch_matvec(Kv, L.Pp[0].v, L.Ku.v, lowp, s));
        QTT_HIP(launch_copy_tt(L.Ku.v, L.R.v, s));
        QTT_HIP(round_sk(L.R.v, o->eps_in, rin));
        QTT_HIP(launch_dot3(L.Rin, Cv, L.Rin, sc + S_CR, L.dot_ws, L.dot_elems, s));
        QTT_HIP(launch_matvec(Cv, L.R.v, L.Q.v, lowp, s));
        QTT_HIP(launch_copy_tt(L.Q.v, L.Pp[0].v, s));
        QTT_HIP(round_sk(L.Pp[0].v, o->eps_in, rin));
      }
      double pk = 0.0, cr = 0.0;
      QTT_HIP(read_scalar(S_PK, pk));
      QTT_HIP(read_scalar(S_CR, cr));
      if (!(pk > 0.0) || !std::isfinite(cr)) return fail(QTT_E_INVAL, "K is not SPD (power step)");
      lmax = 1.12 * cr / pk;
      if (!(lmax > lmin)) lmax = 2.0 * lmin;
      if (trace) std::fprintf(stderr, "[qtt_solve] %.3fs lmax estimate %.4f\n", secs(), lmax);
    }
    R.lmax = cheb ? lmax : 0.0;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    int pi = 0, nh = 0;
    bool have_d = false;
    int it = 0;
    for (it = 0; it <= o->maxit_in; ++it) {
      // r = round(f - K u): exact FP64 product and difference, then rounding
      // relative to ||r|| (the residual sets the attainable accuracy, so it
      // stays FP64 in every compute mode; the low-precision mode applies to
      // the preconditioner product C r only)
      if (have_u) {
        QTT_HIP(launch_matvec(Kv, L.U[cur].v, L.Ku.v, QTT_F64, s));
        QTT_HIP(launch_axpby(1.0, nullptr, fv, -1.0, nullptr, L.Ku.v, L.R.v, s));
      } else {
        QTT_HIP(launch_copy_tt(fv, L.R.v, s));
      }
      QTT_HIP(round_sk(L.R.v, o->eps_in, rin));
      // the criterion <r, C r>, then C r
      QTT_HIP(launch_dot3(L.Rin, Cv, L.Rin, sc + S_RES, L.dot_ws, L.dot_elems, s));
      QTT_HIP(launch_matvec(Cv, L.R.v, L.Q.v, lowp, s));
      if (it % o->check_every == 0 || it == o->maxit_in) {
        double rcr = 0.0;
        QTT_HIP(read_scalar(S_RES, rcr));
        if (!std::isfinite(rcr)) return fail(QTT_E_NOCONV, "residual is not finite");
        const double crit = std::sqrt(std::fmax(rcr, 0.0) / fcf);
        if (nh < 64) R.residual_hist[nh] = crit;
        ++nh;
        R.criterion = crit;
        if (trace)
          std::fprintf(stderr, "[qtt_solve] %.3fs it %d criterion %.3e\n", secs(), it, crit);
        if (crit <= o->tol) {
          converged = true;
          break;
        }
      }
      if (it == o->maxit_in) break;
      // z = round(C r)
      QTT_HIP(round_sk(L.Q.v, o->eps_in, rin));
      if (!cheb) {
        // p = round(z - beta p), beta = <z, K p> / <p, K p>
        if (!have_d) {
          QTT_HIP(launch_copy_tt(L.Q.v, L.Pp[pi].v, s));
          have_d = true;
        } else {
          QTT_HIP(launch_dot3(L.Qin, Kv, pi == 0 ? L.Pin : L.Pin1, sc + S_ZKP, L.dot_ws,
                              L.dot_elems, s));
          QTT_HIP(launch_scalar(SC_DIV_POS, sc + S_BETA, sc + S_ZKP, sc + S_PKP, 0.0, s));
          QTT_HIP(launch_axpby(1.0, nullptr, L.Q.v, -1.0, sc + S_BETA, L.Pp[pi].v,
                               L.Pp[1 - pi].v, s));
          pi = 1 - pi;
          QTT_HIP(round_tt(L.Pp[pi].v, o->eps_in, rin, rw, s, false, 2 * rin));
        }
        // alpha = <f - K u, p> / <p, K p> from u and p themselves
        const TTView &pv = pi == 0 ? L.Pin : L.Pin1;
        QTT_HIP(launch_dot3(pv, Kv, pv, sc + S_PKP, L.dot_ws, L.dot_elems, s));
        QTT_HIP(launch_dot(fv, pv, sc + S_FP, L.dot_ws, L.dot_elems, s));
        if (have_u)
          QTT_HIP(launch_dot3(L.Uin[cur], Kv, pv, sc + S_XKP, L.dot_ws, L.dot_elems, s));
        else
          QTT_HIP(launch_scalar(SC_SET, sc + S_XKP, nullptr, nullptr, 0.0, s));
        QTT_HIP(launch_scalar(SC_DIFF_DIV, sc + S_ALPHA, sc + S_FP, sc + S_PKP, 0.0, s));
        if (have_u) {
          QTT_HIP(launch_axpby(1.0, nullptr, L.U[cur].v, 1.0, sc + S_ALPHA, L.Pp[pi].v,
                               L.U[1 - cur].v, s));
          cur = 1 - cur;
          QTT_HIP(round_tt(L.U[cur].v, o->eps, o->rmax, rw, s, false, o->rmax + rin));
        } else {
          QTT_HIP(launch_copy_tt(L.Pp[pi].v, L.U[cur].v, s));
          QTT_HIP(launch_scale(L.U[cur].v, 1.0, s, sc + S_ALPHA));
          have_u = true;
        }
        continue;
      }
      // Chebyshev: d = c1 d + c2 z
      if (!have_d) {
        QTT_HIP(launch_copy_tt(L.Q.v, L.Pp[pi].v, s));
        QTT_HIP(launch_scale(L.Pp[pi].v, 1.0 / theta, s));
        have_d = true;
      } else {
        const double rho_new = 1.0 / (2.0 * sigma - rho);
        QTT_HIP(launch_axpby(rho_new * rho, nullptr, L.Pp[pi].v, 2.0 * rho_new / delta, nullptr,
                             L.Q.v, L.Pp[1 - pi].v, s));
        pi = 1 - pi;
        QTT_HIP(round_tt(L.Pp[pi].v, o->eps_in, rin, rw, s, false, 2 * rin));
        rho = rho_new;
      }
      // u = round(u + d)
      if (have_u) {
        QTT_HIP(launch_axpby(1.0, nullptr, L.U[cur].v, 1.0, nullptr, L.Pp[pi].v, L.U[1 - cur].v,
                             s));
        cur = 1 - cur;
        QTT_HIP(round_tt(L.U[cur].v, o->eps, o->rmax, rw, s, false, o->rmax + rin));
      } else {
        QTT_HIP(launch_copy_tt(L.Pp[pi].v, L.U[cur].v, s));
        have_u = true;
      }
    }
    R.inner = it;
    // FP64 check of the returned iterate
    if (have_u) {
      double rel = 0.0;
      QTT_HIP(launch_matvec(Kv, L.U[cur].v, L.Ku.v, QTT_F64, s));
      QTT_HIP(launch_axpby(1.0, nullptr, fv, -1.0, nullptr, L.Ku.v, L.R.v, s));
      int32_t ur[QTT_MAXD + 1];
      std::vector<int32_t> rr(D + 1);
      QTT_HIP(hipMemcpyAsync(ur, L.U[cur].v.rk, sizeof(int32_t) * (D + 1), hipMemcpyDeviceToHost,
                             s));
      QTT_HIP(hipStreamSynchronize(s));
      for (int k = 0; k <= D; ++k) {
        rr[k] = (k == 0 || k == D) ? 1 : f->ranks[k] + K->ranks[k] * ur[k];
        if (ur[k] < 1 || ur[k] > L.U[cur].v.cap[k] || rr[k] > L.R.v.cap[k])
          return fail(QTT_E_CAPACITY, "iterate rank exceeds its buffer");
      }
      QTT_HIP(tt_full(L.R.v, rr.data(), L.dense, L.full_ws, s));
      QTT_HIP(launch_diff_norm2(L.dense, nullptr, L.N, sc + S_RES, s));
      double rn2[2];
      QTT_HIP(hipMemcpyAsync(rn2, sc + S_RES, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
      QTT_HIP(hipStreamSynchronize(s));
      rel = std::sqrt(rn2[0]) / fnorm;
      R.residual = rel;
    }
  }
  for (int out = 0; out <= o->maxit_out && fnorm > 0.0 && o->method == QTT_SOLVE_CG_IR; ++out) {
    // residual r = f - K u (exact product and difference)
    if (have_u) {
      QTT_HIP(launch_matvec(Kv, L.U[cur].v, L.Ku.v, QTT_F64, s));
      QTT_HIP(launch_axpby(1.0, nullptr, fv, -1.0, nullptr, L.Ku.v, L.R.v, s));
    } else {
      QTT_HIP(launch_copy_tt(fv, L.R.v, s));
    }
    // FP64 check: ||f - K u|| from the exact dense contraction of the
    // residual train (its ranks are known: f's plus K's times u's)
    double rel;
    {
      int32_t ur[QTT_MAXD + 1];
      std::vector<int32_t> rr(D + 1);
      if (have_u) {
        QTT_HIP(hipMemcpyAsync(ur, L.U[cur].v.rk, sizeof(int32_t) * (D + 1),
                               hipMemcpyDeviceToHost, s));
        QTT_HIP(hipStreamSynchronize(s));
        for (int k = 0; k <= D; ++k) {
          rr[k] = (k == 0 || k == D) ? 1 : f->ranks[k] + K->ranks[k] * ur[k];
          if (ur[k] < 1 || ur[k] > L.U[cur].v.cap[k] || rr[k] > L.R.v.cap[k])
            return fail(QTT_E_CAPACITY, "iterate rank exceeds its buffer");
        }
      } else {
        for (int k = 0; k <= D; ++k) rr[k] = f->ranks[k];
      }
      QTT_HIP(tt_full(L.R.v, rr.data(), L.dense, L.full_ws, s));
      QTT_HIP(launch_diff_norm2(L.dense, nullptr, L.N, sc + S_RES, s));
      double rn2[2];
      QTT_HIP(hipMemcpyAsync(rn2, sc + S_RES, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
      QTT_HIP(hipStreamSynchronize(s));
      rel = std::sqrt(rn2[0]) / fnorm;
    }
    if (out < 64) R.residual_hist[out] = rel;
    R.residual = rel;
    if (trace)
      std::fprintf(stderr, "[qtt_solve] %.3fs outer %d residual %.3e inner total %d\n", secs(), out,
                   rel, R.inner);
    if (!std::isfinite(rel)) return fail(QTT_E_NOCONV, "residual is not finite");
    if (rel <= o->tol) {
      converged = true;
      break;
    }
    if (out == o->maxit_out) break;
    // the correction's right-hand side: the residual rounded to (eps_in, rmax_in)
    if (o->sketch > 0) QTT_HIP(sketch_tt(L.R.v, o->rmax_in + o->sketch, o->seed, call++, L.sk_ws, s));
    QTT_HIP(round_tt(L.R.v, o->eps_in, o->rmax_in, rw, s, o->sketch > 0,
                     o->sketch > 0 ? o->rmax_in + o->sketch : 0));
    double nr[2];
    QTT_HIP(hipMemcpyAsync(nr, rw.scal, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
    QTT_HIP(hipStreamSynchronize(s));
    // inner CG on K e = r: x = 0, r_c = r, p = r
    int xi = 0, ri = 0, pi = 0;
    {
      std::vector<int32_t> ones(D + 1, 1);
      QTT_HIP(upload_ranks(L.X[0].v, ones.data(), s));
      QTT_HIP(hipMemsetAsync(L.X[0].v.data, 0, sizeof(double) * L.X[0].elems, s));
    }
    QTT_HIP(launch_copy_tt(L.R.v, L.Rr[0].v, s));
    // truncated (P)CG: products exact, sums rounded (see the file comment)
    auto round_in = [&](const TTView &v) -> hipError_t {
      hipError_t e = hipSuccess;
      if (o->sketch > 0) e = sketch_tt(v, o->rmax_in + o->sketch, o->seed, call++, L.sk_ws, s);
      if (e != hipSuccess) return e;
      return round_tt(v, o->eps_in, o->rmax_in, rw, s, o->sketch > 0,
                      o->sketch > 0 ? o->rmax_in + o->sketch : 0);
    };
    if (pre) {
      // z = C r (exact), rho = <r, z>, p = round(z)
      QTT_HIP(launch_matvec(Cv, L.R.v, L.Q.v, lowp, s));
      QTT_HIP(launch_dot(L.R.v, L.Q.v, sc + S_RHO, L.dot_ws, L.dot_elems, s));
      QTT_HIP(launch_copy_tt(L.Q.v, L.Pp[0].v, s));
      QTT_HIP(round_in(L.Pp[0].v));
    } else {
      QTT_HIP(launch_copy_tt(L.R.v, L.Pp[0].v, s));
      // rho = ||r||^2 after the rounding above
      QTT_HIP(launch_scalar(SC_NORM2, sc + S_RHO, rw.scal, nullptr, 0.0, s));
    }
    const double bn = nr[0] * std::sqrt(std::fmax(1.0 - (nr[1] / (nr[0] * nr[0] + 1e-300)), 0.0));
    int it = 0;
    for (it = 1; it <= o->maxit_in; ++it) {
      // q = K p (exact), alpha = rho / <p, q>
      QTT_HIP(launch_matvec(Kv, L.Pp[pi].v, L.Q.v, lowp, s));
      QTT_HIP(launch_dot(L.Pp[pi].v, L.Q.v, sc + S_PQ, L.dot_ws, L.dot_elems, s));
      QTT_HIP(launch_scalar(SC_DIV_POS, sc + S_ALPHA, sc + S_RHO, sc + S_PQ, 0.0, s));
      // x = round(x + alpha p) at the outer accuracy: its truncation error
      // reaches the true residual multiplied by ||K||
      QTT_HIP(launch_axpby(1.0, nullptr, L.X[xi].v, 1.0, sc + S_ALPHA, L.Pp[pi].v, L.X[1 - xi].v, s));
      xi = 1 - xi;
      QTT_HIP(round_tt(L.X[xi].v, o->eps, o->rmax, rw, s, false, o->rmax + o->rmax_in));
      // r = round(r - alpha q), rounded as one sum; ||r||^2 from the rounding
      QTT_HIP(launch_axpby(1.0, nullptr, L.Rr[ri].v, -1.0, sc + S_ALPHA, L.Q.v, L.Rr[1 - ri].v, s));
      ri = 1 - ri;
      QTT_HIP(round_in(L.Rr[ri].v));
      QTT_HIP(launch_scalar(SC_NORM2, sc + S_RES, rw.scal, nullptr, 0.0, s));
      if (it % o->check_every == 0 || it == o->maxit_in) {
        double rr = 0.0;
        QTT_HIP(hipMemcpyAsync(&rr, sc + S_RES, sizeof(double), hipMemcpyDeviceToHost, s));
        QTT_HIP(hipStreamSynchronize(s));
        if (!std::isfinite(rr)) return fail(QTT_E_NOCONV, "inner residual is not finite");
        if (trace && it % 50 == 0)
          std::fprintf(stderr, "[qtt_solve] %.3fs   inner %d ||r||/||b|| %.3e\n", secs(), it,
                       std::sqrt(rr) / bn);
        if (std::sqrt(rr) <= o->red_in * bn) break;
      }
      const TTView *zv = &L.Rr[ri].v;
      if (pre) {
        // z = C r (exact), rho_new = <r, z>
        QTT_HIP(launch_matvec(Cv, L.Rr[ri].v, L.Q.v, lowp, s));
        QTT_HIP(launch_dot(L.Rr[ri].v, L.Q.v, sc + S_RHONEW, L.dot_ws, L.dot_elems, s));
        zv = &L.Q.v;
      } else {
        QTT_HIP(launch_scalar(SC_COPY, sc + S_RHONEW, sc + S_RES, nullptr, 0.0, s));
      }
      // p = round(z + beta p), rounded as one sum
      QTT_HIP(launch_scalar(SC_DIV, sc + S_BETA, sc + S_RHONEW, sc + S_RHO, 0.0, s));
      QTT_HIP(launch_axpby(1.0, nullptr, *zv, 1.0, sc + S_BETA, L.Pp[pi].v, L.Pp[1 - pi].v, s));
      pi = 1 - pi;
      QTT_HIP(round_in(L.Pp[pi].v));
      QTT_HIP(launch_scalar(SC_COPY, sc + S_RHO, sc + S_RHONEW, nullptr, 0.0, s));
    }
    R.inner += it > o->maxit_in ? o->maxit_in : it;
    // u = round(u + e)
    if (have_u) {
      QTT_HIP(launch_axpby(1.0, nullptr, L.U[cur].v, 1.0, nullptr, L.X[xi].v, L.U[1 - cur].v, s));
      cur = 1 - cur;
    } else {
      QTT_HIP(launch_copy_tt(L.X[xi].v, L.U[cur].v, s));
      have_u = true;
    }
    QTT_HIP(round_tt(L.U[cur].v, o->eps, o->rmax, rw, s, false, 2 * o->rmax));
    R.outer += 1;
  }
  if (!have_u) {
    std::vector<int32_t> ones(D + 1, 1);
    QTT_HIP(upload_ranks(L.U[cur].v, ones.data(), s));
    QTT_HIP(hipMemsetAsync(L.U[cur].v.data, 0, sizeof(double) * L.U[cur].elems, s));
  }
  // pack u into the caller's buffer
  int32_t rkh[QTT_MAXD + 1];
  QTT_HIP(hipMemcpyAsync(rkh, L.U[cur].v.rk, sizeof(int32_t) * (D + 1), hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));
  int64_t need = 0;
  for (int k = 0; k < D; ++k) need += (int64_t)rkh[k] * K->nrow[k] * rkh[k + 1];
  if (need > u->capacity) return fail(QTT_E_CAPACITY, "u: capacity too small for the result");
  QTT_HIP(launch_pack(L.U[cur].v, u->data, s));
  QTT_HIP(hipStreamSynchronize(s));
  int mr = 1;
  for (int k = 0; k <= D; ++k) {
    u->ranks[k] = rkh[k];
    mr = rkh[k] > mr ? rkh[k] : mr;
  }
  R.max_rank = mr;
  QTT_HIP(publish_ranks(u, s));
  R.status = converged ? QTT_OK : QTT_E_NOCONV;
  R.warm_start = x0 ? 1 : 0;
  if (rep) *rep = R;
  if (!converged) return fail(QTT_E_NOCONV, "tolerance not reached");
  return QTT_OK;
}
