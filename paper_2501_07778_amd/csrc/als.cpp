// als.cpp — one-site alternating least squares (ALS) solve of K u = f on the
// QTT format: the host driver of the sweeps (kernels in k_als.hip).
//
// The paper solves its QTT systems with AMEn (Dolgov and Savostyanov 2014),
// which optimises one core at a time with the others fixed and orthogonal.
// This is that core update without AMEn's residual enrichment, at fixed
// ranks (Holtz, Rohwedder and Schneider 2012):
//   * u is kept with cores left of the active core k left-orthogonal and the
//     cores right of it right-orthogonal, so the map from core k to u is an
//     isometry U_k and the energy J(u) = <u, K u>/2 - <u, f> restricted to
//     core k is the quadratic form of B_k = U_k^T K U_k (SPD) and
//     g_k = U_k^T f;
//   * B_k and g_k are formed from the environments of <u, K u> and <u, f>
//     (kept for every bond and updated as the active core moves), B_k y = g_k
//     is solved by Cholesky, and y becomes core k;
//   * the active core moves by a QR (forward) or LQ (backward) step that
//     passes the triangular factor into the next core, leaving u unchanged.
// After a local solve J(u) = -<y, g_k>/2, so the energy is known after every
// sweep without a global product; it can only decrease (it is traced).
// Because the frames are orthonormal, replacing core k by y changes u by
// exactly ||y - x_k|| (x_k the core before the solve), so the sum of these
// over a sweep bounds ||u_s - u_{s-1}|| from above (triangle inequality).
// The sweeps stop when that sum, relative to ||u|| = ||y|| at the last
// solve, falls to tol.  The criterion resolves changes down to round-off (an
// energy difference would not: it is quadratic in the change and cancels at
// FP64 precision near 1e-7).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "internal.h"

namespace qtt {

namespace {

struct AlsLayout {
  std::vector<int> caps;          // ranks of u during the sweeps
  TTDesc U;                       // the iterate (slotted, ranks = caps)
  std::vector<double *> PK, PF;   // environments of <u, K u> and <u, f>
  double *W1 = nullptr, *W2 = nullptr;    // environment stages
  double *T = nullptr, *B = nullptr, *g = nullptr;  // local system
  double *Ld = nullptr, *z = nullptr;   // diagonal blocks of the factor, L^-1 g
  double *tmp = nullptr;          // core-sized scratch
  double *Rq = nullptr, *tau = nullptr;   // QR factor and reflector scales
  double *sc = nullptr;           // device scalars
  int *flag = nullptr;            // Cholesky breakdown
  RoundWs rw;                     // final rounding at eps
  TTDesc Ku, Rs;                  // residual check: K u and f - K u
  double *dense = nullptr, *full_ws = nullptr;
  int64_t N = 0;
  int32_t *rk_in = nullptr;       // device ranks of the packed K, f, x0
  double *start_ws = nullptr;     // energy of a start vector (<= caps)
  int64_t start_elems = 0;
  // AMEn enrichment: the rounded residual z, u + alpha z, their scratch
  TTDesc Z, U2;
  RoundWs rws;                    // rounding of f - K u after its sketch
  double *sk_ws = nullptr;
  double *en_ws = nullptr;
  int64_t en_elems = 0;
};

// device scalars: energy, ||f||^2, residual, <x0, K x0> and <f, x0> of a
// start vector, then per local solve of a sweep the pair
// (||y - x_k||^2, ||y||^2)
enum { A_YG = 0, A_FN2 = 2, A_RES = 4, A_X0KX0 = 6, A_FX0 = 7, A_LOC = 8 };
// enrichment scalars after the per-solve pairs: <f, z> and <u, K z>
// adjacent (the numerator of alpha), <z, K z>, alpha, <z, z>
enum { A_ZF = A_LOC + 2 * (QTT_MAXD + 1), A_UKZ, A_ZKZ, A_ALPHA, A_ZZ, A_END };
constexpr int ENRICH_OVERSAMPLE = 8;

bool carve_als(Arena &ar, const qtt_tt *K, const qtt_tt *f, const qtt_solve_opts *o,
               AlsLayout &L) {
  const int D = K->ncores;
  const int32_t *n = K->nrow;
  L.caps = bounded_caps(D, n, nullptr, o->rmax);
  const std::vector<int> &c = L.caps;
  bool ok = arena_tt(ar, L.U, D, n, nullptr, c);
  L.PK.assign(D + 1, nullptr);
  L.PF.assign(D + 1, nullptr);
  for (int k = 0; k <= D; ++k) {
    L.PK[k] = (double *)ar.take(sizeof(double) * c[k] * K->ranks[k] * c[k]);
    L.PF[k] = (double *)ar.take(sizeof(double) * c[k] * f->ranks[k]);
  }
  int64_t w = 1, tl = 1, nmax = 1, rmax = 1;
  for (int k = 0; k < D; ++k) {
    const int64_t r0 = c[k], r1 = c[k + 1], ra0 = K->ranks[k], ra1 = K->ranks[k + 1];
    w = std::max({w, r0 * ra0 * n[k] * r1, r0 * n[k] * ra1 * r1, r0 * n[k] * f->ranks[k + 1]});
    tl = std::max(tl, r0 * r0 * n[k] * n[k] * ra1);
    nmax = std::max(nmax, r0 * n[k] * r1);
    rmax = std::max({rmax, r0, r1});
  }
  L.W1 = (double *)ar.take(sizeof(double) * w);
  L.W2 = (double *)ar.take(sizeof(double) * w);
  L.T = (double *)ar.take(sizeof(double) * tl);
  L.B = (double *)ar.take(sizeof(double) * nmax * nmax);
  L.g = (double *)ar.take(sizeof(double) * nmax);
  L.Ld = (double *)ar.take(sizeof(double) * als_chol_diag_elems(nmax));
  L.z = (double *)ar.take(sizeof(double) * nmax);
  L.tmp = (double *)ar.take(sizeof(double) * nmax);
  L.Rq = (double *)ar.take(sizeof(double) * rmax * rmax);
  L.tau = (double *)ar.take(sizeof(double) * rmax);
  L.sc = (double *)ar.take(sizeof(double) * A_END);
  L.flag = (int *)ar.take(sizeof(int) * 4);
  if (o->method == QTT_SOLVE_AMEN) {
    // u + alpha z: the iterate's ranks (<= rmax - rmax_in after every
    // enrichment) plus the residual's (<= rmax_in), not limited by the
    // mode products; its rounding workspace also serves the final one
    const std::vector<int> cu = bounded_caps(D, n, nullptr, o->rmax - o->rmax_in);
    const std::vector<int> cz = bounded_caps(D, n, nullptr, o->rmax_in);
    std::vector<int> c2(D + 1, 1);
    for (int k = 1; k < D; ++k) c2[k] = cu[k] + cz[k];
    ok = arena_tt(ar, L.Z, D, n, nullptr, cz) && ok;
    ok = arena_tt(ar, L.U2, D, n, nullptr, c2) && ok;
    ok = round_ws_take(ar, L.U2.v, L.rw) && ok;
  } else {
    ok = round_ws_take(ar, L.U.v, L.rw) && ok;
  }
  // residual: K u has ranks R_k c_k, f - K u has f's ranks added
  std::vector<int> pc(c), rc(c);
  for (int k = 0; k <= D; ++k) {
    pc[k] = c[k] * K->ranks[k];
    rc[k] = (k == 0 || k == D) ? 1 : pc[k] + f->ranks[k];
  }
  ok = arena_tt(ar, L.Ku, D, n, nullptr, pc) && ok;
  ok = arena_tt(ar, L.Rs, D, n, nullptr, rc) && ok;
  L.N = 1;
  for (int k = 0; k < D; ++k) L.N *= n[k];
  L.dense = (double *)ar.take(sizeof(double) * L.N);
  std::vector<int32_t> rc32(rc.begin(), rc.end());
  int64_t fw = full_ws_elems(L.Rs.v, rc32.data());
  std::vector<int32_t> fr(f->ranks, f->ranks + D + 1);
  TTView fv;
  layout(fv, D, n, nullptr, std::vector<int>(fr.begin(), fr.end()));
  fw = std::max(fw, full_ws_elems(fv, fr.data()));
  L.full_ws = (double *)ar.take(sizeof(double) * fw);
  L.rk_in = (int32_t *)ar.take(sizeof(int32_t) * 3 * (QTT_MAXD + 1));
  // <x0, K x0> and <f, x0> of a start vector with ranks up to the caps
  {
    TTView uv, kv, fv2;
    layout(uv, D, n, nullptr, c);
    layout(kv, D, n, K->ncol, std::vector<int>(K->ranks, K->ranks + D + 1));
    layout(fv2, D, n, nullptr, std::vector<int>(f->ranks, f->ranks + D + 1));
    L.start_elems = std::max(dot3_ws_elems(uv, kv, uv), dot_ws_elems(fv2, uv));
    L.start_ws = (double *)ar.take(sizeof(double) * L.start_elems);
  }
  if (o->method == QTT_SOLVE_AMEN) {
    ok = round_ws_take(ar, L.Rs.v, L.rws) && ok;
    L.sk_ws = (double *)ar.take(sizeof(double) *
                                sketch_ws_elems(L.Rs.v, o->rmax_in + ENRICH_OVERSAMPLE));
    TTView kv, fv2;
    layout(kv, D, n, K->ncol, std::vector<int>(K->ranks, K->ranks + D + 1));
    layout(fv2, D, n, nullptr, std::vector<int>(f->ranks, f->ranks + D + 1));
    L.en_elems = std::max({dot3_ws_elems(L.U.v, kv, L.Z.v), dot3_ws_elems(L.Z.v, kv, L.Z.v),
                           dot_ws_elems(fv2, L.Z.v), dot_ws_elems(L.Z.v, L.Z.v)});
    L.en_ws = (double *)ar.take(sizeof(double) * L.en_elems);
  }
  return ok && ar.ok();
}

// element offsets of the cores of a packed train
std::vector<int64_t> packed_offsets(const qtt_tt *t) {
  std::vector<int64_t> off(t->ncores + 1, 0);
  for (int k = 0; k < t->ncores; ++k)
    off[k + 1] = off[k] + (int64_t)t->ranks[k] * t->nrow[k] * (t->ncol ? t->ncol[k] : 1) *
                              t->ranks[k + 1];
  return off;
}

void view_of_packed(const qtt_tt *t, TTView &v, int32_t *rk_dev) {
  std::vector<int> r(t->ranks, t->ranks + t->ncores + 1);
  layout(v, t->ncores, t->nrow, t->ncol, r);
  // packed: no slot padding
  std::vector<int64_t> off = packed_offsets(t);
  for (int k = 0; k < t->ncores; ++k) v.off[k] = off[k];
  for (int k = t->ncores; k < QTT_MAXD; ++k) v.off[k] = off[t->ncores];
  v.rk = rk_dev;
  v.data = t->data;
}

}  // namespace

qtt_status check_als_opts(const qtt_solve_opts *o) {
  if (!(o->tol > 0.0) || !(o->eps >= 0.0)) return fail(QTT_E_INVAL, "ALS: tol > 0, eps >= 0");
  if (o->method == QTT_SOLVE_AMEN &&
      (o->rmax_in < 1 || o->rmax < 2 * o->rmax_in || !(o->eps_in >= 0.0)))
    return fail(QTT_E_INVAL, "AMEN: rmax_in >= 1, rmax >= 2 rmax_in and eps_in >= 0 required");
  if (o->rmax < 1 || o->rmax > 512) return fail(QTT_E_INVAL, "ALS: rmax must be in 1..512");
  if (o->maxit_out < 1) return fail(QTT_E_INVAL, "ALS: maxit_out (sweeps) must be >= 1");
  if (o->compute != QTT_F64)
    return fail(QTT_E_UNSUPPORTED, "ALS: local systems are FP64 only (compute = QTT_F64)");
  return QTT_OK;
}

size_t als_workspace_bytes(const qtt_tt *K, const qtt_tt *f, const qtt_solve_opts *o) {
  Arena ar;
  ar.dry = true;
  AlsLayout L;
  carve_als(ar, K, f, o, L);
  return ar.used + 4096;
}

qtt_status solve_als(const qtt_tt *K, const qtt_tt *f, const qtt_tt *xin,
                     const qtt_solve_opts *o, qtt_tt *u, qtt_solve_report *rep, void *ws,
                     size_t ws_bytes, hipStream_t s) {
  const qtt_tt *x0 = xin;
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  AlsLayout L;
  if (!carve_als(ar, K, f, o, L)) return fail(QTT_E_CAPACITY, "solve workspace too small");
  const int D = K->ncores;
  const int32_t *n = K->nrow;
  // rank ramp: stages at rmax_in, 2 rmax_in, ... then rmax (cheap sweeps at
  // low rank find the subspace; the local solves cost O((r n r)^3))
  const bool amen = o->method == QTT_SOLVE_AMEN;
  std::vector<int> stage_r;
  if (amen)
    stage_r.push_back(o->rmax_in);   // start ranks; the enrichment sets the rest
  else if (o->rmax_in > 0 && o->rmax_in < o->rmax)
    for (int r = o->rmax_in; r < o->rmax; r *= 2) stage_r.push_back(r);
  if (!amen) stage_r.push_back(o->rmax);
  // a stage whose caps (limited by the mode products) equal the next one's
  // is not a lower rank: drop it
  for (size_t i = 0; i + 1 < stage_r.size();) {
    if (bounded_caps(D, n, nullptr, stage_r[i]) == bounded_caps(D, n, nullptr, stage_r[i + 1]))
      stage_r.erase(stage_r.begin() + i);
    else
      ++i;
  }
  size_t st0 = 0;
  if (amen && x0) {
    const std::vector<int> cs = bounded_caps(D, n, nullptr, o->rmax - o->rmax_in);
    for (int k = 0; k <= D; ++k)
      if (x0->ranks[k] > cs[k])
        return fail(QTT_E_SHAPE, "AMEN: x0 ranks must be <= rmax - rmax_in");
  }
  if (x0 && !amen)  // start at the first stage whose caps hold x0
    while (st0 + 1 < stage_r.size()) {
      const std::vector<int> cs = bounded_caps(D, n, nullptr, stage_r[st0]);
      bool fits = true;
      for (int k = 0; k <= D; ++k) fits = fits && x0->ranks[k] <= cs[k];
      if (fits) break;
      ++st0;
    }
  std::vector<int> c = bounded_caps(D, n, nullptr, stage_r[st0]);
  if (amen && x0) c.assign(x0->ranks, x0->ranks + D + 1);
  const int32_t *RK = K->ranks, *RF = f->ranks;
  const std::vector<int64_t> koff = packed_offsets(K), foff = packed_offsets(f);
  auto core = [&](int k) { return L.U.v.data + L.U.v.off[k]; };
  auto kc = [&](int k) { return (const double *)K->data + koff[k]; };
  auto fc = [&](int k) { return (const double *)f->data + foff[k]; };
  auto csize = [&](int k) { return (int64_t)c[k] * n[k] * c[k + 1]; };
  const bool trace = std::getenv("QTT_SOLVE_TRACE") != nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  auto secs = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };

  // ||f|| on the dense grid (FP64)
  TTView fv;
  view_of_packed(f, fv, L.rk_in);
  QTT_HIP(upload_ranks(fv, f->ranks, s));
  QTT_HIP(tt_full(fv, f->ranks, L.dense, L.full_ws, s));
  QTT_HIP(launch_diff_norm2(L.dense, nullptr, L.N, L.sc + A_FN2, s));

  // the view of K for products and three-operand inner products
  TTView Kv;
  view_of_packed(K, Kv, L.rk_in + (QTT_MAXD + 1));
  QTT_HIP(upload_ranks(Kv, K->ranks, s));

  // A start vector enters scaled by alpha = <f, x0> / <x0, K x0>, the
  // minimiser of the energy J(alpha x0) = alpha^2 <x0, K x0> / 2 -
  // alpha <f, x0>, whose value -<f, x0>^2 / (2 <x0, K x0>) is below J(0) = 0
  // unless x0 has no component along the solution (<f, x0> = 0) or its
  // values are not finite: then the solve falls back to its cold start.
  double x0_energy = 0.0, x0_alpha = 1.0;
  if (x0) {
    TTView xv;
    view_of_packed(x0, xv, L.rk_in + 2 * (QTT_MAXD + 1));
    QTT_HIP(upload_ranks(xv, x0->ranks, s));
    QTT_HIP(launch_dot3(xv, Kv, xv, L.sc + A_X0KX0, L.start_ws, L.start_elems, s));
    QTT_HIP(launch_dot(fv, xv, L.sc + A_FX0, L.start_ws, L.start_elems, s));
    double e2[2];
    QTT_HIP(hipMemcpyAsync(e2, L.sc + A_X0KX0, sizeof(e2), hipMemcpyDeviceToHost, s));
    QTT_HIP(hipStreamSynchronize(s));
    const double xkx = e2[0], fx = e2[1];
    x0_alpha = fx / xkx;
    x0_energy = -0.5 * fx * fx / xkx;
    if (!(xkx > 0.0) || !std::isfinite(x0_alpha) || !(x0_energy < 0.0)) {
      x0 = nullptr;
      st0 = 0;
      c = bounded_caps(D, n, nullptr, stage_r[0]);
    }
  }
  const int warm = xin ? (x0 ? 1 : -1) : 0;
  // start: x0 zero-padded to the caps, else deterministic random cores
  if (x0) {
    const std::vector<int64_t> xoff = packed_offsets(x0);
    for (int k = 0; k < D; ++k)
      QTT_HIP(als_pad_core((const double *)x0->data + xoff[k], x0->ranks[k], n[k],
                           x0->ranks[k + 1], core(k), c[k], c[k + 1], s));
  } else {
    QTT_HIP(als_fill(L.U.v.data, L.U.elems, o->seed, 1.0, s));
  }
  {
    std::vector<int32_t> c32(c.begin(), c.end());
    QTT_HIP(upload_ranks(L.U.v, c32.data(), s));
  }
  if (x0) QTT_HIP(launch_scale(L.U.v, x0_alpha, s));
  QTT_HIP(hipMemsetAsync(L.flag, 0, sizeof(int), s));

  // orthogonality-centre moves
  auto qr_step = [&](int k) -> hipError_t {  // centre k -> k + 1
    const int rows = c[k] * n[k], cols = c[k + 1];
    hipError_t e = als_qr(core(k), rows, cols, L.Rq, L.tau, s);
    if (e != hipSuccess) return e;
    const int ncol = n[k + 1] * c[k + 2];
    e = als_gemm(L.Rq, cols, core(k + 1), cols, false, L.tmp, cols, cols, ncol, cols, s);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(core(k + 1), L.tmp, sizeof(double) * csize(k + 1),
                          hipMemcpyDeviceToDevice, s);
  };
  auto lq_step = [&](int k) -> hipError_t {  // centre k -> k - 1
    const int r0 = c[k], ncol = n[k] * c[k + 1];
    hipError_t e = als_transpose(core(k), r0, ncol, L.tmp, s);
    if (e != hipSuccess) return e;
    if ((e = als_qr(L.tmp, ncol, r0, L.Rq, L.tau, s)) != hipSuccess) return e;
    if ((e = als_transpose(L.tmp, ncol, r0, core(k), s)) != hipSuccess) return e;
    const int rows = c[k - 1] * n[k - 1];
    if ((e = als_gemm(core(k - 1), rows, L.Rq, r0, true, L.tmp, rows, rows, r0, r0, s)) !=
        hipSuccess)
      return e;
    return hipMemcpyAsync(core(k - 1), L.tmp, sizeof(double) * csize(k - 1),
                          hipMemcpyDeviceToDevice, s);
  };
  auto env_left = [&](int k) -> hipError_t {  // PK, PF at bond k + 1 from bond k
    hipError_t e = als_env3_left(L.PK[k], core(k), kc(k), core(k), L.PK[k + 1], L.W1, L.W2, c[k],
                                 RK[k], n[k], RK[k + 1], c[k + 1], s);
    if (e != hipSuccess) return e;
    return als_env2_left(L.PF[k], core(k), fc(k), L.PF[k + 1], L.W1, c[k], RF[k], n[k], c[k + 1],
                         RF[k + 1], s);
  };
  auto env_right = [&](int k) -> hipError_t {  // PK, PF at bond k from bond k + 1
    hipError_t e = als_env3_right(L.PK[k + 1], core(k), kc(k), core(k), L.PK[k], L.W1, L.W2, c[k],
                                  RK[k], n[k], RK[k + 1], c[k + 1], s);
    if (e != hipSuccess) return e;
    return als_env2_right(L.PF[k + 1], core(k), fc(k), L.PF[k], L.W1, c[k], RF[k], n[k],
                          c[k + 1], RF[k + 1], s);
  };
  int solves = 0;
  // slot: index of the solve within its sweep (its change lands in A_LOC)
  auto solve_core = [&](int k, int slot) -> hipError_t {
    hipError_t e = als_local_system(L.PK[k], kc(k), L.PK[k + 1], L.PF[k], fc(k), L.PF[k + 1], L.T,
                                    L.B, L.g, c[k], RK[k], n[k], RK[k + 1], c[k + 1], RF[k],
                                    RF[k + 1], s);
    if (e != hipSuccess) return e;
    const int64_t N = csize(k);
    if ((e = hipMemcpyAsync(L.tmp, core(k), sizeof(double) * N, hipMemcpyDeviceToDevice, s)) !=
        hipSuccess)
      return e;
    ++solves;
    if ((e = als_cholesky_solve(L.B, N, L.g, core(k), L.Ld, L.z, L.flag, L.sc + A_YG, s)) !=
        hipSuccess)
      return e;
    return launch_diff_norm2(core(k), L.tmp, N, L.sc + A_LOC + 2 * slot, s);
  };

  QTT_HIP(als_fill_value(L.PK[0], 1, 1.0, s));
  QTT_HIP(als_fill_value(L.PF[0], 1, 1.0, s));
  QTT_HIP(als_fill_value(L.PK[D], 1, 1.0, s));
  QTT_HIP(als_fill_value(L.PF[D], 1, 1.0, s));

  qtt_solve_report R;
  std::memset(&R, 0, sizeof(R));
  auto read_energy = [&](double &J, int &flag) -> qtt_status {
    double yg = 0.0;
    QTT_HIP(hipMemcpyAsync(&yg, L.sc + A_YG, sizeof(double), hipMemcpyDeviceToHost, s));
    QTT_HIP(hipMemcpyAsync(&flag, L.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    QTT_HIP(hipStreamSynchronize(s));
    J = -0.5 * yg;
    return QTT_OK;
  };
  double J = 0.0, crit = 0.0;
  int flag = 0, sweep = 0;
  qtt_status st;
  bool converged = false;
  constexpr int RAMP_SWEEPS = 3;
  double unorm = 0.0;
  // right-orthogonalise cores D-1..1, the environments from the right, then
  // solve the first core
  auto restart = [&]() -> qtt_status {
    for (int k = D - 1; k >= 1; --k) QTT_HIP(lq_step(k));
    for (int k = D - 1; k >= 1; --k) QTT_HIP(env_right(k));
    QTT_HIP(solve_core(0, 0));
    qtt_status e = read_energy(J, flag);
    if (e != QTT_OK) return e;
    if (flag) return fail(QTT_E_INVAL, "ALS: local matrix not positive definite (is K SPD?)");
    return QTT_OK;
  };
  // one sweep (forward on even, backward on odd counts); crit = the change
  // of u over the sweep relative to ||u||
  auto sweep_once = [&](bool forward, int rank_label) -> qtt_status {
    if (forward) {
      for (int k = 0; k + 1 < D; ++k) {
        QTT_HIP(qr_step(k));
        QTT_HIP(env_left(k));
        QTT_HIP(solve_core(k + 1, k));
      }
    } else {
      for (int k = D - 1; k >= 1; --k) {
        QTT_HIP(lq_step(k));
        QTT_HIP(env_right(k));
        QTT_HIP(solve_core(k - 1, D - 1 - k));
      }
    }
    // change of u over the sweep: sum of the local changes over ||u||
    std::vector<double> loc(2 * (D - 1));
    QTT_HIP(hipMemcpyAsync(loc.data(), L.sc + A_LOC, sizeof(double) * 2 * (D - 1),
                           hipMemcpyDeviceToHost, s));
    qtt_status e = read_energy(J, flag);
    if (e != QTT_OK) return e;
    if (flag) return fail(QTT_E_INVAL, "ALS: local matrix not positive definite (is K SPD?)");
    double dsum = 0.0;
    for (int j = 0; j < D - 1; ++j) dsum += std::sqrt(std::max(loc[2 * j], 0.0));
    unorm = std::sqrt(std::max(loc[2 * (D - 2) + 1], 0.0));
    if (!std::isfinite(J) || !std::isfinite(dsum)) return fail(QTT_E_NOCONV, "ALS: not finite");
    crit = unorm > 0.0 ? dsum / unorm : 0.0;
    if (sweep < 64) R.residual_hist[sweep] = crit;
    if (trace)
      std::fprintf(stderr, "[qtt_solve als] %.3fs rank %d sweep %d energy %.15e change %.3e\n",
                   secs(), rank_label, sweep, J, crit);
    return QTT_OK;
  };
  if (D == 1) {
    if ((st = restart()) != QTT_OK) return st;
    converged = true;
  } else if (amen) {
    // residual enrichment: z = round(f - K u, eps_in, rmax_in) by a sketch,
    // alpha = <f - K u, z> / <z, K z>, then u <- round(u + alpha z, eps,
    // rmax - rmax_in); echange = |alpha| ||z|| / ||u||
    uint64_t call = 0;
    double echange = HUGE_VAL;
    auto residual_direction = [&]() -> qtt_status {
      QTT_HIP(launch_matvec(Kv, L.U.v, L.Ku.v, QTT_F64, s));
      QTT_HIP(launch_axpby(1.0, nullptr, fv, -1.0, nullptr, L.Ku.v, L.Rs.v, s));
      const int ell = o->rmax_in + ENRICH_OVERSAMPLE;
      QTT_HIP(sketch_tt(L.Rs.v, ell, o->seed, call++, L.sk_ws, s));
      QTT_HIP(round_tt(L.Rs.v, o->eps_in, o->rmax_in, L.rws, s, true, ell));
      QTT_HIP(launch_copy_tt(L.Rs.v, L.Z.v, s));
      QTT_HIP(launch_dot(fv, L.Z.v, L.sc + A_ZF, L.en_ws, L.en_elems, s));
      QTT_HIP(launch_dot3(L.U.v, Kv, L.Z.v, L.sc + A_UKZ, L.en_ws, L.en_elems, s));
      QTT_HIP(launch_dot3(L.Z.v, Kv, L.Z.v, L.sc + A_ZKZ, L.en_ws, L.en_elems, s));
      QTT_HIP(launch_dot(L.Z.v, L.Z.v, L.sc + A_ZZ, L.en_ws, L.en_elems, s));
      QTT_HIP(launch_scalar(SC_DIFF_DIV, L.sc + A_ALPHA, L.sc + A_ZF, L.sc + A_ZKZ, 0.0, s));
      double v[A_END - A_ZF];
      QTT_HIP(hipMemcpyAsync(v, L.sc + A_ZF, sizeof(v), hipMemcpyDeviceToHost, s));
      QTT_HIP(hipStreamSynchronize(s));
      const double alpha = v[A_ALPHA - A_ZF], zz = v[A_ZZ - A_ZF];
      if (!std::isfinite(alpha) || !std::isfinite(zz))
        return fail(QTT_E_NOCONV, "AMEN: enrichment not finite");
      echange = unorm > 0.0 ? std::fabs(alpha) * std::sqrt(std::max(zz, 0.0)) / unorm : 0.0;
      return QTT_OK;
    };
    auto enrich = [&]() -> qtt_status {
      QTT_HIP(launch_axpby(1.0, nullptr, L.U.v, 1.0, L.sc + A_ALPHA, L.Z.v, L.U2.v, s));
      QTT_HIP(round_tt(L.U2.v, o->eps, o->rmax - o->rmax_in, L.rw, s));
      int32_t r2[QTT_MAXD + 1];
      QTT_HIP(hipMemcpyAsync(r2, L.U2.v.rk, sizeof(int32_t) * (D + 1), hipMemcpyDeviceToHost, s));
      QTT_HIP(hipStreamSynchronize(s));
      QTT_HIP(launch_copy_tt(L.U2.v, L.U.v, s));
      for (int k = 0; k <= D; ++k) c[k] = r2[k];
      return QTT_OK;
    };
    int maxr = 0;
    while (!converged && sweep < o->maxit_out) {
      maxr = *std::max_element(c.begin(), c.end());
      if ((st = restart()) != QTT_OK) return st;
      for (int sw = 0; sw < 2 && sweep < o->maxit_out; ++sw, ++sweep)
        if ((st = sweep_once(sw % 2 == 0, maxr)) != QTT_OK) return st;
      if ((st = residual_direction()) != QTT_OK) return st;
      if (trace)
        std::fprintf(stderr, "[qtt_solve amen] %.3fs ranks up to %d, enrichment change %.3e\n",
                     secs(), maxr, echange);
      if (crit <= o->tol && echange <= o->tol) {
        converged = true;
        break;
      }
      if (sweep >= o->maxit_out) break;
      if ((st = enrich()) != QTT_OK) return st;
    }
  } else {
    for (size_t stg = st0; stg < stage_r.size() && !converged && sweep < o->maxit_out; ++stg) {
      const bool last = stg + 1 == stage_r.size();
      if (stg > st0) {
        // zero-pad every core to the next stage's caps (through the scratch)
        const std::vector<int> cn = bounded_caps(D, n, nullptr, stage_r[stg]);
        for (int k = 0; k < D; ++k) {
          QTT_HIP(hipMemcpyAsync(L.tmp, core(k), sizeof(double) * csize(k),
                                 hipMemcpyDeviceToDevice, s));
          QTT_HIP(als_pad_core(L.tmp, c[k], n[k], c[k + 1], core(k), cn[k], cn[k + 1], s));
        }
        c = cn;
        std::vector<int32_t> c32(c.begin(), c.end());
        QTT_HIP(upload_ranks(L.U.v, c32.data(), s));
      }
      if ((st = restart()) != QTT_OK) return st;
      const int budget =
          last ? o->maxit_out - sweep : std::min(RAMP_SWEEPS, o->maxit_out - sweep);
      for (int sw = 0; sw < budget && !converged; ++sw, ++sweep) {
        if ((st = sweep_once(sw % 2 == 0, stage_r[stg])) != QTT_OK) return st;
        if (last && crit <= o->tol) converged = true;
      }
    }
  }
  R.outer = sweep;
  R.inner = solves;
  R.criterion = crit;

  // optional compression of the result at eps (exact rounding)
  if (o->eps > 0.0) QTT_HIP(round_tt(L.U.v, o->eps, o->rmax, L.rw, s));
  int32_t ur[QTT_MAXD + 1];
  QTT_HIP(hipMemcpyAsync(ur, L.U.v.rk, sizeof(int32_t) * (D + 1), hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));

  // FP64 check: ||f - K u|| from the exact dense contraction of f - K u
  QTT_HIP(launch_matvec(Kv, L.U.v, L.Ku.v, QTT_F64, s));
  QTT_HIP(launch_axpby(1.0, nullptr, fv, -1.0, nullptr, L.Ku.v, L.Rs.v, s));
  std::vector<int32_t> rr(D + 1);
  for (int k = 0; k <= D; ++k) rr[k] = (k == 0 || k == D) ? 1 : RF[k] + RK[k] * ur[k];
  QTT_HIP(tt_full(L.Rs.v, rr.data(), L.dense, L.full_ws, s));
  QTT_HIP(launch_diff_norm2(L.dense, nullptr, L.N, L.sc + A_RES, s));
  double fn2[2], rn2[2];
  QTT_HIP(hipMemcpyAsync(fn2, L.sc + A_FN2, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  QTT_HIP(hipMemcpyAsync(rn2, L.sc + A_RES, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));
  const double fnorm = std::sqrt(std::max(fn2[1], 0.0));
  R.residual = fnorm > 0.0 ? std::sqrt(std::max(rn2[0], 0.0)) / fnorm : 0.0;
  if (trace)
    std::fprintf(stderr, "[qtt_solve als] %.3fs residual %.3e after %d sweeps\n", secs(),
                 R.residual, R.outer);

  // pack u
  int64_t need = 0;
  for (int k = 0; k < D; ++k) need += (int64_t)ur[k] * n[k] * ur[k + 1];
  if (need > u->capacity) return fail(QTT_E_CAPACITY, "u: capacity too small for the result");
  QTT_HIP(launch_pack(L.U.v, u->data, s));
  QTT_HIP(hipStreamSynchronize(s));
  int mr = 1;
  for (int k = 0; k <= D; ++k) {
    u->ranks[k] = ur[k];
    mr = std::max(mr, (int)ur[k]);
  }
  R.max_rank = mr;
  QTT_HIP(publish_ranks(u, s));
  R.status = converged ? QTT_OK : QTT_E_NOCONV;
  R.warm_start = warm;
  R.warm_energy = xin ? x0_energy : 0.0;
  if (rep) *rep = R;
  if (!converged) return fail(QTT_E_NOCONV, "ALS: change of u above tol after maxit_out sweeps");
  return QTT_OK;
}

}  // namespace qtt
