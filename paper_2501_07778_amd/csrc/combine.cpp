// combine.cpp — TT utilities of the learned warm start.
// qtt_tt_combine: z = sum_i c_i x_i for TT vectors of equal modes by core
// concatenation (the sum of Sec. 4's format): the first cores side by side
// (the coefficients scale them), middle cores block-diagonal, last cores
// stacked; ranks add.
// qtt_tt_align: the gauge of one train brought to that of a reference by an
// orthogonal Procrustes rotation at every bond, right to left.
// qtt_tt_contract_last: a train with a parameter mode as its last core,
// evaluated at one parameter vector (the last core contracted with the
// weights and merged into the one before).
#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

namespace qtt {
namespace {

struct PlaceArg {
  int D;
  int n[QTT_MAXD];
  int r[QTT_MAXD + 1];        // ranks of the term
  int zr[QTT_MAXD + 1];       // ranks of z
  int o[QTT_MAXD + 1];        // rank offset of the term's block at each bond
  int64_t xoff[QTT_MAXD];     // core offsets in the packed term
  int64_t zoff[QTT_MAXD];     // core offsets in the packed z
};

__global__ void k_zero(double *z, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    z[e] = 0.0;
}

// core k = blockIdx.y of the term into its block of z (scaled by c on core 0)
__global__ void k_place(const double *x, double *z, PlaceArg a, double c) {
  const int k = blockIdx.y;
  const int r0 = a.r[k], n = a.n[k], r1 = a.r[k + 1];
  const int Z0 = a.zr[k];
  const int o0 = a.o[k], o1 = a.o[k + 1];
  const double *xc = x + a.xoff[k];
  double *zc = z + a.zoff[k];
  const double sc = (k == 0) ? c : 1.0;
  const int64_t ne = (int64_t)r0 * n * r1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int al = (int)(e % r0);
    const int64_t t = e / r0;
    const int j = (int)(t % n), be = (int)(t / n);
    zc[(o0 + al) + (int64_t)Z0 * (j + (int64_t)n * (o1 + be))] = sc * xc[e];
  }
}

constexpr int ALIGN_RMAX = 48;
constexpr int ALIGN_SWEEPS = 40;

struct AlignArg {
  int D;
  int n[QTT_MAXD];
  int r[QTT_MAXD + 1];
  int64_t off[QTT_MAXD];
};

// One block of 256 threads.  For k = D-1..1: M = X_k R_k^T (r x r), its SVD
// by one-sided Jacobi (M V = B, columns of B = U S), Q = B S^-1 V^T, then
// X_k <- Q^T X_k and X_{k-1} <- X_{k-1} Q, staged through LDS in chunks of
// ALIGN_RMAX columns (rows).
__global__ void __launch_bounds__(256) k_align(double *x, const double *ref, AlignArg a) {
  constexpr int R = ALIGN_RMAX;
  __shared__ double Bm[R * R], Vm[R * R], Qm[R * R], sig[R];
  __shared__ int rotated, skip;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int k = a.D - 1; k >= 1; --k) {
    const int r = a.r[k], n = a.n[k], r1 = a.r[k + 1];
    double *Xk = x + a.off[k];
    const double *Rk = ref + a.off[k];
    const int ncolk = n * r1;
    for (int e = t; e < r * r; e += nt) {
      const int p = e % r, c = e / r;
      double s = 0.0;
      for (int ib = 0; ib < ncolk; ++ib) s += Xk[p + (int64_t)r * ib] * Rk[c + (int64_t)r * ib];
      Bm[p + r * c] = s;
      Vm[p + r * c] = (p == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    // one-sided Jacobi on the columns of Bm, round-robin pairs, a thread a pair
    const int N = r + (r & 1);
    for (int sweep = 0; sweep < ALIGN_SWEEPS; ++sweep) {
      if (t == 0) rotated = 0;
      __syncthreads();
      for (int rd = 0; rd < N - 1; ++rd) {
        if (t < N / 2) {
          int p = (rd + t) % (N - 1);
          int q = (t == 0) ? (N - 1) : (rd - t + N - 1) % (N - 1);
          if (p > q) { const int tmp = p; p = q; q = tmp; }
          if (q < r) {
            double al = 0.0, be = 0.0, ga = 0.0;
            for (int l = 0; l < r; ++l) {
              const double u = Bm[l + r * p], v = Bm[l + r * q];
              al += u * u;
              be += v * v;
              ga += u * v;
            }
            if (ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
              const double zeta = (be - al) / (2.0 * ga);
              const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
              const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
              for (int l = 0; l < r; ++l) {
                const double u = Bm[l + r * p], v = Bm[l + r * q];
                Bm[l + r * p] = c * u - sn * v;
                Bm[l + r * q] = sn * u + c * v;
                const double vu = Vm[l + r * p], vv = Vm[l + r * q];
                Vm[l + r * p] = c * vu - sn * vv;
                Vm[l + r * q] = sn * vu + c * vv;
              }
              rotated = 1;
            }
          }
        }
        __syncthreads();
      }
      const int more = rotated;
      __syncthreads();
      if (!more) break;
    }
    for (int j = t; j < r; j += nt) {
      double s = 0.0;
      for (int l = 0; l < r; ++l) s += Bm[l + r * j] * Bm[l + r * j];
      sig[j] = sqrt(s);
    }
    __syncthreads();
    if (t == 0) {
      double smax = 0.0, smin = HUGE_VAL;
      for (int j = 0; j < r; ++j) {
        smax = fmax(smax, sig[j]);
        smin = fmin(smin, sig[j]);
      }
      skip = !(smax > 0.0) || smin <= 1e-13 * smax;
    }
    __syncthreads();
    if (skip) continue;   // block-uniform
    // Q[p, c] = sum_j B[p, j] V[c, j] / sig_j
    for (int e = t; e < r * r; e += nt) {
      const int p = e % r, c = e / r;
      double s = 0.0;
      for (int j = 0; j < r; ++j) s += Bm[p + r * j] * Vm[c + r * j] / sig[j];
      Qm[p + r * c] = s;
    }
    __syncthreads();
    // X_k <- Q^T X_k, ALIGN_RMAX columns (i, b) at a time through Bm
    for (int c0 = 0; c0 < ncolk; c0 += R) {
      const int nc = min(R, ncolk - c0);
      for (int e = t; e < r * nc; e += nt) Bm[e] = Xk[(int64_t)r * c0 + e];
      __syncthreads();
      for (int e = t; e < r * nc; e += nt) {
        const int p = e % r, cc = e / r;
        double s = 0.0;
        for (int c = 0; c < r; ++c) s += Qm[c + r * p] * Bm[c + r * cc];
        Xk[(int64_t)r * c0 + e] = s;
      }
      __syncthreads();
    }
    // X_{k-1} <- X_{k-1} Q: rows (alpha, i) of the (r0 n0) x r unfolding
    const int r0 = a.r[k - 1], n0 = a.n[k - 1];
    const int nrows = r0 * n0;
    double *Xp = x + a.off[k - 1];
    for (int q0 = 0; q0 < nrows; q0 += R) {
      const int nr = min(R, nrows - q0);
      for (int e = t; e < nr * r; e += nt) {
        const int rw = e % nr, b = e / nr;
        Bm[rw + R * b] = Xp[(q0 + rw) + (int64_t)nrows * b];
      }
      __syncthreads();
      for (int e = t; e < nr * r; e += nt) {
        const int rw = e % nr, b2 = e / nr;
        double s = 0.0;
        for (int b = 0; b < r; ++b) s += Bm[rw + R * b] * Qm[b + r * b2];
        Xp[(q0 + rw) + (int64_t)nrows * b2] = s;
      }
      __syncthreads();
    }
  }
}

// y's last core (r0 x n x 1) = x's core D-2 (r0 x n x r1) times v, with
// v = x's last core (r1 x nl) times the weights w (nl); one block
__global__ void __launch_bounds__(256)
    k_contract_last(const double *xc, const double *xl, const double *w, double *yc, int r0,
                    int n, int r1, int nl) {
  __shared__ double v[1024];
  for (int b = threadIdx.x; b < r1; b += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < nl; ++i) s += xl[b + (int64_t)r1 * i] * w[i];
    v[b] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r0 * n; e += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < r1; ++b) s += xc[e + (int64_t)r0 * n * b] * v[b];
    yc[e] = s;
  }
}

}  // namespace
}  // namespace qtt

using namespace qtt;

extern "C" qtt_status qtt_tt_contract_last(const qtt_tt *x, const double *w, qtt_tt *y,
                                           void *stream) {
  qtt::clear_stale_error();
  qtt_status st;
  if ((st = check_tt(x, "x", true)) != QTT_OK) return st;
  if (x->ncol) return fail(QTT_E_INVAL, "qtt_tt_contract_last takes a TT vector");
  const int D = x->ncores;
  if (D < 3) return fail(QTT_E_UNSUPPORTED, "qtt_tt_contract_last needs at least three cores");
  if (!w) return fail(QTT_E_INVAL, "w is NULL");
  if (!y || !y->ranks || !y->data || !y->nrow) return fail(QTT_E_INVAL, "y: NULL field");
  if (y->ncores != D - 1 || y->ncol) return fail(QTT_E_SHAPE, "y must be a vector of D - 1 cores");
  if (y->data == x->data) return fail(QTT_E_INVAL, "y must not alias x");
  for (int k = 0; k < D - 1; ++k)
    if (y->nrow[k] != x->nrow[k]) return fail(QTT_E_SHAPE, "modes differ");
  const int r1 = x->ranks[D - 1];
  if (r1 > 1024) return fail(QTT_E_UNSUPPORTED, "qtt_tt_contract_last: last bond rank <= 1024");
  int64_t off = 0, need = 0;
  std::vector<int64_t> xoff(D);
  for (int k = 0; k < D; ++k) {
    xoff[k] = off;
    off += (int64_t)x->ranks[k] * x->nrow[k] * x->ranks[k + 1];
  }
  for (int k = 0; k < D - 2; ++k) need += (int64_t)x->ranks[k] * x->nrow[k] * x->ranks[k + 1];
  const int r0 = x->ranks[D - 2], n = x->nrow[D - 2], nl = x->nrow[D - 1];
  need += (int64_t)r0 * n;
  if (need > y->capacity) return fail(QTT_E_CAPACITY, "y: capacity " + std::to_string(y->capacity) +
                                                          " < " + std::to_string(need));
  hipStream_t s = (hipStream_t)stream;
  if (xoff[D - 2] > 0)
    QTT_HIP(hipMemcpyAsync(y->data, x->data, sizeof(double) * xoff[D - 2],
                           hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_contract_last, dim3(1), dim3(256), 0, s,
                     (const double *)x->data + xoff[D - 2], (const double *)x->data + xoff[D - 1],
                     w, y->data + xoff[D - 2], r0, n, r1, nl);
  QTT_HIP(hipGetLastError());
  for (int k = 0; k < D - 1; ++k) y->ranks[k] = x->ranks[k];
  y->ranks[D - 1] = 1;
  QTT_HIP(publish_ranks(y, s));
  return QTT_OK;
}

extern "C" qtt_status qtt_tt_align(qtt_tt *x, const qtt_tt *ref, void *stream) {
  qtt::clear_stale_error();
  qtt_status st;
  if ((st = check_tt(x, "x", true)) != QTT_OK) return st;
  if ((st = check_tt(ref, "ref", true)) != QTT_OK) return st;
  if (x->ncol || ref->ncol) return fail(QTT_E_INVAL, "qtt_tt_align takes TT vectors");
  const int D = x->ncores;
  if (D < 2 || D > QTT_MAXD) return fail(QTT_E_UNSUPPORTED, "qtt_tt_align: 2..QTT_MAXD cores");
  if (ref->ncores != D) return fail(QTT_E_SHAPE, "core counts differ");
  if (x->data == ref->data) return fail(QTT_E_INVAL, "x must not alias ref");
  AlignArg a;
  a.D = D;
  int64_t off = 0;
  for (int k = 0; k < D; ++k) {
    if (x->nrow[k] != ref->nrow[k]) return fail(QTT_E_SHAPE, "modes differ");
    a.n[k] = x->nrow[k];
    a.off[k] = off;
    off += (int64_t)x->ranks[k] * x->nrow[k] * x->ranks[k + 1];
  }
  for (int k = 0; k <= D; ++k) {
    if (x->ranks[k] != ref->ranks[k]) return fail(QTT_E_SHAPE, "ranks differ");
    if (x->ranks[k] > ALIGN_RMAX)
      return fail(QTT_E_UNSUPPORTED, "qtt_tt_align: ranks up to " + std::to_string(ALIGN_RMAX));
    a.r[k] = x->ranks[k];
  }
  hipLaunchKernelGGL(k_align, dim3(1), dim3(256), 0, (hipStream_t)stream, x->data,
                     (const double *)ref->data, a);
  QTT_HIP(hipGetLastError());
  return QTT_OK;
}

extern "C" qtt_status qtt_tt_combine(int32_t nterms, const double *coeffs, const qtt_tt *const *x,
                                     qtt_tt *z, void *stream) {
  qtt::clear_stale_error();
  if (nterms < 1 || !coeffs || !x) return fail(QTT_E_INVAL, "nterms >= 1, coeffs and x required");
  qtt_status st;
  for (int i = 0; i < nterms; ++i) {
    if ((st = check_tt(x[i], "x[i]", true)) != QTT_OK) return st;
    if (x[i]->ncol) return fail(QTT_E_INVAL, "x[i] must be vectors");
  }
  if (!z || !z->ranks || !z->data || !z->nrow) return fail(QTT_E_INVAL, "z: NULL field");
  const int D = x[0]->ncores;
  if (D < 2) return fail(QTT_E_UNSUPPORTED, "qtt_tt_combine needs at least two cores");
  if (z->ncores != D) return fail(QTT_E_SHAPE, "core counts differ");
  for (int i = 0; i < nterms; ++i) {
    if (x[i]->ncores != D) return fail(QTT_E_SHAPE, "core counts differ");
    if (x[i]->data == z->data) return fail(QTT_E_INVAL, "z must not alias a term");
    for (int k = 0; k < D; ++k)
      if (x[i]->nrow[k] != x[0]->nrow[k] || z->nrow[k] != x[0]->nrow[k])
        return fail(QTT_E_SHAPE, "modes differ");
  }
  std::vector<int> zr(D + 1, 0);
  zr[0] = zr[D] = 1;
  for (int k = 1; k < D; ++k) {
    int64_t sum = 0;
    for (int i = 0; i < nterms; ++i) sum += x[i]->ranks[k];
    if (sum > (1 << 20)) return fail(QTT_E_SHAPE, "summed rank beyond 2^20");
    zr[k] = (int)sum;
  }
  for (int k = 0; k <= D; ++k) z->ranks[k] = zr[k];
  int64_t need = 0;
  std::vector<int64_t> zoff(D);
  for (int k = 0; k < D; ++k) {
    zoff[k] = need;
    need += (int64_t)zr[k] * z->nrow[k] * zr[k + 1];
  }
  if (need > z->capacity) return fail(QTT_E_CAPACITY, "z: capacity " + std::to_string(z->capacity) +
                                                          " < " + std::to_string(need));
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero, dim3((int)std::min<int64_t>((need + 255) / 256, 4096)), dim3(256), 0, s,
                     z->data, need);
  QTT_HIP(hipGetLastError());
  std::vector<int> off(D + 1, 0);   // running block offsets per bond
  for (int i = 0; i < nterms; ++i) {
    PlaceArg a;
    a.D = D;
    int64_t xo = 0, mx = 1;
    for (int k = 0; k < D; ++k) {
      a.n[k] = x[i]->nrow[k];
      a.xoff[k] = xo;
      a.zoff[k] = zoff[k];
      const int64_t ce = (int64_t)x[i]->ranks[k] * a.n[k] * x[i]->ranks[k + 1];
      xo += ce;
      mx = ce > mx ? ce : mx;
    }
    for (int k = 0; k <= D; ++k) {
      a.r[k] = x[i]->ranks[k];
      a.zr[k] = zr[k];
      a.o[k] = (k == 0 || k == D) ? 0 : off[k];
    }
    const int blocks = (int)std::min<int64_t>((mx + 255) / 256, 1024);
    hipLaunchKernelGGL(k_place, dim3(blocks, D), dim3(256), 0, s, (const double *)x[i]->data,
                       z->data, a, coeffs[i]);
    QTT_HIP(hipGetLastError());
    for (int k = 1; k < D; ++k) off[k] += x[i]->ranks[k];
  }
  QTT_HIP(publish_ranks(z, s));
  return QTT_OK;
}
