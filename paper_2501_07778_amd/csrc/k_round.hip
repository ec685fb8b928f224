// k_round.hip — TT rounding (the cited rounding algorithm) on gfx950.
//
// Left-to-right: for k = 0..D-2 the left unfolding of core k (rows = rank *
// mode, columns = right rank) is factored by Householder QR, Q becomes the
// new left-orthogonal core and R is multiplied into core k+1 ("absorb").
// The norm of the tensor is then the Frobenius norm of the last core.
// Right-to-left: for k = D-1..1 the right unfolding of core k is split by a
// one-sided Jacobi SVD; the smallest rank whose discarded tail satisfies
// sqrt(sum sigma_i^2) <= eps ||y|| / sqrt(D-1), capped at rmax, is kept;
// V^T becomes the right-orthogonal core k and U Sigma is multiplied into
// core k-1 ("fold").
//
// Ranks live on the device: nr[] holds the ranks after the QR sweep and
// fr[] the final ranks, both in the integer workspace, so the whole sweep
// is a fixed sequence of launches with no host round trip.  The QR and SVD
// steps of one core run in one workgroup; the GEMMs of absorb and fold use
// the whole chip.
#include "dev_gemm.h"
#include "dev_qr.h"
#include "dev_reduce.h"
#include "internal.h"

namespace qtt {

namespace {

constexpr int WG = 1024;           // threads of the one-workgroup kernels
constexpr int NWAVE = WG / 64;
constexpr int JACOBI_MAX_SWEEPS = 40;
constexpr int GL = 16;             // lanes per column pair in the Jacobi sweeps
constexpr int NGRP = WG / GL;
// LDS-resident variants hold the whole working set of one step (matrix and
// its second factor) in 150 KiB of LDS
constexpr int LDS_DBL = 19200;
constexpr int LDS_TAU = 160;       // min(rows, cols) <= sqrt(LDS_DBL)
// the SVD step keeps nothing else in LDS but the Jacobi column norms, so its
// array can take 156 KiB
constexpr int LDS_SVD = 20000;
constexpr int YREG = 13;          // Y elements per thread staged in registers (wide SVD step)
constexpr int JNRM = 160;          // columns whose squared norms the Jacobi tracks

// sums over a wavefront (every lane active): DPP row moves, dev_reduce.h
__device__ __forceinline__ double wave_sum(double v) { return dev::wave64_sum(v); }

// block-wide sum; `red` holds NWAVE doubles of LDS
__device__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NWAVE; ++i) t += red[i];
  return t;
}

// integer workspace layout
struct IW {
  int *nr;    // D+1 ranks after the QR sweep
  int *fr;    // D+1 final ranks
  int *perm;  // singular value order
};
__device__ __forceinline__ IW iw_of(int *iwork, int D) {
  IW w;
  w.nr = iwork;
  w.fr = iwork + (D + 1);
  w.perm = iwork + 2 * (D + 1);
  return w;
}

__global__ void k_round_init(TTView x, int *iwork, double *scal) {
  IW w = iw_of(iwork, x.D);
  const int t = threadIdx.x;
  if (t <= x.D) {
    w.nr[t] = x.rk[t];
    w.fr[t] = x.rk[t];
  }
  if (t == 0) {
    scal[0] = 0.0;  // norm
    scal[1] = 0.0;  // sum of discarded sigma^2
  }
}

// carry <- last core (input already left-orthogonal: no QR sweep)
__global__ void k_last_to_carry(TTView x, double *carry) {
  const int D = x.D;
  if (x.rk[D - 1] > x.cap[D - 1]) return;
  const int64_t ne = (int64_t)x.rk[D - 1] * x.n[D - 1] * x.m[D - 1];
  const double *c = x.data + x.off[D - 1];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x)
    carry[e] = c[e];
}

// Householder QR, Q and products with Q: dev_qr.h (LAPACK's reflector
// convention, one workgroup barrier per column)
using dev::apply_q;
using dev::form_q_inplace;
using dev::householder_qr;

// Left sweep, core k: QR of the left unfolding (rows = nr[k]*nm_k,
// cols = rk[k+1]); Q -> slot k, R -> rbuf (ld = r'), nr[k+1] = r'.  The LDS
// variant factors in LDS and forms Q there before writing it out.
template <bool LDS>
__global__ void __launch_bounds__(WG)
    k_qr_step(TTView x, int k, const double *src, double *work, double *rbuf,
              double *tau_g, int *iwork) {
  __shared__ double lds[LDS ? LDS_DBL : 1];
  __shared__ double tau_l[LDS ? LDS_TAU : 1];
  IW w = iw_of(iwork, x.D);
  const int nm = x.n[k] * x.m[k];
  const int rows = w.nr[k] * nm;
  const int cols = x.rk[k + 1];
  const int rq = rows < cols ? rows : cols;
  if (w.nr[k] > x.cap[k] || cols > x.cap[k + 1]) return;  // ranks beyond the slots
  const bool use_lds = LDS && (int64_t)rows * cols <= LDS_DBL && rq <= LDS_TAU;
  double *W = use_lds ? lds : work;
  double *tau = use_lds ? tau_l : tau_g;
  for (int64_t e = threadIdx.x; e < (int64_t)rows * cols; e += WG) W[e] = src[e];
  __syncthreads();
  householder_qr<NWAVE>(W, rows, cols, tau);
  // R: rq x cols, upper trapezoid
  for (int64_t e = threadIdx.x; e < (int64_t)rq * cols; e += WG) {
    const int i = (int)(e % rq), c = (int)(e / rq);
    rbuf[e] = (i <= c) ? W[i + (int64_t)rows * c] : 0.0;
  }
  // Q in place of the reflectors, then out to slot k
  form_q_inplace<NWAVE>(W, rows, rq, tau);
  double *slot = x.data + x.off[k];
  for (int64_t e = threadIdx.x; e < (int64_t)rows * rq; e += WG) slot[e] = W[e];
  if (threadIdx.x == 0) w.nr[k + 1] = rq;
}

// Column-major FP64 GEMM tiles of dev_gemm.h (64 x 64 per 256-thread block)
using dev::GT;
using dev::gemm_tile;

// absorb: carry (nr[k+1] x nm_{k+1} rk[k+2]) = R (nr[k+1] x rk[k+1]) *
// slot k+1 (rk[k+1] x nm_{k+1} rk[k+2])
__global__ void __launch_bounds__(256)
    k_absorb(TTView x, int k, const double *rbuf, double *carry, int *iwork) {
  IW w = iw_of(iwork, x.D);
  const int M = w.nr[k + 1];
  const int K = x.rk[k + 1];
  const int N = x.n[k + 1] * x.m[k + 1] * x.rk[k + 2];
  if (M > x.cap[k + 1] || K > x.cap[k + 1] || x.rk[k + 2] > x.cap[k + 2]) return;
  if (blockIdx.x * GT >= M || blockIdx.y * GT >= N) return;
  gemm_tile<false>(rbuf, M, x.data + x.off[k + 1], K, carry, M, M, N, K, blockIdx.x,
                   blockIdx.y);
}

// fold: carry ((nr[k-1] nm_{k-1}) x fr[k]) = slot k-1 ((nr[k-1] nm) x nr[k])
// * F (nr[k] x fr[k])
__global__ void __launch_bounds__(256)
    k_fold(TTView x, int k, const double *F, double *carry, int *iwork) {
  IW w = iw_of(iwork, x.D);
  const int M = w.nr[k - 1] * x.n[k - 1] * x.m[k - 1];
  const int K = w.nr[k];
  const int N = w.fr[k];
  if (w.nr[k - 1] > x.cap[k - 1] || K > x.cap[k] || N > x.cap[k]) return;
  if (blockIdx.x * GT >= M || blockIdx.y * GT >= N) return;
  gemm_tile<false>(x.data + x.off[k - 1], M, F, K, carry, M, M, N, K, blockIdx.x,
                   blockIdx.y);
}

// norm of the last core after the QR sweep
__global__ void __launch_bounds__(WG)
    k_last_norm(TTView x, const double *carry, int *iwork, double *scal) {
  __shared__ double red[NWAVE];
  IW w = iw_of(iwork, x.D);
  const int D = x.D;
  const int64_t ne = (int64_t)w.nr[D - 1] * x.n[D - 1] * x.m[D - 1];
  double p = 0.0;
  for (int64_t e = threadIdx.x; e < ne; e += WG) p += carry[e] * carry[e];
  p = block_sum(p, red);
  if (threadIdx.x == 0) scal[0] = sqrt(p);
}

// Sum over the 16 lanes of a group (GL = 16: a group is one DPP row).
__device__ __forceinline__ double group_sum(double v) {
  static_assert(GL == 16, "group_sum reduces one 16-lane DPP row");
  return dev::row16_sum(v);
}

using dev::rcp_nr;
using dev::rsq_nr;

// The Jacobi rotation of a column pair with squared norms al, be and inner
// product ga: rotate when |ga| > tol sqrt(al be) (tested with the hardware
// reciprocal square root estimates: the threshold needs no precision);
// then zeta = (be - al) / (2 ga), t = sign(zeta) / (|zeta| + sqrt(1 +
// zeta^2)) (the smaller root of t^2 + 2 zeta t - 1 = 0), c = 1 / sqrt(1 +
// t^2), s = c t.  Only c must be accurate (c^2 + s^2 = 1 to rounding
// whatever t is): it takes two Newton steps, zeta and t one (t to about 46
// bits, which only steers the rotation); |zeta| beyond 5e149 gives t = 1 /
// (2 zeta) and a ga below 1e-290 the IEEE chain.
__device__ __forceinline__ bool jac_angle(double al, double be, double ga, double tol, double &c,
                                          double &sn, double &t) {
  if (!(ga != 0.0 &&
        fabs(ga) * (__builtin_amdgcn_rsq(al) * __builtin_amdgcn_rsq(be)) > tol))
    return false;
  const double d = be - al;
  if (fabs(d) > 1e150 * fabs(ga)) {
    t = ga / d;
  } else if (fabs(ga) >= 1e-290) {
    const double zeta = 0.5 * d * rcp_nr<1>(ga);
    const double h = fma(zeta, zeta, 1.0);
    t = copysign(rcp_nr<1>(fabs(zeta) + h * rsq_nr<1>(h)), zeta >= 0.0 ? 1.0 : -1.0);
  } else {
    const double zeta = d / (2.0 * ga);
    t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  }
  c = rsq_nr<2>(fma(t, t, 1.0));
  sn = c * t;
  return true;
}

// One-sided Jacobi (Hestenes) on the columns of B (mb x nb, ld = mb) with V
// (nb x nb) accumulated: B V has mutually orthogonal columns.  Round-robin
// ordering: each round pairs all columns disjointly, one 16-lane group per
// pair.  A pair is rotated while |b_p . b_q| > tol ||b_p|| ||b_q||; since V
// stays orthogonal, B_in = (B V) V^T holds whatever tol is, and columns
// dropped later contribute exactly their norms to the truncation error.
// Up to JNRM columns the squared norms are computed once per sweep and then
// carried through the rotations (the rotation that zeroes b_p . b_q = g with
// tangent t maps them to al - t g and be + t g, as in Hestenes' method), so
// a pair needs one reduction instead of three; a norm that the update would
// shrink below a quarter is recomputed.  The norms only steer the angles:
// every rotation is exact, so B V V^T = B_in holds regardless.
__device__ int jacobi(double *B, int mb, int nb, double *V, double *rot_log, int *flag,
                      double tol) {
  __shared__ double cn[JNRM];
  const bool track = nb <= JNRM;
  const int gl = threadIdx.x % GL, grp = threadIdx.x / GL;
  if (V)
    for (int64_t e = threadIdx.x; e < (int64_t)nb * nb; e += WG)
      V[e] = ((e % nb) == (e / nb)) ? 1.0 : 0.0;
  const int N = nb + (nb & 1);
  int sweeps = 0;
  for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
    __syncthreads();
    if (threadIdx.x == 0) *flag = 0;
    if (track) {
      for (int j = grp; j < nb; j += NGRP) {
        const double *bj = B + (int64_t)mb * j;
        double sacc = 0.0;
        for (int l = gl; l < mb; l += GL) sacc = fma(bj[l], bj[l], sacc);
        sacc = group_sum(sacc);
        if (gl == 0) cn[j] = sacc;
      }
    }
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      double *lg = rot_log ? rot_log + 2 * ((int64_t)(sweep * (N - 1) + r) * (N / 2)) : nullptr;
      // every group runs the same number of passes (idle groups sum zeros)
      for (int i0 = 0; i0 < N / 2; i0 += NGRP) {
        const int i = i0 + grp;
        int p = (r + i) % (N - 1);
        int q = (i == 0) ? (N - 1) : (r - i + N - 1) % (N - 1);
        const bool act = i < N / 2 && p < nb && q < nb;
        if (p > q) { int t = p; p = q; q = t; }
        double *bp = B + (int64_t)mb * (act ? p : 0), *bq = B + (int64_t)mb * (act ? q : 0);
        double al = 0.0, be = 0.0, ga = 0.0;
        if (track) {
          if (act)
            for (int l = gl; l < mb; l += GL) ga = fma(bp[l], bq[l], ga);
          ga = group_sum(ga);
          if (act) {
            al = cn[p];
            be = cn[q];
          }
        } else {
          if (act) {
            for (int l = gl; l < mb; l += GL) {
              const double u = bp[l], v = bq[l];
              al = fma(u, u, al);
              be = fma(v, v, be);
              ga = fma(u, v, ga);
            }
          }
          al = group_sum(al);
          be = group_sum(be);
          ga = group_sum(ga);
        }
        double c = 1.0, sn = 0.0, t = 0.0;
        if (act && jac_angle(al, be, ga, tol, c, sn, t)) {
          double np = 0.0, nq = 0.0;
          for (int l = gl; l < mb; l += GL) {
            const double u = bp[l], v = bq[l];
            const double u2 = c * u - sn * v, v2 = sn * u + c * v;
            bp[l] = u2;
            bq[l] = v2;
            np = fma(u2, u2, np);
            nq = fma(v2, v2, nq);
          }
          if (track) {
            double ap = al - t * ga, aq = be + t * ga;
            // cancellation: measure instead (uniform over the group)
            if (!(ap >= 0.25 * al) || !(aq >= 0.25 * be)) {
              ap = group_sum(np);
              aq = group_sum(nq);
            }
            if (gl == 0) {
              cn[p] = ap;
              cn[q] = aq;
            }
          }
          if (V) {
            double *vp = V + (int64_t)nb * p, *vq = V + (int64_t)nb * q;
            for (int l = gl; l < nb; l += GL) {
              const double u = vp[l], v = vq[l];
              vp[l] = c * u - sn * v;
              vq[l] = sn * u + c * v;
            }
          }
          if (gl == 0) *flag = 1;
        }
        if (lg && gl == 0 && i < N / 2) {
          lg[2 * i] = c;
          lg[2 * i + 1] = sn;
        }
      }
      __syncthreads();
    }
    sweeps = sweep + 1;
    __syncthreads();
    if (*flag == 0) break;
  }
  __syncthreads();
  return sweeps;
}

// One Jacobi rotation of the column pair (xp, xq) held by a 16-lane group
// (K rows per lane) together with the same columns of V (vp, vq); al and be
// are the columns' squared norms, carried through the rotation.  The test
// and the angle are those of jacobi(); every value is uniform over the
// group.  Returns whether the pair was rotated.
template <int K>
__device__ __forceinline__ bool jac_pair(double (&xp)[K], double (&xq)[K], double (&vp)[K],
                                         double (&vq)[K], double &al, double &be, bool act,
                                         double tol) {
  double g0 = 0.0, g1 = 0.0;
#pragma unroll
  for (int k = 0; k < K; k += 2) g0 = fma(xp[k], xq[k], g0);
#pragma unroll
  for (int k = 1; k < K; k += 2) g1 = fma(xp[k], xq[k], g1);
  const double ga = group_sum(g0 + g1);
  double c, sn, t;
  if (!(act && jac_angle(al, be, ga, tol, c, sn, t))) return false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double u = xp[k], v = xq[k];
    xq[k] = fma(sn, u, c * v);
    xp[k] = fma(c, u, -(sn * v));
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double u = vp[k], v = vq[k];
    vq[k] = fma(sn, u, c * v);
    vp[k] = fma(c, u, -(sn * v));
  }
  double ap = al - t * ga, aq = be + t * ga;
  if (!(ap >= 0.25 * al) || !(aq >= 0.25 * be)) {
    // cancellation: measure instead (uniform over the group)
    double np = 0.0, nq = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      np = fma(xp[k], xp[k], np);
      nq = fma(xq[k], xq[k], nq);
    }
    ap = group_sum(np);
    aq = group_sum(nq);
  }
  al = ap;
  be = aq;
  return true;
}

// exchange of a group's column (registers of B and V, norm and index) with
// the group whose lanes differ in bit 4 (MASK 16) or bit 5 (MASK 32)
template <int K, int MASK>
__device__ __forceinline__ void jac_swap(double (&x)[K], double (&v)[K], double &nrm, int &col) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    x[k] = __shfl_xor(x[k], MASK);
    v[k] = __shfl_xor(v[k], MASK);
  }
  nrm = __shfl_xor(nrm, MASK);
  col = __shfl_xor(col, MASK);
}

// Block-cyclic one-sided Jacobi on B (mb x nb, ld mb) with V (nb x nb, ld
// nb) accumulated, for mb, nb <= 16 K; the result has the properties stated
// for jacobi().  The columns form blocks of four.  The blocks meet in
// round-robin order, one block pair per wavefront and a workgroup barrier
// per block round; within a pair each 16-lane group holds one column of
// each block, and of V, in registers (rows gl + 16 k).  The four pairings
// of the two blocks' columns take four inner rounds, between which the
// second block's columns pass to another group by lane exchanges (bit 4,
// bit 5, bit 4 of the lane index), so the inner rounds touch no LDS.  The
// six pairs inside each block are rotated in the first block round of each
// sweep (three rounds, two pairs per block).  Every column pair is visited
// once per sweep, as in the cyclic order.
template <int K>
__device__ __forceinline__ int jacobi_blk(double *B, int mb, int nb, double *V, int *flag,
                                           double tol) {
  const int gl = threadIdx.x & 15, g = (threadIdx.x >> 4) & 3, wave = threadIdx.x >> 6;
  for (int64_t e = threadIdx.x; e < (int64_t)nb * nb; e += WG)
    V[e] = ((e % nb) == (e / nb)) ? 1.0 : 0.0;
  const int nblk = (nb + 3) / 4, NB = nblk + (nblk & 1);
  // loads read an in-bounds element for every lane (the last row or column
  // instead of one past the end) and zero what lies outside
  auto load = [&](double (&x)[K], double (&v)[K], int c) {
    const bool in = c < nb;
    const int cc = in ? c : nb - 1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int l = gl + GL * k;
      const double bx = B[(l < mb ? l : mb - 1) + (int64_t)mb * cc];
      const double vx = V[(l < nb ? l : nb - 1) + (int64_t)nb * cc];
      x[k] = (in && l < mb) ? bx : 0.0;
      v[k] = (in && l < nb) ? vx : 0.0;
    }
  };
  auto store = [&](const double (&x)[K], const double (&v)[K], int c) {
    if (c >= nb) return;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int l = gl + GL * k;
      if (l < mb) B[l + (int64_t)mb * c] = x[k];
      if (l < nb) V[l + (int64_t)nb * c] = v[k];
    }
  };
  auto sqnorm = [&](const double (&x)[K]) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) s = fma(x[k], x[k], s);
    return group_sum(s);
  };
  int sweeps = 0;
  for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
    __syncthreads();
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    bool rotated = false;
    for (int r = 0; r < NB - 1; ++r) {
      for (int i = wave; i < NB / 2; i += NWAVE) {
        int a = (r + i) % (NB - 1);
        int b = (i == 0) ? (NB - 1) : (r - i + NB - 1) % (NB - 1);
        if (a > b) { const int t = a; a = b; b = t; }
        double xp[K], xq[K], vp[K], vq[K];
        if (r == 0) {
          // pairs inside blocks a (groups 0, 1) and b (groups 2, 3): (0,1)
          // (2,3), then (0,2) (1,3), then (0,3) (1,2)
          const int h = g & 1, base = 4 * ((g < 2) ? a : b);
          int cp = base + 2 * h, cq = cp + 1;
          load(xp, vp, cp);
          load(xq, vq, cq);
          double al = sqnorm(xp), be = sqnorm(xq);
          rotated |= jac_pair<K>(xp, xq, vp, vq, al, be, cq < nb, tol);
          // group h = 0 passes its second column, h = 1 its first
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const double xr = __shfl_xor(h ? xp[k] : xq[k], 16);
            const double vr = __shfl_xor(h ? vp[k] : vq[k], 16);
            if (h) { xp[k] = xr; vp[k] = vr; } else { xq[k] = xr; vq[k] = vr; }
          }
          {
            const double nr = __shfl_xor(h ? al : be, 16);
            const int cr = __shfl_xor(h ? cp : cq, 16);
            if (h) { al = nr; cp = cr; } else { be = nr; cq = cr; }
          }
          rotated |= jac_pair<K>(xp, xq, vp, vq, al, be, cp < nb && cq < nb, tol);
          jac_swap<K, 16>(xq, vq, be, cq);
          rotated |= jac_pair<K>(xp, xq, vp, vq, al, be, cp < nb && cq < nb, tol);
          store(xp, vp, cp);
          store(xq, vq, cq);
          // the same wavefront reads these columns back below (in order)
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        if (b < nblk) {
          int cp = 4 * a + g, cq = 4 * b + g;
          load(xp, vp, cp);
          load(xq, vq, cq);
          double al = sqnorm(xp), be = sqnorm(xq);
          rotated |= jac_pair<K>(xp, xq, vp, vq, al, be, cp < nb && cq < nb, tol);
          jac_swap<K, 16>(xq, vq, be, cq);
          rotated |= jac_pair<K>(xp, xq, vp, vq, al, be, cp < nb && cq < nb, tol);
          jac_swap<K, 32>(xq, vq, be, cq);
          rotated |= jac_pair<K>(xp, xq, vp, vq, al, be, cp < nb && cq < nb, tol);
          jac_swap<K, 16>(xq, vq, be, cq);
          rotated |= jac_pair<K>(xp, xq, vp, vq, al, be, cp < nb && cq < nb, tol);
          store(xp, vp, cp);
          store(xq, vq, cq);
        }
      }
      __syncthreads();
    }
    if (rotated && gl == 0) *flag = 1;
    __syncthreads();
    sweeps = sweep + 1;
    if (*flag == 0) break;
  }
  __syncthreads();
  return sweeps;
}

// V (nb x nb) = product of the logged rotations, replayed in the order of
// the sweeps: identical to accumulating them during the sweeps.
__device__ void jacobi_replay(double *V, int nb, const double *rot_log, int sweeps) {
  const int gl = threadIdx.x % GL, grp = threadIdx.x / GL;
  for (int64_t e = threadIdx.x; e < (int64_t)nb * nb; e += WG)
    V[e] = ((e % nb) == (e / nb)) ? 1.0 : 0.0;
  const int N = nb + (nb & 1);
  __syncthreads();
  for (int sweep = 0; sweep < sweeps; ++sweep) {
    for (int r = 0; r < N - 1; ++r) {
      const double *lg = rot_log + 2 * ((int64_t)(sweep * (N - 1) + r) * (N / 2));
      for (int i = grp; i < N / 2; i += NGRP) {
        int p = (r + i) % (N - 1);
        int q = (i == 0) ? (N - 1) : (r - i + N - 1) % (N - 1);
        if (p >= nb || q >= nb) continue;
        if (p > q) { int t = p; p = q; q = t; }
        const double c = lg[2 * i], sn = lg[2 * i + 1];
        if (sn == 0.0 && c == 1.0) continue;
        double *vp = V + (int64_t)nb * p, *vq = V + (int64_t)nb * q;
        for (int l = gl; l < nb; l += GL) {
          const double u = vp[l], v = vq[l];
          vp[l] = c * u - sn * v;
          vq[l] = sn * u + c * v;
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ double jacobi_tol(double eps, int mb) {
  const double floor = 1e-15 * sqrt((double)mb);
  const double t = fmin(1e-2 * eps, 1e-6);
  return t > floor ? t : floor;
}

// Truncation after the Jacobi sweeps: sigma_j = ||(B V)_j||, descending
// order by parallel ranking, smallest rank with discarded tail <= delta,
// capped at rmax.  Shared by the LDS and global variants.
__device__ int truncate_rank(const double *Bv, int mb, int nb, double *sig, int *perm,
                             double delta, int rmax, double *scal, int *rank_s) {
  for (int j = threadIdx.x / 64; j < nb; j += NWAVE) {
    const double *bj = Bv + (int64_t)mb * j;
    double sacc = 0.0;
    for (int l = threadIdx.x & 63; l < mb; l += 64) sacc = fma(bj[l], bj[l], sacc);
    sacc = wave_sum(sacc);
    if ((threadIdx.x & 63) == 0) sig[j] = sqrt(sacc);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nb; j += WG) {
    const double sj = sig[j];
    int pos = 0;
    for (int i = 0; i < nb; ++i) {
      const double si = sig[i];
      pos += (si > sj || (si == sj && i < j)) ? 1 : 0;
    }
    perm[pos] = j;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tail2 = 0.0;
    int rank = nb;
    for (int j = nb - 1; j >= 0; --j) {
      const double sj = sig[perm[j]];
      if (sqrt(tail2 + sj * sj) <= delta) {
        tail2 += sj * sj;
        rank = j;
      } else {
        break;
      }
    }
    if (rank < 1) rank = 1;
    if (rmax > 0 && rank > rmax) rank = rmax;
    double disc = 0.0;
    for (int j = rank; j < nb; ++j) disc += sig[perm[j]] * sig[perm[j]];
    scal[1] += disc;
    *rank_s = rank;
  }
  __syncthreads();
  return *rank_s;
}

// Write the new right-orthogonal core and the fold operand from B V = W
// (tall: B = M) or B = M^T (wide).
__device__ void svd_outputs(bool tall, const double *Wb, const double *V, int mb, int nb,
                            int r0, int nc, int rank, const double *sig, const int *perm,
                            double *core, double *F) {
  if (tall) {
    for (int64_t e = threadIdx.x; e < (int64_t)r0 * rank; e += WG) {
      const int a = (int)(e % r0), l = (int)(e / r0);
      F[e] = Wb[a + (int64_t)mb * perm[l]];
    }
    for (int64_t e = threadIdx.x; e < (int64_t)rank * nc; e += WG) {
      const int l = (int)(e % rank), col = (int)(e / rank);
      core[e] = V[col + (int64_t)nb * perm[l]];
    }
  } else {
    for (int64_t e = threadIdx.x; e < (int64_t)r0 * rank; e += WG) {
      const int a = (int)(e % r0), l = (int)(e / r0);
      F[e] = V[a + (int64_t)nb * perm[l]] * sig[perm[l]];
    }
    for (int64_t e = threadIdx.x; e < (int64_t)rank * nc; e += WG) {
      const int l = (int)(e % rank), col = (int)(e / rank);
      const double sv = sig[perm[l]];
      core[e] = (sv > 0.0) ? Wb[col + (int64_t)mb * perm[l]] / sv : ((col == l) ? 1.0 : 0.0);
    }
  }
}

// Right sweep, core k: SVD of the right unfolding M (r0 = nr[k] rows,
// nc = nm_k * fr[k+1] columns) held in `carry`; writes the right-orthogonal
// core to slot k, the fold operand F (r0 x rank) and fr[k] = rank.  The LDS
// variant keeps B and V in LDS (the host picks it when the caps fit).
template <bool LDS>
__global__ void __launch_bounds__(WG)
    k_svd_step(TTView x, int k, double eps, int rmax, const double *carry,
               double *work, double *vbuf, double *F, double *sig,
               int *iwork, double *scal, double *rot_log) {
  __shared__ int flag;
  __shared__ int rank_s;
  __shared__ double lds[LDS ? LDS_SVD : 1];
  __shared__ double tau_s[LDS ? LDS_TAU : 1];
  IW w = iw_of(iwork, x.D);
  const int D = x.D;
  const int nm = x.n[k] * x.m[k];
  const int r0 = w.nr[k];
  const int nc = nm * w.fr[k + 1];
  const bool tall = r0 >= nc;
  const int mb = tall ? r0 : nc, nb = tall ? nc : r0;
  if (r0 > x.cap[k] || w.fr[k + 1] > x.cap[k + 1]) return;  // ranks beyond the slots
  const double delta0 = (D > 1) ? eps * scal[0] / sqrt((double)(D - 1)) : 0.0;
  double *core0 = x.data + x.off[k];
  if (LDS && !tall && (int64_t)mb * nb + 2 * (int64_t)nb * nb <= LDS_SVD && nb <= LDS_TAU) {
    // Wide unfolding M (r0 x nc): QR of B = M^T = Q R, one-sided Jacobi on
    // X = R^T (r0 x r0) with X V = W, so M = W (Q V)^T.  The kept core rows
    // (Q V)^T are orthonormal for any Jacobi tolerance (V is a product of
    // rotations), which allows the same loose tolerance as the tall case,
    // and the Jacobi works on r0-long instead of nc-long columns.
    double *Bq = lds;                        // nc x r0, then R and reflectors
    double *X = lds + (int64_t)mb * nb;      // r0 x r0
    double *Vv = X + (int64_t)nb * nb;       // r0 x r0
    for (int64_t e = threadIdx.x; e < (int64_t)mb * nb; e += WG) {
      const int i = (int)(e % mb), j = (int)(e / mb);
      Bq[e] = carry[j + (int64_t)r0 * i];
    }
    __syncthreads();
    double *tau = tau_s;
    householder_qr<NWAVE>(Bq, mb, nb, tau);
    for (int64_t e = threadIdx.x; e < (int64_t)nb * nb; e += WG) {
      const int i = (int)(e % nb), j = (int)(e / nb);
      X[e] = (j <= i) ? Bq[j + (int64_t)mb * i] : 0.0;  // X[i, j] = R[j, i]
    }
    __syncthreads();
    if (nb <= 80)
      jacobi_blk<5>(X, nb, nb, Vv, &flag, jacobi_tol(eps, nb));
    else
      jacobi_blk<6>(X, nb, nb, Vv, &flag, jacobi_tol(eps, nb));
    const int rank = truncate_rank(X, nb, nb, sig, w.perm, delta0, rmax, scal, &rank_s);
    if (threadIdx.x == 0) w.fr[k] = rank;
    // F = kept columns of W (r0 x rank); Y = Q [V_kept; 0] (nc x rank), in
    // LDS over X and V (staged through registers) when it fits there
    for (int64_t e = threadIdx.x; e < (int64_t)r0 * rank; e += WG) {
      const int a = (int)(e % r0), l = (int)(e / r0);
      F[e] = X[a + (int64_t)nb * w.perm[l]];
    }
    const int64_t ny = (int64_t)mb * rank;
    const bool y_lds = ny <= 2 * (int64_t)nb * nb && ny <= (int64_t)YREG * WG;
    double *Y = y_lds ? X : work;
    if (y_lds) {
      double yv[YREG];
#pragma unroll
      for (int q = 0; q < YREG; ++q) {
        const int64_t e = threadIdx.x + (int64_t)WG * q;
        const int i = (int)(e % mb), l = (int)(e / mb);
        yv[q] = (e < ny && i < nb) ? Vv[i + (int64_t)nb * w.perm[l]] : 0.0;
      }
      __syncthreads();  // X and V are read: Y may take their place
#pragma unroll
      for (int q = 0; q < YREG; ++q) {
        const int64_t e = threadIdx.x + (int64_t)WG * q;
        if (e < ny) Y[e] = yv[q];
      }
    } else {
      for (int64_t e = threadIdx.x; e < ny; e += WG) {
        const int i = (int)(e % mb), l = (int)(e / mb);
        Y[e] = (i < nb) ? Vv[i + (int64_t)nb * w.perm[l]] : 0.0;
      }
    }
    __syncthreads();
    apply_q<NWAVE>(Bq, mb, nb, tau, Y, mb, rank);
    for (int64_t e = threadIdx.x; e < (int64_t)rank * nc; e += WG) {
      const int l = (int)(e % rank), col = (int)(e / rank);
      core0[e] = Y[col + (int64_t)mb * l];
    }
    return;
  }
  // B and V both in LDS, or B in LDS with the rotations logged and replayed
  // onto V in the same LDS afterwards, or both in global memory
  const bool both = LDS && (int64_t)mb * nb + (int64_t)nb * nb <= LDS_DBL;
  const bool replay = LDS && !both && (int64_t)mb * nb <= LDS_DBL &&
                      (int64_t)nb * nb <= LDS_DBL;
  double *B = (both || replay) ? lds : work;
  double *V = both ? lds + (int64_t)mb * nb : (replay ? nullptr : vbuf);
  // B = M (tall) or M^T (wide), column-major mb x nb
  for (int64_t e = threadIdx.x; e < (int64_t)mb * nb; e += WG) {
    const int i = (int)(e % mb), j = (int)(e / mb);
    B[e] = tall ? carry[e] : carry[j + (int64_t)r0 * i];
  }
  __syncthreads();
  // tall: the kept core is V^T, orthogonal for any stopping tolerance; wide:
  // it is built from the columns of B V, which must be orthogonal to FP64
  const double jtol = jacobi_tol(tall ? eps : 0.0, mb);
  int sweeps;
  if (both && mb <= 80 && nb <= 80)
    sweeps = jacobi_blk<5>(B, mb, nb, V, &flag, jtol);
  else if (both && mb <= 96 && nb <= 96)
    sweeps = jacobi_blk<6>(B, mb, nb, V, &flag, jtol);
  else
    sweeps = jacobi(B, mb, nb, V, replay ? rot_log : nullptr, &flag, jtol);
  const double delta = (D > 1) ? eps * scal[0] / sqrt((double)(D - 1)) : 0.0;
  const int rank = truncate_rank(B, mb, nb, sig, w.perm, delta, rmax, scal, &rank_s);
  if (threadIdx.x == 0) w.fr[k] = rank;
  double *core = x.data + x.off[k];
  if (!replay) {
    svd_outputs(tall, B, V, mb, nb, r0, nc, rank, sig, w.perm, core, F);
    return;
  }
  // outputs that need B, then V replayed into the LDS B occupied
  if (tall) {
    for (int64_t e = threadIdx.x; e < (int64_t)r0 * rank; e += WG) {
      const int a = (int)(e % r0), l = (int)(e / r0);
      F[e] = B[a + (int64_t)mb * w.perm[l]];
    }
  } else {
    for (int64_t e = threadIdx.x; e < (int64_t)rank * nc; e += WG) {
      const int l = (int)(e % rank), col = (int)(e / rank);
      const double sv = sig[w.perm[l]];
      core[e] = (sv > 0.0) ? B[col + (int64_t)mb * w.perm[l]] / sv : ((col == l) ? 1.0 : 0.0);
    }
  }
  __syncthreads();
  jacobi_replay(lds, nb, rot_log, sweeps);
  __syncthreads();
  const double *Vl = lds;
  if (tall) {
    for (int64_t e = threadIdx.x; e < (int64_t)rank * nc; e += WG) {
      const int l = (int)(e % rank), col = (int)(e / rank);
      core[e] = Vl[col + (int64_t)nb * w.perm[l]];
    }
  } else {
    for (int64_t e = threadIdx.x; e < (int64_t)r0 * rank; e += WG) {
      const int a = (int)(e % r0), l = (int)(e / r0);
      F[e] = Vl[a + (int64_t)nb * w.perm[l]] * sig[w.perm[l]];
    }
  }
}

// slot 0 <- carry (1 x nm_0 x fr[1]), ranks <- fr
__global__ void k_round_finish(TTView x, const double *carry, int *iwork) {
  IW w = iw_of(iwork, x.D);
  if (w.fr[1] > x.cap[1]) return;
  const int64_t ne = (int64_t)x.n[0] * x.m[0] * w.fr[1];
  double *core = x.data + x.off[0];
  for (int64_t e = threadIdx.x; e < ne; e += blockDim.x) core[e] = carry[e];
  __syncthreads();
  if (threadIdx.x <= x.D) x.rk[threadIdx.x] = w.fr[threadIdx.x];
}

// D == 1: only the norm
__global__ void k_round_single(TTView x, double *scal) {
  __shared__ double red[NWAVE];
  const int64_t ne = (int64_t)x.n[0] * x.m[0];
  double p = 0.0;
  for (int64_t e = threadIdx.x; e < ne; e += WG) p += x.data[e] * x.data[e];
  p = block_sum(p, red);
  if (threadIdx.x == 0) {
    scal[0] = sqrt(p);
    scal[1] = 0.0;
  }
}

int64_t max_slot(const TTView &x) {
  int64_t mx = 1;
  for (int k = 0; k < x.D; ++k) {
    int64_t c = (int64_t)x.cap[k] * x.n[k] * x.m[k] * x.cap[k + 1];
    mx = c > mx ? c : mx;
  }
  return mx;
}

int max_cap(const TTView &x) {
  int mx = 1;
  for (int k = 0; k <= x.D; ++k) mx = x.cap[k] > mx ? x.cap[k] : mx;
  return mx;
}

int max_nm(const TTView &x) {
  int mx = 1;
  for (int k = 0; k < x.D; ++k) mx = x.n[k] * x.m[k] > mx ? x.n[k] * x.m[k] : mx;
  return mx;
}

}  // namespace

int64_t round_ws_bytes(const TTView &x) {
  Arena ar;
  ar.dry = true;
  RoundWs w;
  round_ws_take(ar, x, w);
  return (int64_t)ar.used;
}

bool round_ws_take(Arena &ar, const TTView &x, RoundWs &w) {
  const int64_t slot = max_slot(x);
  const int64_t cap = max_cap(x);
  const int64_t nm = max_nm(x);
  // work holds the QR step's (r n m) x r' block and the SVD step's unfolding
  // (or its transpose) or the wide case's r' x rank product, each at most
  // the largest slot; the Jacobi V (at most cap x cap) lives in vbuf
  w.carry_elems = slot;
  w.sq_elems = slot;
  w.carry = (double *)ar.take(sizeof(double) * slot);
  w.work = (double *)ar.take(sizeof(double) * slot);
  w.rbuf = (double *)ar.take(sizeof(double) * cap * cap);
  w.vbuf = (double *)ar.take(sizeof(double) * cap * cap);
  w.fold = (double *)ar.take(sizeof(double) * cap * cap * nm);
  w.scal = (double *)ar.take(sizeof(double) * (4 + 2 * nm * cap));
  w.iwork = (int *)ar.take(sizeof(int) * (2 * (x.D + 1) + nm * cap + 8));
  // Jacobi rotation log: (c, s) for every pair of every round of every sweep
  // for matrices up to the LDS size (nb <= 138 columns)
  const int64_t nbl = 140;
  w.rotlog = (double *)ar.take(sizeof(double) * 2 * JACOBI_MAX_SWEEPS * nbl * (nbl / 2));
  return ar.ok();
}

hipError_t round_tt(const TTView &x, double eps, int rmax, const RoundWs &w,
                    hipStream_t s, bool left_orth, int rank_bound) {
  // the kernel variants are chosen from bounds on the ranks: the slot caps,
  // tightened by rank_bound when the caller knows one
  auto cap_of = [&](int k) {
    return (rank_bound > 0 && rank_bound < x.cap[k]) ? rank_bound : x.cap[k];
  };
  const int D = x.D;
  if (D == 1) {
    hipLaunchKernelGGL(k_round_single, dim3(1), dim3(WG), 0, s, x, w.scal);
    return hipGetLastError();
  }
  double *tau = w.scal + 4;
  double *sig = w.scal + 4;
  const int cap = max_cap(x);
  const int nmx = max_nm(x);
  hipLaunchKernelGGL(k_round_init, dim3(1), dim3(64), 0, s, x, w.iwork, w.scal);
  if (left_orth) {
    const int64_t ne = (int64_t)x.cap[D - 1] * x.n[D - 1] * x.m[D - 1];
    const int blocks = (int)std::min<int64_t>((ne + 255) / 256, 1024);
    hipLaunchKernelGGL(k_last_to_carry, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, x,
                       w.carry);
  }
  for (int k = 0; k < D - 1 && !left_orth; ++k) {
    const double *src = (k == 0) ? x.data + x.off[0] : w.carry;
    const int64_t rc = (int64_t)cap_of(k) * x.n[k] * x.m[k];
    const int64_t cc = cap_of(k + 1);
    const int th = ktimer_begin(KT_QR_STEP, s);
    if (rc * cc <= LDS_DBL && (rc < cc ? rc : cc) <= LDS_TAU)
      hipLaunchKernelGGL(k_qr_step<true>, dim3(1), dim3(WG), 0, s, x, k, src, w.work,
                         w.rbuf, tau, w.iwork);
    else
      hipLaunchKernelGGL(k_qr_step<false>, dim3(1), dim3(WG), 0, s, x, k, src, w.work,
                         w.rbuf, tau, w.iwork);
    ktimer_end(th, s);
    const int mt = (x.cap[k + 1] + GT - 1) / GT;
    const int nt = (x.n[k + 1] * x.m[k + 1] * x.cap[k + 2] + GT - 1) / GT;
    hipLaunchKernelGGL(k_absorb, dim3(mt, nt), dim3(256), 0, s, x, k, w.rbuf,
                       w.carry, w.iwork);
  }
  hipLaunchKernelGGL(k_last_norm, dim3(1), dim3(WG), 0, s, x, w.carry, w.iwork,
                     w.scal);
  for (int k = D - 1; k >= 1; --k) {
    // fr[k+1] <= min(cap, rmax): the truncation already happened to its right
    const int64_t frc = (rmax > 0 && rmax < cap_of(k + 1)) ? rmax : cap_of(k + 1);
    const int64_t r0c = cap_of(k);
    const int64_t ncc = (int64_t)x.n[k] * x.m[k] * frc;
    const int64_t nbc = r0c < ncc ? r0c : ncc;
    const int64_t mbc = r0c > ncc ? r0c : ncc;
    const bool wide_qr = r0c < ncc && mbc * nbc + 2 * nbc * nbc <= LDS_SVD;
    const int th = ktimer_begin(KT_SVD_STEP, s);
    if ((mbc * nbc <= LDS_DBL && nbc * nbc <= LDS_DBL) || wide_qr)
      hipLaunchKernelGGL(k_svd_step<true>, dim3(1), dim3(WG), 0, s, x, k, eps, rmax,
                         w.carry, w.work, w.vbuf, w.fold, sig, w.iwork, w.scal, w.rotlog);
    else
      hipLaunchKernelGGL(k_svd_step<false>, dim3(1), dim3(WG), 0, s, x, k, eps, rmax,
                         w.carry, w.work, w.vbuf, w.fold, sig, w.iwork, w.scal, w.rotlog);
    ktimer_end(th, s);
    const int mt = (x.cap[k - 1] * x.n[k - 1] * x.m[k - 1] + GT - 1) / GT;
    const int nt = (x.cap[k] + GT - 1) / GT;
    hipLaunchKernelGGL(k_fold, dim3(mt, nt), dim3(256), 0, s, x, k, w.fold,
                       w.carry, w.iwork);
  }
  hipLaunchKernelGGL(k_round_finish, dim3(1), dim3(256), 0, s, x, w.carry,
                     w.iwork);
  (void)cap;
  (void)nmx;
  return hipGetLastError();
}

}  // namespace qtt
