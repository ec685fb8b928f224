// dev_qr.h — Householder QR of a matrix held by one workgroup (LDS or
// global memory), and the products with its Q (device code only).
// Reflectors follow LAPACK's convention: H_j = I - tau_j v v^T with v(j) =
// 1, R on and above the diagonal, v below it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_reduce.h"

namespace qtt {
namespace dev {

// The Householder scalars of a column with entry alpha on the diagonal and
// squared norm xnorm2 below it: beta (the new diagonal), tau, and the factor
// that scales the entries below the diagonal into the reflector.
__device__ __forceinline__ void hh_scalars(double alpha, double xnorm2, double &beta, double &t,
                                           double &scale) {
  t = 0.0;
  beta = alpha;
  scale = 1.0;
  if (xnorm2 > 0.0) {
    beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
    t = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
}

// Householder QR for rows <= 16 REFL_RG: every column lies in the registers
// of one 16-lane group (rows j + lane + 16 k).  The group that applies H_j
// to column j+1 (group 0) then forms that column's norm below the diagonal
// and the scalars of H_{j+1} and publishes them in LDS (two buffers by step
// parity), so the other groups spend nothing on them; each group applies H_j
// to the columns j+2 + its index + 4 NW m.  One workgroup barrier per
// column; column j is rewritten by wavefront 0 one step later, as below.
template <int NW>
__device__ __forceinline__ void householder_qr_short(double *W, int rows, int cols, double *tau) {
  __shared__ double qs[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gl = threadIdx.x & 15, grp = threadIdx.x >> 4;
  constexpr int NG = NW * 4;
  const int kmax = rows < cols ? rows : cols;
  if (kmax <= 0) {
    __syncthreads();
    return;
  }
  double pscale = 1.0, pbeta = 0.0;
  auto finish = [&](int jj) {
    double *w = W + (int64_t)rows * jj;
    if (pscale != 1.0)
      for (int i = jj + 1 + lane; i < rows; i += 64) w[i] *= pscale;
    if (lane == 0) w[jj] = pbeta;
  };
  // group 0: the scalars of column c from its entries y (rows c - 1 + gl +
  // 16 k when the column was just updated by H_{c-1}; `base` is that first
  // row), published in qs[buf]
  auto publish = [&](const double (&y)[REFL_RG], int base, int c, int buf) {
    double p = 0.0;
#pragma unroll
    for (int k = 0; k < REFL_RG; ++k) {
      const int i = base + gl + 16 * k;
      p = fma((i > c && i < rows) ? y[k] : 0.0, (i > c && i < rows) ? y[k] : 0.0, p);
    }
    const double xnorm2 = row16_sum(p);
    // the diagonal entry, row c, sits in lane c - base of the group, k = 0
    const int src = c - base;
    const double alpha = __hiloint2double(
        __builtin_amdgcn_readlane(__double2hiint(y[0]), src),
        __builtin_amdgcn_readlane(__double2loint(y[0]), src));
    double beta, t, scale;
    hh_scalars(alpha, xnorm2, beta, t, scale);
    if (gl == 0) {
      qs[buf][0] = beta;
      qs[buf][1] = t;
      qs[buf][2] = scale;
    }
  };
  if (grp == 0) {
    double y[REFL_RG];
#pragma unroll
    for (int k = 0; k < REFL_RG; ++k) {
      const int i = gl + 16 * k;
      y[k] = W[i < rows ? i : 0];
    }
    publish(y, 0, 0, 0);
  }
  __syncthreads();
  for (int j = 0; j < kmax; ++j) {
    const double beta = qs[j & 1][0], t = qs[j & 1][1], scale = qs[j & 1][2];
    const double *wj = W + (int64_t)rows * j;
    int iv[REFL_RG];
    double wv[REFL_RG];
#pragma unroll
    for (int k = 0; k < REFL_RG; ++k) {
      const int i = j + gl + 16 * k;
      const bool ok = i < rows;
      iv[k] = ok ? i : j;
      const double w = wj[iv[k]];
      wv[k] = (i == j) ? 1.0 : (ok ? scale * w : 0.0);
    }
    for (int c = j + 1 + grp; c < cols; c += NG) {
      double *yc = W + (int64_t)rows * c;
      double yv[REFL_RG];
#pragma unroll
      for (int k = 0; k < REFL_RG; ++k) yv[k] = yc[iv[k]];
      if (t != 0.0) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < REFL_RG; k += 2) s0 = fma(wv[k], yv[k], s0);
#pragma unroll
        for (int k = 1; k < REFL_RG; k += 2) s1 = fma(wv[k], yv[k], s1);
        const double s = row16_sum(s0 + s1) * t;
#pragma unroll
        for (int k = 0; k < REFL_RG; ++k) {
          yv[k] -= s * wv[k];
          if (j + gl + 16 * k < rows) yc[iv[k]] = yv[k];
        }
      }
      if (c == j + 1 && c < kmax) publish(yv, j, c, (j + 1) & 1);
    }
    if (wave == 0 && j > 0) finish(j - 1);
    if (threadIdx.x == 0) tau[j] = t;
    pscale = (t != 0.0) ? scale : 1.0;
    pbeta = beta;
    __syncthreads();
  }
  if (wave == 0) finish(kmax - 1);
  __syncthreads();
}

// Householder QR of W (rows x cols, ld rows) in place, NW wavefronts, one
// workgroup barrier per column (short columns: householder_qr_short below).
// Otherwise every wavefront forms the norm of column j
// below the diagonal itself (the same sum in every wavefront), so the
// reflector needs no workgroup reduction, and applies it, scaled in
// registers, to its share of the trailing columns.  Column j is rewritten
// (scaled reflector, beta on the diagonal) by wavefront 0 one step later,
// when no wavefront reads it any more.
template <int NW>
__device__ __forceinline__ void householder_qr(double *W, int rows, int cols, double *tau) {
  if (rows <= 16 * REFL_RG) {
    householder_qr_short<NW>(W, rows, cols, tau);
    return;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kmax = rows < cols ? rows : cols;
  double pscale = 1.0, pbeta = 0.0;
  auto finish = [&](int jj) {
    double *w = W + (int64_t)rows * jj;
    if (pscale != 1.0)
      for (int i = jj + 1 + lane; i < rows; i += 64) w[i] *= pscale;
    if (lane == 0) w[jj] = pbeta;
  };
  for (int j = 0; j < kmax; ++j) {
    const double *wj = W + (int64_t)rows * j;
    double p = 0.0;
    for (int i = j + 1 + lane; i < rows; i += 64) p = fma(wj[i], wj[i], p);
    const double xnorm2 = wave64_sum(p);
    const double alpha = wj[j];
    double beta, t, scale;
    hh_scalars(alpha, xnorm2, beta, t, scale);
    if (t != 0.0) reflect_cols<NW>(wj, j, rows, scale, t, W, rows, j + 1, cols);
    if (wave == 0 && j > 0) finish(j - 1);
    if (threadIdx.x == 0) tau[j] = t;
    pscale = (t != 0.0) ? scale : 1.0;
    pbeta = beta;
    __syncthreads();
  }
  if (wave == 0 && kmax > 0) finish(kmax - 1);
  __syncthreads();
}

// Q (rows x kq, ld ldq) = H_0 ... H_{kq-1} [I; 0] from the reflectors in W
template <int NW>
__device__ void form_q(const double *W, int rows, int kq, const double *tau, double *Q,
                       int64_t ldq) {
  for (int64_t e = threadIdx.x; e < (int64_t)rows * kq; e += NW * 64) {
    const int i = (int)(e % rows), c = (int)(e / rows);
    Q[i + ldq * c] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = kq - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t != 0.0) reflect_cols<NW>(W + (int64_t)rows * j, j, rows, 1.0, t, Q, ldq, j, kq);
    __syncthreads();
  }
}

// Q (rows x kq) = H_0 ... H_{kq-1} [I; 0] formed in place of the first kq
// columns of W (LAPACK's order of dorg2r): for j = kq-1 down to 0, H_j is
// applied to the columns j+1.. (already the trailing columns of Q, zero
// above row j+1) and column j becomes H_j e_j = e_j - tau_j v_j.  Column
// j+1 is formed at step j by wavefront 0, which owns it in reflect_cols,
// just before it applies H_j to it, so a step needs one barrier.  Whatever
// W held on and above the diagonal (R) is overwritten.
template <int NW>
__device__ __forceinline__ void form_q_inplace(double *W, int rows, int kq, const double *tau) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wavefront 0: column c <- H_c e_c from its reflector
  auto form = [&](int c) {
    double *wc = W + (int64_t)rows * c;
    const double t = tau[c];
    for (int i = lane; i < rows; i += 64)
      wc[i] = (i < c) ? 0.0 : ((i == c) ? 1.0 - t : -t * wc[i]);
    // other lanes of this wavefront read these rows next: wait for the stores
    // (W may be in global memory, where a wavefront's accesses to one address
    // from different lanes are not ordered without it)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  };
  __syncthreads();
  for (int j = kq - 1; j >= 0; --j) {
    const double t = tau[j];
    if (wave == 0 && j + 1 < kq) form(j + 1);
    if (t != 0.0) reflect_cols<NW>(W + (int64_t)rows * j, j, rows, 1.0, t, W, rows, j + 1, kq);
    __syncthreads();
  }
  if (wave == 0 && kq > 0) form(0);
  __syncthreads();
}

// Y (rows x ncols, ld ldy) <- H_0 H_1 ... H_{kq-1} Y
template <int NW>
__device__ __forceinline__ void apply_q(const double *W, int rows, int kq, const double *tau, double *Y,
                        int64_t ldy, int ncols) {
  for (int j = kq - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t != 0.0) reflect_cols<NW>(W + (int64_t)rows * j, j, rows, 1.0, t, Y, ldy, 0, ncols);
    __syncthreads();
  }
}

}  // namespace dev
}  // namespace qtt
