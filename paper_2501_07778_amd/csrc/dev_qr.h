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

// Householder QR of W (rows x cols, ld rows) in place, NW wavefronts, one
// workgroup barrier per column.  Every wavefront forms the norm of column j
// below the diagonal itself (the same sum in every wavefront), so the
// reflector needs no workgroup reduction, and applies it, scaled in
// registers, to its share of the trailing columns.  Column j is rewritten
// (scaled reflector, beta on the diagonal) by wavefront 0 one step later,
// when no wavefront reads it any more.
template <int NW>
__device__ void householder_qr(double *W, int rows, int cols, double *tau) {
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
    double t = 0.0, beta = alpha, scale = 1.0;
    if (xnorm2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
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
__device__ void form_q_inplace(double *W, int rows, int kq, const double *tau) {
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
__device__ void apply_q(const double *W, int rows, int kq, const double *tau, double *Y,
                        int64_t ldy, int ncols) {
  for (int j = kq - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t != 0.0) reflect_cols<NW>(W + (int64_t)rows * j, j, rows, 1.0, t, Y, ldy, 0, ncols);
    __syncthreads();
  }
}

}  // namespace dev
}  // namespace qtt
