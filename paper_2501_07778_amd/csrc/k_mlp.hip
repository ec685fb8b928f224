// k_mlp.hip — learned warm start: an MLP from load parameters to the QTT
// cores of the displacement, trained on the GPU with a gauge-invariant loss
// in TT space (Frobenius, or the energy norm of the stiffness matrix) or a
// plain loss on the cores of targets brought to one gauge, gfx950.
//
// Layout: column-major, one sample per column.  Layer l has W_l (out x in)
// and b_l (out); hidden layers use ReLU, the output layer is linear.  The
// output column of a sample is a train with a fixed rank pattern, cores
// packed one after another, each (r_k, n_k, r_{k+1}) column-major.  The loss
// of a sample is ||TT(o) - u||^2 / ||u||^2 = (<x,x> - 2<x,u> + <u,u>)/<u,u>,
// its gradient core k is 2 (Lxx_k X_k Rxx_{k+1} - Lxu_k U_k Rxu_{k+1}) / <u,u>
// with the left/right environments of the inner products (FP64 in the
// kernel; parameters, activations and gradients are FP32).  Adam (Kingma
// and Ba, ICLR 2015) updates the parameters.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace qtt {
namespace {

constexpr int TM = 64, TK = 16;

// C (M x N) = op(A) op(B) (+ bias per row) (ReLU), column-major, FP32
// accumulate; 64 x 64 output tile per 256-thread block, 4 x 4 per thread.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256)
    k_gemm32(const float *A, int lda, const float *B, int ldb, float *C, int ldc, int M, int N,
             int K, const float *bias, int relu) {
  __shared__ float As[TK][TM + 1];
  __shared__ float Bs[TK][TM + 1];
  const int tid = threadIdx.x;
  const int tr = tid % 16, tc = tid / 16;
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TM;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += TK) {
    for (int e = tid; e < TK * TM; e += 256) {
      const int mm = e % TM, kk = e / TM;
      const int gm = m0 + mm, gk = k0 + kk;
      float av = 0.f;
      if (gm < M && gk < K) av = TA ? A[gk + (int64_t)lda * gm] : A[gm + (int64_t)lda * gk];
      As[kk][mm] = av;
      const int kk2 = e % TK, nn = e / TK;
      const int gk2 = k0 + kk2, gn = n0 + nn;
      float bv = 0.f;
      if (gk2 < K && gn < N) bv = TB ? B[gn + (int64_t)ldb * gk2] : B[gk2 + (int64_t)ldb * gn];
      Bs[kk2][nn] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = As[kk][tr + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = Bs[kk][tc + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gm = m0 + tr + 16 * u, gn = n0 + tc + 16 * v;
      if (gm < M && gn < N) {
        float r = acc[u][v] + (bias ? bias[gm] : 0.f);
        if (relu) r = r > 0.f ? r : 0.f;
        C[gm + (int64_t)ldc * gn] = r;
      }
    }
}

// ------------------------------------------------------------ BF16 MFMA
// C (M x N) = op(A) op(B) (+ bias per row) (ReLU) with the operands rounded
// to BF16 (round to nearest even) as they are staged in LDS and FP32
// accumulation in v_mfma_f32_16x16x32_bf16; FP32 in and out, column-major
// like k_gemm32.  A 256-thread block computes a 64 x 64 tile; each of its
// four wavefronts a 32 x 32 quarter as 2 x 2 MFMA tiles of 16 x 16, K in
// steps of 32.  Operand layout of the instruction: lane l supplies row
// (A) or column (B) l % 16 and eight K positions chosen by l / 16; both
// operands use the same positions, so any such assignment sums over all
// 32; the result: lane l holds rows 4 (l / 16) + v, v = 0..3, of column
// l % 16.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
constexpr int BT = 64, BK = 32, BKP = BK + 8;   // LDS rows padded against bank conflicts

__device__ __forceinline__ __bf16 to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);   // nearest even
  const unsigned short h = (unsigned short)(u >> 16);
  return __builtin_bit_cast(__bf16, h);
}

template <bool TA, bool TB>
__global__ void __launch_bounds__(256)
    k_gemm_bf16(const float *A, int lda, const float *B, int ldb, float *C, int ldc, int M, int N,
                int K, const float *bias, int relu) {
  __shared__ __bf16 As[BT][BKP];   // As[m][k]
  __shared__ __bf16 Bs[BT][BKP];   // Bs[n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int m0 = blockIdx.x * BT, n0 = blockIdx.y * BT;
  f32x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += BK) {
    for (int e = tid; e < BT * BK; e += 256) {
      int mm, kk;
      if (TA) { kk = e % BK; mm = e / BK; } else { mm = e % BT; kk = e / BT; }
      const int gm = m0 + mm, gk = k0 + kk;
      float av = 0.f;
      if (gm < M && gk < K) av = TA ? A[gk + (int64_t)lda * gm] : A[gm + (int64_t)lda * gk];
      As[mm][kk] = to_bf16(av);
      int nn, kb;
      if (TB) { nn = e % BT; kb = e / BT; } else { kb = e % BK; nn = e / BK; }
      const int gn = n0 + nn, gk2 = k0 + kb;
      float bv = 0.f;
      if (gk2 < K && gn < N) bv = TB ? B[gn + (int64_t)ldb * gk2] : B[gk2 + (int64_t)ldb * gn];
      Bs[nn][kb] = to_bf16(bv);
    }
    __syncthreads();
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    bf16x8_t a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        a[t][v] = As[32 * wr + 16 * t + r16][kq + v];
        b[t][v] = Bs[32 * wc + 16 * t + r16][kq + v];
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  const int col = lane & 15, rb = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + 32 * wr + 16 * i + rb + v;
        const int gn = n0 + 32 * wc + 16 * j + col;
        if (gm < M && gn < N) {
          float r = acc[i][j][v] + (bias ? bias[gm] : 0.f);
          if (relu) r = r > 0.f ? r : 0.f;
          C[gm + (int64_t)ldc * gn] = r;
        }
      }
}

// db[i] = sum_j dZ[i + M j]
__global__ void k_rowsum(const float *dZ, int M, int N, float *db) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  float s = 0.f;
  for (int j = 0; j < N; ++j) s += dZ[i + (int64_t)M * j];
  db[i] = s;
}

// dH <- dH * (H > 0): the ReLU derivative from the stored activations
__global__ void k_relu_mask(float *dH, const float *H, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    if (!(H[e] > 0.f)) dH[e] = 0.f;
}

struct TTShape {
  int D;
  int n[QTT_MAXD];
  int r[QTT_MAXD + 1];
  int64_t off[QTT_MAXD + 1];  // core offsets within a column; off[D] = column length
  int rmax;
};

// L' = sum_i X_i^T L Y_i (left) for cores k of x and y (both with the
// shape's ranks); T is scratch of r*n*r doubles
__device__ void env_left(const float *X, const float *Y, const double *L, double *Lout,
                         double *Tm, int r0, int n, int r1) {
  // T[a, i, b'] = sum_a' L[a, a'] Y[a', i, b']
  for (int e = threadIdx.x; e < r0 * n * r1; e += blockDim.x) {
    const int a = e % r0, ib = e / r0;
    double s = 0.0;
    for (int a2 = 0; a2 < r0; ++a2) s += L[a + r0 * a2] * (double)Y[a2 + r0 * ib];
    Tm[e] = s;
  }
  __syncthreads();
  // L'[b, b'] = sum_{a, i} X[a, i, b] T[a, i, b']
  for (int e = threadIdx.x; e < r1 * r1; e += blockDim.x) {
    const int b = e % r1, b2 = e / r1;
    double s = 0.0;
    for (int l = 0; l < r0 * n; ++l) s += (double)X[l + r0 * n * b] * Tm[l + r0 * n * b2];
    Lout[e] = s;
  }
  __syncthreads();
}

// R = sum_i X_i R' Y_i^T (right)
__device__ void env_right(const float *X, const float *Y, const double *R, double *Rout,
                          double *Tm, int r0, int n, int r1) {
  // T[a, i, b'] = sum_b X[a, i, b] R[b, b'] ... T[a,i,b'] = sum_b X[a,i,b] R[b,b']
  for (int e = threadIdx.x; e < r0 * n * r1; e += blockDim.x) {
    const int ai = e % (r0 * n), b2 = e / (r0 * n);
    double s = 0.0;
    for (int b = 0; b < r1; ++b) s += (double)X[ai + r0 * n * b] * R[b + r1 * b2];
    Tm[e] = s;
  }
  __syncthreads();
  // Rout[a, a'] = sum_{i, b'} T[a, i, b'] Y[a', i, b']
  for (int e = threadIdx.x; e < r0 * r0; e += blockDim.x) {
    const int a = e % r0, a2 = e / r0;
    double s = 0.0;
    for (int ib = 0; ib < n * r1; ++ib) s += Tm[a + r0 * ib] * (double)Y[a2 + r0 * ib];
    Rout[e] = s;
  }
  __syncthreads();
}

// one block per sample j: loss_j and dOut column j (scaled by `scale`)
__global__ void __launch_bounds__(256)
    k_tt_loss_grad(const float *out, const float *tgt, float *dout, double *loss, TTShape sh,
                   double *scratch, int64_t per_sample, float scale, int angle) {
  const int j = blockIdx.x;
  const int64_t P = sh.off[sh.D];
  const float *x = out + P * j;
  const float *u = tgt + P * j;
  float *g = dout + P * j;
  const int D = sh.D, R = sh.rmax;
  const int64_t env = (int64_t)R * R;
  double *base = scratch + per_sample * j;
  double *Lxx = base, *Lxu = Lxx + (D + 1) * env, *Luu = Lxu + (D + 1) * env;
  double *Rxx = Luu + (D + 1) * env, *Rxu = Rxx + (D + 1) * env;
  double *Tm = Rxu + (D + 1) * env;  // r n r scratch
  if (threadIdx.x == 0) {
    Lxx[0] = Lxu[0] = Luu[0] = 1.0;
    Rxx[D * env] = Rxu[D * env] = 1.0;
  }
  __syncthreads();
  for (int k = 0; k < D; ++k) {
    const int r0 = sh.r[k], n = sh.n[k], r1 = sh.r[k + 1];
    const float *Xk = x + sh.off[k], *Uk = u + sh.off[k];
    env_left(Xk, Xk, Lxx + k * env, Lxx + (k + 1) * env, Tm, r0, n, r1);
    env_left(Xk, Uk, Lxu + k * env, Lxu + (k + 1) * env, Tm, r0, n, r1);
    env_left(Uk, Uk, Luu + k * env, Luu + (k + 1) * env, Tm, r0, n, r1);
  }
  for (int k = D - 1; k >= 1; --k) {
    const int r0 = sh.r[k], n = sh.n[k], r1 = sh.r[k + 1];
    const float *Xk = x + sh.off[k], *Uk = u + sh.off[k];
    env_right(Xk, Xk, Rxx + (k + 1) * env, Rxx + k * env, Tm, r0, n, r1);
    env_right(Xk, Uk, Rxu + (k + 1) * env, Rxu + k * env, Tm, r0, n, r1);
  }
  const double xx = Lxx[D * env], xu = Lxu[D * env], uu = Luu[D * env];
  const double inv = uu > 0.0 ? 1.0 / uu : 0.0;
  // distance: L = (xx - 2 xu + uu) / uu, dL/dX = 2 (Gxx - Gxu) / uu;
  // angle: L = 1 - xu^2 / (xx uu), dL/dX = 2 xu / (xx uu) (xu / xx Gxx - Gxu),
  // with Gxx = Lxx X Rxx (half the gradient of xx) and Gxu = Lxu U Rxu
  const bool ang = angle && xx > 0.0 && uu > 0.0;
  const double cxx = ang ? 2.0 * xu * xu / (xx * xx * uu) : 2.0 * inv;
  const double cxu = ang ? -2.0 * xu / (xx * uu) : -2.0 * inv;
  if (threadIdx.x == 0) loss[j] = angle ? (ang ? 1.0 - xu * xu / (xx * uu) : 1.0)
                                        : (xx - 2.0 * xu + uu) * inv;
  for (int k = 0; k < D; ++k) {
    const int r0 = sh.r[k], n = sh.n[k], r1 = sh.r[k + 1];
    const float *Xk = x + sh.off[k], *Uk = u + sh.off[k];
    const double *lxx = Lxx + k * env, *lxu = Lxu + k * env;
    const double *rxx = Rxx + (k + 1) * env, *rxu = Rxu + (k + 1) * env;
    for (int e = threadIdx.x; e < r0 * n * r1; e += blockDim.x) {
      const int a = e % r0, ib = e / r0;
      const int i = ib % n, b = ib / n;
      double sx = 0.0, su = 0.0;
      for (int a2 = 0; a2 < r0; ++a2) {
        double tx = 0.0, tu = 0.0;
        for (int b2 = 0; b2 < r1; ++b2) {
          tx += (double)Xk[a2 + r0 * (i + n * b2)] * rxx[b + r1 * b2];
          tu += (double)Uk[a2 + r0 * (i + n * b2)] * rxu[b + r1 * b2];
        }
        sx += lxx[a + r0 * a2] * tx;
        su += lxu[a + r0 * a2] * tu;
      }
      g[sh.off[k] + e] = (float)(cxx * sx + cxu * su) * scale;
    }
  }
}

struct OpShape {
  int ra[QTT_MAXD + 1];
  int64_t off[QTT_MAXD + 1];
  const double *data;
};

// partial W2[a, i, be, b'] = sum_{al, j, a'} Phi[a, al, a'] A[al, i, j, be] Y[a', j, b']
// (Phi r0 x ra0 x r0, Y r0 x n x r1); W1 scratch r0 ra0 n r1
__device__ void op_partial(const double *Phi, const double *Ak, const float *Y, double *W1,
                           double *W2, int r0, int ra0, int ra1, int n, int r1) {
  const int64_t n1 = (int64_t)r0 * ra0 * n * r1;
  for (int64_t e = threadIdx.x; e < n1; e += blockDim.x) {
    const int aal = (int)(e % ((int64_t)r0 * ra0));
    const int jb = (int)(e / ((int64_t)r0 * ra0));
    const float *yc = Y + (int64_t)r0 * jb;
    double acc = 0.0;
    for (int a2 = 0; a2 < r0; ++a2) acc += Phi[aal + (int64_t)r0 * ra0 * a2] * (double)yc[a2];
    W1[e] = acc;
  }
  __syncthreads();
  const int64_t n2 = (int64_t)r0 * n * ra1 * r1;
  for (int64_t e = threadIdx.x; e < n2; e += blockDim.x) {
    const int a = (int)(e % r0);
    int64_t t = e / r0;
    const int i = (int)(t % n);
    t /= n;
    const int be = (int)(t % ra1);
    const int b2 = (int)(t / ra1);
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
      const double *w = W1 + a + (int64_t)r0 * ra0 * (j + (int64_t)n * b2);
      const double *av = Ak + (int64_t)ra0 * (i + (int64_t)n * (j + (int64_t)n * be));
      for (int al = 0; al < ra0; ++al) acc += w[(int64_t)r0 * al] * av[al];
    }
    W2[e] = acc;
  }
  __syncthreads();
}

// Phi'[b, be, b'] = sum_{a, i} X[a, i, b] W2[a, i, be, b']
__device__ void op_left_close(const float *X, const double *W2, double *Phin, int r0, int n,
                              int ra1, int r1) {
  const int L = r0 * n;
  for (int e = threadIdx.x; e < r1 * ra1 * r1; e += blockDim.x) {
    const int b = e % r1, col = e / r1;
    double acc = 0.0;
    for (int l = 0; l < L; ++l) acc += (double)X[l + L * b] * W2[l + (int64_t)L * col];
    Phin[e] = acc;
  }
  __syncthreads();
}

// right environment Psi_k[a, al, a'] = sum X[a,i,b] A[al,i,j,be] Y[a',j,b'] Psi_{k+1}[b,be,b']
// via V1[a, i, be, b'] = sum_b X[a,i,b] Psi[b,be,b'], then
// Psi_k[a, al, a'] = sum_{i, j, be, b'} V1[a,i,be,b'] A[al,i,j,be] Y[a',j,b']
__device__ void op_right(const float *X, const double *Ak, const float *Y, const double *Psi,
                         double *Psin, double *V1, double *V2, int r0, int ra0, int ra1, int n,
                         int r1) {
  const int64_t n1 = (int64_t)r0 * n * ra1 * r1;
  for (int64_t e = threadIdx.x; e < n1; e += blockDim.x) {
    const int ai = (int)(e % ((int64_t)r0 * n));
    const int64_t bb = e / ((int64_t)r0 * n);  // be + ra1 b'
    double acc = 0.0;
    for (int b = 0; b < r1; ++b) acc += (double)X[ai + (int64_t)r0 * n * b] * Psi[b + (int64_t)r1 * bb];
    V1[e] = acc;
  }
  __syncthreads();
  // V2[a, al, j, b'] = sum_{i, be} V1[a, i, be, b'] A[al, i, j, be]
  const int64_t n2 = (int64_t)r0 * ra0 * n * r1;
  for (int64_t e = threadIdx.x; e < n2; e += blockDim.x) {
    const int a = (int)(e % r0);
    int64_t t = e / r0;
    const int al = (int)(t % ra0);
    t /= ra0;
    const int j = (int)(t % n);
    const int b2 = (int)(t / n);
    double acc = 0.0;
    for (int be = 0; be < ra1; ++be)
      for (int i = 0; i < n; ++i)
        acc += V1[a + (int64_t)r0 * (i + (int64_t)n * (be + (int64_t)ra1 * b2))] *
               Ak[al + (int64_t)ra0 * (i + (int64_t)n * (j + (int64_t)n * be))];
    V2[e] = acc;
  }
  __syncthreads();
  // Psi_k[a, al, a'] = sum_{j, b'} V2[a, al, j, b'] Y[a', j, b']
  for (int e = threadIdx.x; e < r0 * ra0 * r0; e += blockDim.x) {
    const int aal = e % (r0 * ra0), a2 = e / (r0 * ra0);
    double acc = 0.0;
    for (int jb = 0; jb < n * r1; ++jb)
      acc += V2[aal + (int64_t)r0 * ra0 * jb] * (double)Y[a2 + (int64_t)r0 * jb];
    Psin[e] = acc;
  }
  __syncthreads();
}

// energy-norm loss ||x - u||_A^2 / ||u||_A^2 for a symmetric positive
// definite TT operator A (the stiffness matrix) and its gradient
__global__ void __launch_bounds__(256)
    k_tt_energy_loss_grad(const float *out, const float *tgt, float *dout, double *loss,
                          TTShape sh, OpShape op, double *scratch, int64_t per_sample,
                          int64_t env_cap, int64_t w_cap, float scale, int angle) {
  const int j = blockIdx.x;
  const int64_t P = sh.off[sh.D];
  const float *x = out + P * j;
  const float *u = tgt + P * j;
  float *g = dout + P * j;
  const int D = sh.D;
  double *base = scratch + per_sample * j;
  double *Pxx = base;                          // right environments, D + 1 each
  double *Pxu = Pxx + (D + 1) * env_cap;
  double *Fxx = Pxu + (D + 1) * env_cap;       // current left environments
  double *Fxu = Fxx + env_cap, *Fuu = Fxu + env_cap, *Fn = Fuu + env_cap;
  double *W1 = Fn + env_cap, *W2 = W1 + w_cap, *W3 = W2 + w_cap;
  double *Gx = W3 + w_cap, *Gu = Gx + P;       // angle: the two gradient parts
  if (threadIdx.x == 0) {
    Pxx[D * env_cap] = Pxu[D * env_cap] = 1.0;
    Fxx[0] = Fxu[0] = Fuu[0] = 1.0;
  }
  __syncthreads();
  for (int k = D - 1; k >= 1; --k) {
    const int r0 = sh.r[k], n = sh.n[k], r1 = sh.r[k + 1];
    const double *Ak = op.data + op.off[k];
    const float *Xk = x + sh.off[k], *Uk = u + sh.off[k];
    op_right(Xk, Ak, Xk, Pxx + (k + 1) * env_cap, Pxx + k * env_cap, W1, W2, r0, op.ra[k],
             op.ra[k + 1], n, r1);
    op_right(Xk, Ak, Uk, Pxu + (k + 1) * env_cap, Pxu + k * env_cap, W1, W2, r0, op.ra[k],
             op.ra[k + 1], n, r1);
  }
  // forward: gradient of core k from the partials and the right environments
  for (int k = 0; k < D; ++k) {
    const int r0 = sh.r[k], n = sh.n[k], r1 = sh.r[k + 1];
    const int ra0 = op.ra[k], ra1 = op.ra[k + 1];
    const double *Ak = op.data + op.off[k];
    const float *Xk = x + sh.off[k], *Uk = u + sh.off[k];
    const double *pxx = Pxx + (k + 1) * env_cap, *pxu = Pxu + (k + 1) * env_cap;
    // partials with y = x and y = u
    op_partial(Fxx, Ak, Xk, W1, W2, r0, ra0, ra1, n, r1);
    op_partial(Fxu, Ak, Uk, W1, W3, r0, ra0, ra1, n, r1);
    // G[a, i, b] = sum_{be, b'} W[a, i, be, b'] Psi[b, be, b']
    for (int e = threadIdx.x; e < r0 * n * r1; e += blockDim.x) {
      const int ai = e % (r0 * n), b = e / (r0 * n);
      double gx = 0.0, gu = 0.0;
      for (int bb = 0; bb < ra1 * r1; ++bb) {
        gx += W2[ai + (int64_t)r0 * n * bb] * pxx[b + (int64_t)r1 * bb];
        gu += W3[ai + (int64_t)r0 * n * bb] * pxu[b + (int64_t)r1 * bb];
      }
      if (angle) {
        Gx[sh.off[k] + e] = gx;
        Gu[sh.off[k] + e] = gu;
      } else {
        W1[e] = 2.0 * gx - 2.0 * gu;   // W1 is free again: keep the raw gradient
      }
    }
    __syncthreads();
    if (!angle)
      for (int e = threadIdx.x; e < r0 * n * r1; e += blockDim.x) g[sh.off[k] + e] = (float)W1[e];
    __syncthreads();
    op_left_close(Xk, W2, Fn, r0, n, ra1, r1);
    for (int e = threadIdx.x; e < r1 * ra1 * r1; e += blockDim.x) Fxx[e] = Fn[e];
    __syncthreads();
    op_left_close(Xk, W3, Fn, r0, n, ra1, r1);
    for (int e = threadIdx.x; e < r1 * ra1 * r1; e += blockDim.x) Fxu[e] = Fn[e];
    __syncthreads();
    op_partial(Fuu, Ak, Uk, W1, W2, r0, ra0, ra1, n, r1);
    op_left_close(Uk, W2, Fn, r0, n, ra1, r1);
    for (int e = threadIdx.x; e < r1 * ra1 * r1; e += blockDim.x) Fuu[e] = Fn[e];
    __syncthreads();
  }
  const double xx = Fxx[0], xu = Fxu[0], uu = Fuu[0];
  const double inv = uu > 0.0 ? 1.0 / uu : 0.0;
  if (angle) {
    // L = 1 - xu^2 / (xx uu), dL/dX = 2 xu / (xx uu) (xu / xx Gx - Gu)
    const bool ok = xx > 0.0 && uu > 0.0;
    const double cxx = ok ? 2.0 * xu * xu / (xx * xx * uu) : 0.0;
    const double cxu = ok ? -2.0 * xu / (xx * uu) : 0.0;
    if (threadIdx.x == 0) loss[j] = ok ? 1.0 - xu * xu / (xx * uu) : 1.0;
    for (int64_t e = threadIdx.x; e < P; e += blockDim.x)
      g[e] = (float)(cxx * Gx[e] + cxu * Gu[e]) * scale;
    return;
  }
  if (threadIdx.x == 0) loss[j] = (xx - 2.0 * xu + uu) * inv;
  // scale the raw gradients by 1/<u, A u> and the batch factor
  for (int64_t e = threadIdx.x; e < P; e += blockDim.x) g[e] = (float)((double)g[e] * inv) * scale;
}

// one block per sample j: loss_j = ||x - u||^2 / ||u||^2 over the packed
// cores themselves (targets in one fixed gauge) and dOut = 2 (x - u) / ||u||^2
// times `scale`
__global__ void __launch_bounds__(256)
    k_core_loss_grad(const float *out, const float *tgt, float *dout, double *loss, int64_t P,
                     float scale) {
  __shared__ double red[2][256];
  const int j = blockIdx.x;
  const float *x = out + P * j;
  const float *u = tgt + P * j;
  float *g = dout + P * j;
  double dd = 0.0, uu = 0.0;
  for (int64_t e = threadIdx.x; e < P; e += blockDim.x) {
    const double d = (double)x[e] - (double)u[e];
    dd += d * d;
    uu += (double)u[e] * (double)u[e];
  }
  red[0][threadIdx.x] = dd;
  red[1][threadIdx.x] = uu;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  const double inv = red[1][0] > 0.0 ? 1.0 / red[1][0] : 0.0;
  if (threadIdx.x == 0) loss[j] = red[0][0] * inv;
  for (int64_t e = threadIdx.x; e < P; e += blockDim.x)
    g[e] = (float)(2.0 * ((double)x[e] - (double)u[e]) * inv) * scale;
}

__global__ void k_mean(const double *v, int n, double *out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += v[i];
    out[0] = s / n;
  }
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                       float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

int64_t param_count(int nl, const int32_t *sz) {
  int64_t c = 0;
  for (int l = 0; l < nl; ++l) c += (int64_t)sz[l + 1] * sz[l] + sz[l + 1];
  return c;
}

hipError_t gemm(bool ta, bool tb, const float *A, int lda, const float *B, int ldb, float *C,
                int ldc, int M, int N, int K, const float *bias, int relu, hipStream_t s,
                bool bf16 = false) {
  dim3 grid((M + TM - 1) / TM, (N + TM - 1) / TM);
  if (bf16) {
    if (!ta && !tb)
      hipLaunchKernelGGL((k_gemm_bf16<false, false>), grid, dim3(256), 0, s, A, lda, B, ldb, C,
                         ldc, M, N, K, bias, relu);
    else if (ta && !tb)
      hipLaunchKernelGGL((k_gemm_bf16<true, false>), grid, dim3(256), 0, s, A, lda, B, ldb, C,
                         ldc, M, N, K, bias, relu);
    else
      hipLaunchKernelGGL((k_gemm_bf16<false, true>), grid, dim3(256), 0, s, A, lda, B, ldb, C,
                         ldc, M, N, K, bias, relu);
    return hipGetLastError();
  }
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm32<false, false>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc,
                       M, N, K, bias, relu);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm32<true, false>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc,
                       M, N, K, bias, relu);
  else
    hipLaunchKernelGGL((k_gemm32<false, true>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc,
                       M, N, K, bias, relu);
  return hipGetLastError();
}

qtt_status check_net(const qtt_mlp *net) {
  if (!net || !net->sizes || !net->params) return fail(QTT_E_INVAL, "net: NULL field");
  if (net->nlayers < 1 || net->nlayers > 16) return fail(QTT_E_INVAL, "nlayers must be 1..16");
  if (net->gemm_dtype != QTT_F64 && net->gemm_dtype != QTT_F32 && net->gemm_dtype != QTT_BF16)
    return fail(QTT_E_INVAL, "gemm_dtype must be QTT_F32 or QTT_BF16");
  if (net->loss != QTT_LOSS_TT && net->loss != QTT_LOSS_CORES && net->loss != QTT_LOSS_ANGLE)
    return fail(QTT_E_INVAL, "loss must be QTT_LOSS_TT, QTT_LOSS_CORES or QTT_LOSS_ANGLE");
  for (int l = 0; l <= net->nlayers; ++l)
    if (net->sizes[l] < 1 || net->sizes[l] > (1 << 20)) return fail(QTT_E_INVAL, "bad layer size");
  return QTT_OK;
}

struct MlpWs {
  std::vector<float *> H;  // activations per layer (H[0] = input, not stored)
  float *dA = nullptr, *dB = nullptr;
  float *grad = nullptr;
  double *loss = nullptr, *lmean = nullptr, *scratch = nullptr;
  int64_t per_sample = 0, env_cap = 0, w_cap = 0;
};

// energy-loss scratch sizes for a train shape and operator ranks
void energy_caps(const TTShape &sh, const int32_t *ra, int64_t &env_cap, int64_t &w_cap) {
  env_cap = 1;
  w_cap = 1;
  for (int k = 0; k <= sh.D; ++k)
    env_cap = std::max<int64_t>(env_cap, (int64_t)sh.r[k] * ra[k] * sh.r[k]);
  for (int k = 0; k < sh.D; ++k) {
    w_cap = std::max<int64_t>(w_cap, (int64_t)sh.r[k] * ra[k] * sh.n[k] * sh.r[k + 1]);
    w_cap = std::max<int64_t>(w_cap, (int64_t)sh.r[k] * sh.n[k] * ra[k + 1] * sh.r[k + 1]);
  }
}

bool carve_mlp(Arena &ar, const qtt_mlp *net, int B, const TTShape *sh, MlpWs &w,
               const int32_t *metric_ranks = nullptr) {
  const int nl = net->nlayers;
  int widest = 1;
  for (int l = 0; l <= nl; ++l) widest = std::max(widest, (int)net->sizes[l]);
  w.H.assign(nl + 1, nullptr);
  for (int l = 1; l <= nl; ++l)
    w.H[l] = (float *)ar.take(sizeof(float) * (int64_t)net->sizes[l] * B);
  w.dA = (float *)ar.take(sizeof(float) * (int64_t)widest * B);
  w.dB = (float *)ar.take(sizeof(float) * (int64_t)widest * B);
  if (sh) {
    w.grad = (float *)ar.take(sizeof(float) * param_count(nl, net->sizes));
    w.loss = (double *)ar.take(sizeof(double) * B);
    w.lmean = (double *)ar.take(sizeof(double) * 4);
    const int64_t env = (int64_t)sh->rmax * sh->rmax;
    int64_t tm = 1;
    for (int k = 0; k < sh->D; ++k)
      tm = std::max<int64_t>(tm, (int64_t)sh->r[k] * sh->n[k] * sh->r[k + 1]);
    w.per_sample = 5 * (sh->D + 1) * env + tm;
    if (metric_ranks) {
      energy_caps(*sh, metric_ranks, w.env_cap, w.w_cap);
      w.per_sample = std::max<int64_t>(
          w.per_sample, (2 * (sh->D + 1) + 4) * w.env_cap + 3 * w.w_cap + 2 * sh->off[sh->D]);
    }
    w.scratch = (double *)ar.take(sizeof(double) * w.per_sample * B);
  }
  return ar.ok();
}

qtt_status make_shape(int D, const int32_t *nrow, const int32_t *ranks, int nout, TTShape &sh) {
  if (D < 1 || D > QTT_MAXD || !nrow || !ranks) return fail(QTT_E_INVAL, "bad train shape");
  if (ranks[0] != 1 || ranks[D] != 1) return fail(QTT_E_SHAPE, "boundary ranks must be 1");
  sh.D = D;
  sh.rmax = 1;
  int64_t off = 0;
  for (int k = 0; k < D; ++k) {
    if (nrow[k] < 1 || nrow[k] > 64 || ranks[k + 1] < 1 || ranks[k + 1] > 256)
      return fail(QTT_E_INVAL, "modes 1..64 and ranks 1..256");
    sh.n[k] = nrow[k];
    sh.r[k] = ranks[k];
    sh.off[k] = off;
    off += (int64_t)ranks[k] * nrow[k] * ranks[k + 1];
    sh.rmax = std::max(sh.rmax, (int)ranks[k + 1]);
  }
  sh.r[D] = 1;
  sh.off[D] = off;
  if (off != nout) return fail(QTT_E_SHAPE, "output size != packed size of the rank pattern");
  return QTT_OK;
}

qtt_status check_metric(const qtt_tt *A, const TTShape &sh, OpShape &op) {
  if (!A) return QTT_OK;
  if (!A->ncol || !A->data || !A->ranks || !A->nrow || A->ncores != sh.D)
    return fail(QTT_E_INVAL, "metric must be a QTT matrix with the train's cores");
  if (A->ranks[0] != 1 || A->ranks[sh.D] != 1) return fail(QTT_E_SHAPE, "metric boundary ranks");
  int64_t off = 0;
  for (int k = 0; k < sh.D; ++k) {
    if (A->nrow[k] != sh.n[k] || A->ncol[k] != sh.n[k])
      return fail(QTT_E_SHAPE, "metric modes differ from the train's");
    if (A->ranks[k + 1] < 1 || A->ranks[k + 1] > 1024) return fail(QTT_E_SHAPE, "metric rank");
    op.ra[k] = A->ranks[k];
    op.off[k] = off;
    off += (int64_t)A->ranks[k] * sh.n[k] * sh.n[k] * A->ranks[k + 1];
  }
  op.ra[sh.D] = 1;
  op.off[sh.D] = off;
  if (off > A->capacity) return fail(QTT_E_CAPACITY, "metric: capacity below its packed size");
  op.data = (const double *)A->data;
  return QTT_OK;
}

// forward pass; activations of layer l in w.H[l] (the last one linear)
hipError_t forward(const qtt_mlp *net, const float *a, int B, MlpWs &w, hipStream_t s) {
  const int nl = net->nlayers;
  const float *p = net->params;
  const float *h = a;
  for (int l = 0; l < nl; ++l) {
    const int in = net->sizes[l], out = net->sizes[l + 1];
    const float *W = p, *b = p + (int64_t)out * in;
    hipError_t e = gemm(false, false, W, out, h, in, w.H[l + 1], out, out, B, in, b,
                        l < nl - 1 ? 1 : 0, s, net->gemm_dtype == QTT_BF16);
    if (e != hipSuccess) return e;
    h = w.H[l + 1];
    p += (int64_t)out * in + out;
  }
  return hipSuccess;
}

}  // namespace
}  // namespace qtt

using namespace qtt;

extern "C" int64_t qtt_mlp_param_count(int32_t nlayers, const int32_t *sizes) {
  if (nlayers < 1 || !sizes) return -1;
  return param_count(nlayers, sizes);
}

extern "C" qtt_status qtt_warmstart_workspace(const qtt_mlp *net, int32_t batch, int32_t ncores,
                                              const int32_t *nrow, const int32_t *ranks,
                                              const qtt_tt *metric, size_t *bytes) {
  qtt_status st = check_net(net);
  if (st != QTT_OK) return st;
  if (batch < 1 || !bytes) return fail(QTT_E_INVAL, "batch >= 1 and bytes required");
  TTShape sh;
  const TTShape *psh = nullptr;
  if (ncores > 0) {
    if ((st = make_shape(ncores, nrow, ranks, net->sizes[net->nlayers], sh)) != QTT_OK) return st;
    psh = &sh;
  }
  OpShape op;
  if (psh && (st = check_metric(metric, sh, op)) != QTT_OK) return st;
  if (metric && net->loss == QTT_LOSS_CORES)
    return fail(QTT_E_INVAL, "QTT_LOSS_CORES takes no metric");
  Arena ar;
  ar.dry = true;
  MlpWs w;
  carve_mlp(ar, net, batch, psh, w, (psh && metric) ? metric->ranks : nullptr);
  *bytes = ar.used + 256;
  return QTT_OK;
}

extern "C" qtt_status qtt_warmstart_infer(const qtt_mlp *net, const float *a, int32_t batch,
                                          float *out, void *ws, size_t ws_bytes, void *stream) {
  qtt::clear_stale_error();
  qtt_status st = check_net(net);
  if (st != QTT_OK) return st;
  if (!a || !out || batch < 1) return fail(QTT_E_INVAL, "a, out and batch >= 1 required");
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  MlpWs w;
  if (!ws || !carve_mlp(ar, net, batch, nullptr, w))
    return fail(QTT_E_CAPACITY, "workspace too small for qtt_warmstart_infer");
  hipStream_t s = (hipStream_t)stream;
  QTT_HIP(forward(net, a, batch, w, s));
  const int nout = net->sizes[net->nlayers];
  QTT_HIP(hipMemcpyAsync(out, w.H[net->nlayers], sizeof(float) * (int64_t)nout * batch,
                         hipMemcpyDeviceToDevice, s));
  return QTT_OK;
}

namespace qtt {
namespace {

// one Adam step on a batch already in device memory; the batch's mean loss
// is left in w.lmean[0] (device), nothing is synchronised
qtt_status train_batch(qtt_mlp *net, const float *a, const float *targets, int batch,
                       const TTShape &sh, const OpShape *op, float lr, MlpWs &w, hipStream_t s) {
  const int nl = net->nlayers;
  QTT_HIP(forward(net, a, batch, w, s));
  // dL/dOut (mean over the batch) and the per-sample losses
  if (net->loss == QTT_LOSS_CORES)
    hipLaunchKernelGGL(k_core_loss_grad, dim3(batch), dim3(256), 0, s, w.H[nl], targets, w.dA,
                       w.loss, sh.off[sh.D], 1.0f / batch);
  else if (op)
    hipLaunchKernelGGL(k_tt_energy_loss_grad, dim3(batch), dim3(256), 0, s, w.H[nl], targets, w.dA,
                       w.loss, sh, *op, w.scratch, w.per_sample, w.env_cap, w.w_cap,
                       1.0f / batch, net->loss == QTT_LOSS_ANGLE ? 1 : 0);
  else
    hipLaunchKernelGGL(k_tt_loss_grad, dim3(batch), dim3(256), 0, s, w.H[nl], targets, w.dA,
                       w.loss, sh, w.scratch, w.per_sample, 1.0f / batch,
                       net->loss == QTT_LOSS_ANGLE ? 1 : 0);
  QTT_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(64), 0, s, w.loss, batch, w.lmean);
  // backward, last layer first; offsets of each layer's parameters
  std::vector<int64_t> off(nl + 1, 0);
  for (int l = 0; l < nl; ++l)
    off[l + 1] = off[l] + (int64_t)net->sizes[l + 1] * net->sizes[l] + net->sizes[l + 1];
  float *dcur = w.dA, *dnext = w.dB;
  const bool bf = net->gemm_dtype == QTT_BF16;
  for (int l = nl - 1; l >= 0; --l) {
    const int in = net->sizes[l], out = net->sizes[l + 1];
    const float *W = net->params + off[l];
    float *gW = w.grad + off[l], *gb = gW + (int64_t)out * in;
    const float *hprev = l == 0 ? a : w.H[l];
    // dW = dZ H_prev^T, db = rowsum(dZ)
    QTT_HIP(gemm(false, true, dcur, out, hprev, in, gW, out, out, in, batch, nullptr, 0, s, bf));
    hipLaunchKernelGGL(k_rowsum, dim3((out + 255) / 256), dim3(256), 0, s, dcur, out, batch, gb);
    QTT_HIP(hipGetLastError());
    if (l > 0) {
      // dH_prev = W^T dZ, then the ReLU mask of layer l
      QTT_HIP(gemm(true, false, W, out, dcur, out, dnext, in, in, batch, out, nullptr, 0, s, bf));
      const int64_t ne = (int64_t)in * batch;
      hipLaunchKernelGGL(k_relu_mask, dim3((int)std::min<int64_t>((ne + 255) / 256, 4096)),
                         dim3(256), 0, s, dnext, w.H[l], ne);
      QTT_HIP(hipGetLastError());
      std::swap(dcur, dnext);
    }
  }
  const int64_t np = off[nl];
  const double t = (double)(net->step + 1);
  const float c1 = (float)(1.0 - std::pow(0.9, t)), c2 = (float)(1.0 - std::pow(0.999, t));
  hipLaunchKernelGGL(k_adam, dim3((int)std::min<int64_t>((np + 255) / 256, 8192)), dim3(256), 0,
                     s, net->params, w.grad, net->adam_m, net->adam_v, np, lr, c1, c2);
  QTT_HIP(hipGetLastError());
  net->step += 1;
  return QTT_OK;
}

// dst[:, j] = src[:, idx[j]] for FP32 columns of length len
__global__ void k_gather_cols(const float *src, const int *idx, int len, int ncols, float *dst) {
  const int64_t ne = (int64_t)len * ncols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / len), r = (int)(e % len);
    dst[e] = src[r + (int64_t)len * idx[j]];
  }
}

// acc[0] += c * v[0]
__global__ void k_accum(double *acc, const double *v, double c) { acc[0] += c * v[0]; }
__global__ void k_zero1(double *p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}
// FP32 column -> FP64 train
__global__ void k_f32_to_f64(const float *src, double *dst, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (double)src[e];
}

uint64_t splitmix64(uint64_t &x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace
}  // namespace qtt

extern "C" qtt_status qtt_warmstart_train_step(qtt_mlp *net, const float *a, const float *targets,
                                               int32_t batch, int32_t ncores, const int32_t *nrow,
                                               const int32_t *ranks, const qtt_tt *metric,
                                               float lr, double *loss, void *ws, size_t ws_bytes,
                                               void *stream) {
  qtt::clear_stale_error();
  qtt_status st = check_net(net);
  if (st != QTT_OK) return st;
  if (!a || !targets || batch < 1) return fail(QTT_E_INVAL, "a, targets and batch >= 1 required");
  if (!net->adam_m || !net->adam_v) return fail(QTT_E_INVAL, "Adam moments are NULL");
  if (!(lr > 0.f)) return fail(QTT_E_INVAL, "lr must be > 0");
  const int nl = net->nlayers;
  TTShape sh;
  if ((st = make_shape(ncores, nrow, ranks, net->sizes[nl], sh)) != QTT_OK) return st;
  OpShape op;
  if ((st = check_metric(metric, sh, op)) != QTT_OK) return st;
  if (metric && net->loss == QTT_LOSS_CORES)
    return fail(QTT_E_INVAL, "QTT_LOSS_CORES takes no metric");
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  MlpWs w;
  if (!ws || !carve_mlp(ar, net, batch, &sh, w, metric ? metric->ranks : nullptr))
    return fail(QTT_E_CAPACITY, "workspace too small for qtt_warmstart_train_step");
  hipStream_t s = (hipStream_t)stream;
  if ((st = train_batch(net, a, targets, batch, sh, metric ? &op : nullptr, lr, w, s)) != QTT_OK)
    return st;
  double lm = 0.0;
  QTT_HIP(hipMemcpyAsync(&lm, w.lmean, sizeof(double), hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));
  if (loss) *loss = lm;
  return QTT_OK;
}

extern "C" qtt_status qtt_warmstart_fit_workspace(const qtt_mlp *net, int32_t n, int32_t batch,
                                                  int32_t ncores, const int32_t *nrow,
                                                  const int32_t *ranks, const qtt_tt *metric,
                                                  size_t *bytes) {
  qtt_status st = qtt_warmstart_workspace(net, batch, ncores, nrow, ranks, metric, bytes);
  if (st != QTT_OK) return st;
  if (n < 1) return fail(QTT_E_INVAL, "n >= 1 required");
  const int nin = net->sizes[0], nout = net->sizes[net->nlayers];
  // batch copies of inputs and targets, the sample order, the epoch losses
  *bytes += 256 * 6 + sizeof(float) * ((int64_t)nin + nout) * batch + sizeof(int) * (int64_t)n +
            sizeof(double) * 4096;
  return QTT_OK;
}

extern "C" qtt_status qtt_warmstart_fit(qtt_mlp *net, const float *a, const float *targets,
                                        int32_t n, int32_t batch, int32_t epochs, float lr,
                                        float lr_final, uint64_t seed, int32_t ncores,
                                        const int32_t *nrow, const int32_t *ranks,
                                        const qtt_tt *metric, double *loss_hist, void *ws,
                                        size_t ws_bytes, void *stream) {
  qtt::clear_stale_error();
  qtt_status st = check_net(net);
  if (st != QTT_OK) return st;
  if (!a || !targets || n < 1 || batch < 1 || batch > n || epochs < 1 || epochs > 4096)
    return fail(QTT_E_INVAL, "a, targets, 1 <= batch <= n and 1 <= epochs <= 4096 required");
  if (!net->adam_m || !net->adam_v) return fail(QTT_E_INVAL, "Adam moments are NULL");
  if (!(lr > 0.f) || !(lr_final > 0.f)) return fail(QTT_E_INVAL, "lr and lr_final must be > 0");
  const int nl = net->nlayers;
  const int nin = net->sizes[0], nout = net->sizes[nl];
  TTShape sh;
  if ((st = make_shape(ncores, nrow, ranks, nout, sh)) != QTT_OK) return st;
  OpShape op;
  if ((st = check_metric(metric, sh, op)) != QTT_OK) return st;
  if (metric && net->loss == QTT_LOSS_CORES)
    return fail(QTT_E_INVAL, "QTT_LOSS_CORES takes no metric");
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  MlpWs w;
  bool ok = ws && carve_mlp(ar, net, batch, &sh, w, metric ? metric->ranks : nullptr);
  float *ab = (float *)ar.take(sizeof(float) * (int64_t)nin * batch);
  float *tb = (float *)ar.take(sizeof(float) * (int64_t)nout * batch);
  int *order = (int *)ar.take(sizeof(int) * (int64_t)n);
  double *hist = (double *)ar.take(sizeof(double) * 4096);
  if (!ok || !ar.ok()) return fail(QTT_E_CAPACITY, "workspace too small for qtt_warmstart_fit");
  hipStream_t s = (hipStream_t)stream;
  const int nb = n / batch;          // full batches per epoch (the rest is reshuffled)
  const int64_t steps = (int64_t)nb * epochs;
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  uint64_t rs = seed;
  hipLaunchKernelGGL(k_zero1, dim3(1), dim3(256), 0, s, hist, epochs);
  int64_t step = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    // Fisher-Yates shuffle with splitmix64 (Steele, Lea and Flood 2014)
    for (int i = n - 1; i > 0; --i) {
      const int j = (int)(splitmix64(rs) % (uint64_t)(i + 1));
      std::swap(perm[i], perm[j]);
    }
    QTT_HIP(hipMemcpyAsync(order, perm.data(), sizeof(int) * (int64_t)n, hipMemcpyHostToDevice, s));
    for (int b = 0; b < nb; ++b, ++step) {
      const int gb = (int)std::min<int64_t>(((int64_t)nin * batch + 255) / 256, 2048);
      hipLaunchKernelGGL(k_gather_cols, dim3(gb), dim3(256), 0, s, a, order + (int64_t)b * batch,
                         nin, batch, ab);
      const int gt = (int)std::min<int64_t>(((int64_t)nout * batch + 255) / 256, 4096);
      hipLaunchKernelGGL(k_gather_cols, dim3(gt), dim3(256), 0, s, targets,
                         order + (int64_t)b * batch, nout, batch, tb);
      QTT_HIP(hipGetLastError());
      // cosine decay of the learning rate from lr to lr_final
      const double fr = steps > 1 ? (double)step / (double)(steps - 1) : 1.0;
      const float lrs = (float)(lr_final + 0.5 * (lr - lr_final) * (1.0 + std::cos(M_PI * fr)));
      if ((st = train_batch(net, ab, tb, batch, sh, metric ? &op : nullptr, lrs, w, s)) != QTT_OK)
        return st;
      hipLaunchKernelGGL(k_accum, dim3(1), dim3(1), 0, s, hist + ep, w.lmean, 1.0 / nb);
    }
    // the host order array is reused next epoch: wait for its copy
    QTT_HIP(hipStreamSynchronize(s));
  }
  if (loss_hist)
    QTT_HIP(hipMemcpyAsync(loss_hist, hist, sizeof(double) * epochs, hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));
  return QTT_OK;
}

extern "C" qtt_status qtt_warmstart_infer_tt(const qtt_mlp *net, const float *a, int32_t ncores,
                                             const int32_t *nrow, const int32_t *ranks,
                                             qtt_tt *x0, void *ws, size_t ws_bytes, void *stream) {
  qtt::clear_stale_error();
  qtt_status st = check_net(net);
  if (st != QTT_OK) return st;
  if (!a || !x0 || !x0->data || !x0->ranks || !x0->nrow || x0->ncol)
    return fail(QTT_E_INVAL, "a and a vector x0 required");
  const int nout = net->sizes[net->nlayers];
  TTShape sh;
  if ((st = make_shape(ncores, nrow, ranks, nout, sh)) != QTT_OK) return st;
  if (x0->ncores != ncores) return fail(QTT_E_SHAPE, "x0 core count differs");
  for (int k = 0; k < ncores; ++k)
    if (x0->nrow[k] != nrow[k]) return fail(QTT_E_SHAPE, "x0 modes differ");
  if (x0->capacity < nout) return fail(QTT_E_CAPACITY, "x0: capacity below the packed size");
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  MlpWs w;
  if (!ws || !carve_mlp(ar, net, 1, nullptr, w))
    return fail(QTT_E_CAPACITY, "workspace too small for qtt_warmstart_infer_tt");
  hipStream_t s = (hipStream_t)stream;
  QTT_HIP(forward(net, a, 1, w, s));
  hipLaunchKernelGGL(k_f32_to_f64, dim3((int)std::min<int64_t>((nout + 255) / 256, 1024)),
                     dim3(256), 0, s, w.H[net->nlayers], x0->data, (int64_t)nout);
  QTT_HIP(hipGetLastError());
  for (int k = 0; k <= ncores; ++k) x0->ranks[k] = ranks[k];
  QTT_HIP(publish_ranks(x0, s));
  return QTT_OK;
}
