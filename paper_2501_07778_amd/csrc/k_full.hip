// k_full.hip — dense vector of a tensor train, for the FP64 residual check
// of the solve, gfx950.
//
// The dense vector is the product of a left and a right partial contraction,
//   x = L_m R_m,  L_{k+1} = L_k G_k  (rows (i_0..i_k), column r_{k+1}),
//                 R_k = G_k R_{k+1}  (row r_k, columns (i_k..i_{D-1})),
// each a column-major GEMM on the cores as stored (left rank fastest), so
// the contraction is exact up to FP64 rounding.  The split m balances the
// two halves.
#include <algorithm>

#include "dev_gemm.h"
#include "internal.h"

namespace qtt {

namespace {

using dev::GT;

__global__ void __launch_bounds__(256) k_gemm(const double *A, int lda, const double *B,
                                              int ldb, double *C, int ldc, int M, int N,
                                              int K) {
  dev::gemm_tile<false>(A, lda, B, ldb, C, ldc, M, N, K, blockIdx.x, blockIdx.y);
}

hipError_t gemm(const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                int64_t M, int64_t N, int64_t K, hipStream_t s) {
  const int64_t mt = (M + GT - 1) / GT, nt = (N + GT - 1) / GT;
  // grid.y is limited to 65535 tiles: split wide products
  for (int64_t n0 = 0; n0 < nt; n0 += 65535) {
    const int64_t nn = std::min<int64_t>(nt - n0, 65535);
    const int64_t ncols = std::min<int64_t>(N - n0 * GT, nn * GT);
    hipLaunchKernelGGL(k_gemm, dim3((unsigned)mt, (unsigned)nn), dim3(256), 0, s, A, lda,
                       B + (int64_t)ldb * n0 * GT, ldb, C + (int64_t)ldc * n0 * GT, ldc,
                       (int)M, (int)ncols, (int)K);
  }
  return hipGetLastError();
}

__global__ void k_diff_norm2(const double *a, const double *b, int64_t n, double *out) {
  __shared__ double r0[256], r1[256];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const double d = a[e] - (b ? b[e] : 0.0);
    s0 = fma(d, d, s0);
    s1 = fma(a[e], a[e], s1);
  }
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = r0[0];
    out[1] = r1[0];
  }
}

struct Split {
  int m;
  int64_t lmax, rmax;
};

Split choose_split(const TTView &v, const int32_t *rk) {
  const int D = v.D;
  Split best{1, 0, 0};
  double bestc = 1e300;
  for (int m = 1; m < D; ++m) {
    int64_t NL = 1, lmax = 1, NR = 1, rmax = 1;
    for (int k = 0; k < m; ++k) {
      NL *= (int64_t)v.n[k] * v.m[k];
      lmax = std::max<int64_t>(lmax, NL * rk[k + 1]);
    }
    for (int k = D - 1; k >= m; --k) {
      NR *= (int64_t)v.n[k] * v.m[k];
      rmax = std::max<int64_t>(rmax, NR * rk[k]);
    }
    const double c = (double)lmax + (double)rmax;
    if (c < bestc) {
      bestc = c;
      best = Split{m, lmax, rmax};
    }
  }
  return best;
}

}  // namespace

int64_t full_ws_elems(const TTView &v, const int32_t *rk) {
  if (v.D == 1) return 64;
  Split sp = choose_split(v, rk);
  return 2 * ((sp.lmax + 31) & ~int64_t(31)) + 2 * ((sp.rmax + 31) & ~int64_t(31)) + 256;
}

hipError_t tt_full(const TTView &v, const int32_t *rk, double *out, double *ws, hipStream_t s) {
  const int D = v.D;
  if (D == 1) {
    return hipMemcpyAsync(out, v.data + v.off[0], sizeof(double) * v.n[0] * v.m[0],
                          hipMemcpyDeviceToDevice, s);
  }
  Split sp = choose_split(v, rk);
  const int64_t la = (sp.lmax + 31) & ~int64_t(31), ra = (sp.rmax + 31) & ~int64_t(31);
  double *Lb[2] = {ws, ws + la};
  double *Rb[2] = {ws + 2 * la, ws + 2 * la + ra};
  hipError_t e;
  // left: L_1 = core 0 (n_0 x r_1)
  const double *L = v.data + v.off[0];
  int64_t NL = (int64_t)v.n[0] * v.m[0];
  int li = 0;
  for (int k = 1; k < sp.m; ++k) {
    const int nk = v.n[k] * v.m[k];
    // (NL x r_k) (r_k x nk r_{k+1})
    if ((e = gemm(L, (int)NL, v.data + v.off[k], rk[k], Lb[li], (int)NL, NL,
                  (int64_t)nk * rk[k + 1], rk[k], s)) != hipSuccess)
      return e;
    L = Lb[li];
    li = 1 - li;
    NL *= nk;
  }
  // right: R_{D-1} = core D-1 (r_{D-1} x n_{D-1})
  const double *R = v.data + v.off[D - 1];
  int64_t NR = (int64_t)v.n[D - 1] * v.m[D - 1];
  int ri = 0;
  for (int k = D - 2; k >= sp.m; --k) {
    const int nk = v.n[k] * v.m[k];
    // (r_k nk x r_{k+1}) (r_{k+1} x NR)
    if ((e = gemm(v.data + v.off[k], rk[k] * nk, R, rk[k + 1], Rb[ri], rk[k] * nk,
                  (int64_t)rk[k] * nk, NR, rk[k + 1], s)) != hipSuccess)
      return e;
    R = Rb[ri];
    ri = 1 - ri;
    NR *= nk;
  }
  // x = L (NL x r_m) R (r_m x NR)
  return gemm(L, (int)NL, R, rk[sp.m], out, (int)NL, NL, NR, rk[sp.m], s);
}

hipError_t launch_diff_norm2(const double *a, const double *b, int64_t n, double *out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_diff_norm2, dim3(1), dim3(256), 0, s, a, b, n, out);
  return hipGetLastError();
}

}  // namespace qtt
