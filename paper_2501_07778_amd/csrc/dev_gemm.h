// dev_gemm.h — FP64 GEMM tile shared by the kernels (device code only).
// C = op(A) B for column-major operands: 64x64 output tile per 256-thread
// block, K staged through LDS in steps of 16, 4x4 outputs per thread.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtt {
namespace dev {

constexpr int GT = 64, GK = 16;

template <bool TA>
__device__ void gemm_tile(const double *A, int lda, const double *B, int ldb, double *C,
                          int ldc, int M, int N, int K, int tm, int tn) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tid = threadIdx.x;
  const int tr = tid % 16, tc = tid / 16;
  double acc[4][4] = {};
  const int m0 = tm * GT, n0 = tn * GT;
  for (int k0 = 0; k0 < K; k0 += GK) {
    for (int e = tid; e < GK * GT; e += 256) {
      const int mm = e % GT, kk = e / GT;
      const int gm = m0 + mm, gk = k0 + kk;
      double av = 0.0;
      if (gm < M && gk < K) av = TA ? A[gk + (int64_t)lda * gm] : A[gm + (int64_t)lda * gk];
      As[kk][mm] = av;
      const int kk2 = e % GK, nn = e / GK;
      const int gk2 = k0 + kk2, gn = n0 + nn;
      Bs[kk2][nn] = (gk2 < K && gn < N) ? B[gk2 + (int64_t)ldb * gn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = As[kk][tr + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = Bs[kk][tc + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gm = m0 + tr + 16 * u, gn = n0 + tc + 16 * v;
      if (gm < M && gn < N) C[gm + (int64_t)ldc * gn] = acc[u][v];
    }
}

typedef double dbl4_t __attribute__((ext_vector_type(4)));
constexpr int MK = 32;   // depth staged per step of the matrix-core tile

// The same 64 x 64 output tile on the FP64 matrix cores: each of the four
// wavefronts owns a 32 x 32 quarter as 2 x 2 blocks of
// v_mfma_f64_16x16x4f64 (A operand: lane l holds row l%16 at depth l/16;
// B operand likewise for the column; result element v of lane l is row
// l/16 + 4v of column l%16).  Depth is staged through LDS in steps of MK,
// loaded so that consecutive threads read consecutive addresses.
template <bool TA>
__device__ void gemm_tile_mfma(const double *A, int lda, const double *B, int ldb, double *C,
                               int ldc, int M, int N, int K, int tm, int tn) {
  __shared__ double As[GT][MK + 1];
  __shared__ double Bs[GT][MK + 1];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int rr = lane & 15, kq = lane >> 4;
  const int m0 = tm * GT, n0 = tn * GT;
  dbl4_t acc00 = {0.0, 0.0, 0.0, 0.0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
  for (int k0 = 0; k0 < K; k0 += MK) {
    __syncthreads();
    for (int e = threadIdx.x; e < GT * MK; e += 256) {
      int mm, kk;
      if (TA) {
        kk = e % MK;
        mm = e / MK;
      } else {
        mm = e % GT;
        kk = e / GT;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      double av = 0.0;
      if (gm < M && gk < K) av = TA ? A[gk + (int64_t)lda * gm] : A[gm + (int64_t)lda * gk];
      As[mm][kk] = av;
      const int kb = e % MK, nn = e / MK;
      const int gn = n0 + nn, gkb = k0 + kb;
      Bs[nn][kb] = (gkb < K && gn < N) ? B[gkb + (int64_t)ldb * gn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < MK; kk += 4) {
      const double a0 = As[wr + rr][kk + kq], a1 = As[wr + 16 + rr][kk + kq];
      const double b0 = Bs[wc + rr][kk + kq], b1 = Bs[wc + 16 + rr][kk + kq];
      acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc01, 0, 0, 0);
      acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc10, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc11, 0, 0, 0);
    }
  }
  const dbl4_t accs[2][2] = {{acc00, acc01}, {acc10, acc11}};
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wr + 16 * bi + kq + 4 * v, gn = n0 + wc + 16 * bj + rr;
        if (gm < M && gn < N) C[gm + (int64_t)ldc * gn] = accs[bi][bj][v];
      }
}

// A matrix-core tile of other shapes: TM = 16 BM WM rows by TN = 16 BN WN
// columns, wavefront w owning rows (w % WM) 16 BM .. and columns (w / WM)
// 16 BN .. as BM x BN blocks of v_mfma_f64_16x16x4f64 (operand and result
// layouts as above).  An 80-wide side (5 blocks) holds the 72-wide sketch
// dimension with 10 % padding where 64 x 64 tiles need two tiles, 44 %
// empty.  The next depth step's operands are loaded into registers while
// the current step is multiplied out of LDS.
template <bool TA, int WM, int WN, int BM, int BN>
__device__ void gemm_tile_mfma_w(const double *A, int lda, const double *B, int ldb, double *C,
                                 int ldc, int M, int N, int K, int tm, int tn) {
  static_assert(WM * WN == 4, "four wavefronts per tile");
  constexpr int TM = 16 * BM * WM, TN = 16 * BN * WN;
  static_assert((TM * MK) % 256 == 0 && (TN * MK) % 256 == 0, "whole loads per thread");
  constexpr int NA = TM * MK / 256, NB = TN * MK / 256;
  __shared__ double As[TM][MK + 1];
  __shared__ double Bs[TN][MK + 1];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int wr = (w % WM) * 16 * BM, wc = (w / WM) * 16 * BN;
  const int rr = lane & 15, kq = lane >> 4;
  const int m0 = tm * TM, n0 = tn * TN;
  dbl4_t acc[BM][BN];
#pragma unroll
  for (int bm = 0; bm < BM; ++bm)
#pragma unroll
    for (int bn = 0; bn < BN; ++bn) acc[bm][bn] = dbl4_t{0.0, 0.0, 0.0, 0.0};
  double ra[NA], rb[NB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + 256 * i;
      const int mm = TA ? e / MK : e % TM, kk = TA ? e % MK : e / TM;
      const int gm = m0 + mm, gk = k0 + kk;
      ra[i] = (gm < M && gk < K) ? (TA ? A[gk + (int64_t)lda * gm] : A[gm + (int64_t)lda * gk])
                                 : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + 256 * i;
      const int kb = e % MK, nn = e / MK;
      const int gk = k0 + kb, gn = n0 + nn;
      rb[i] = (gk < K && gn < N) ? B[gk + (int64_t)ldb * gn] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += MK) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + 256 * i;
      As[TA ? e / MK : e % TM][TA ? e % MK : e / TM] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + 256 * i;
      Bs[e / MK][e % MK] = rb[i];
    }
    __syncthreads();
    if (k0 + MK < K) fetch(k0 + MK);
#pragma unroll
    for (int kk = 0; kk < MK; kk += 4) {
      double a[BM], b[BN];
#pragma unroll
      for (int bm = 0; bm < BM; ++bm) a[bm] = As[wr + 16 * bm + rr][kk + kq];
#pragma unroll
      for (int bn = 0; bn < BN; ++bn) b[bn] = Bs[wc + 16 * bn + rr][kk + kq];
#pragma unroll
      for (int bm = 0; bm < BM; ++bm)
#pragma unroll
        for (int bn = 0; bn < BN; ++bn)
          acc[bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bm], b[bn], acc[bm][bn], 0, 0, 0);
    }
  }
#pragma unroll
  for (int bm = 0; bm < BM; ++bm)
#pragma unroll
    for (int bn = 0; bn < BN; ++bn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wr + 16 * bm + kq + 4 * v, gn = n0 + wc + 16 * bn + rr;
        if (gm < M && gn < N) C[gm + (int64_t)ldc * gn] = acc[bm][bn][v];
      }
}

// the two shapes the sketch uses: 64 x 80 (an 80-wide output column range)
// and 80 x 64 (an 80-wide output row range)
struct TileN80 {
  static constexpr int TM = 64, TN = 80, WM = 4, WN = 1, BM = 1, BN = 5;
};
struct TileM80 {
  static constexpr int TM = 80, TN = 64, WM = 1, WN = 4, BM = 5, BN = 1;
};

// Split-K product on such a tile (see gemm_tile_k below for the layout of
// the partials)
template <bool TA, class TS>
__device__ void gemm_tile_k_w(const double *A, int lda, const double *B, int ldb, double *P,
                              int M, int N, int K, int tm, int tn, int z, int kc) {
  const int per = (K + (int)gridDim.z - 1) / (int)gridDim.z;
  kc = per > kc ? per : kc;
  const int k0 = z * kc;
  const int kk = (K - k0) < kc ? (K - k0) : kc;
  if (kk <= 0) {
    for (int e = threadIdx.x; e < TS::TM * TS::TN; e += 256) {
      const int gm = tm * TS::TM + e % TS::TM, gn = tn * TS::TN + e / TS::TM;
      if (gm < M && gn < N) P[(int64_t)z * M * N + gm + (int64_t)M * gn] = 0.0;
    }
    return;
  }
  const double *Ak = TA ? A + k0 : A + (int64_t)lda * k0;
  gemm_tile_mfma_w<TA, TS::WM, TS::WN, TS::BM, TS::BN>(Ak, lda, B + k0, ldb,
                                                       P + (int64_t)z * M * N, M, M, N, kk, tm,
                                                       tn);
}

// Split-K variant: block z handles the K range [z*kc, (z+1)*kc) and writes
// its partial product to P + z*ldc*N (ldc = M); the partials are summed by
// splitk_reduce.  Thin products (few output tiles, long K) need this to keep
// enough blocks in flight.
template <bool TA>
__device__ void gemm_tile_k(const double *A, int lda, const double *B, int ldb, double *P,
                            int M, int N, int K, int tm, int tn, int z, int kc) {
  // every split takes at least kc; more when K needs more than gridDim.z splits
  const int per = (K + (int)gridDim.z - 1) / (int)gridDim.z;
  kc = per > kc ? per : kc;
  const int k0 = z * kc;
  const int kk = (K - k0) < kc ? (K - k0) : kc;
  if (kk <= 0) {
    // empty range: write zeros so the reduction stays uniform
    for (int e = threadIdx.x; e < GT * GT; e += 256) {
      const int gm = tm * GT + e % GT, gn = tn * GT + e / GT;
      if (gm < M && gn < N) P[(int64_t)z * M * N + gm + (int64_t)M * gn] = 0.0;
    }
    return;
  }
  const double *Ak = TA ? A + k0 : A + (int64_t)lda * k0;
  gemm_tile_mfma<TA>(Ak, lda, B + k0, ldb, P + (int64_t)z * M * N, M, M, N, kk, tm, tn);
}

}  // namespace dev
}  // namespace qtt
