// k_als.hip — alternating least squares (one-site ALS) on the QTT format,
// gfx950: the solve that works on the cores of the solution instead of
// rounding global residuals (the approach of the AMEn family the paper uses,
// without the residual enrichment; Holtz, Rohwedder and Schneider, SIAM J.
// Sci. Comput. 2012).
//
// With the cores left of k left-orthogonal and right of k right-orthogonal,
// core k minimises the energy <x, K x>/2 - <x, f> exactly by solving the
// projected system B y = g, where
//   B[(a,i,b),(a',j,b')] = sum_{al,be} L[a,al,a'] K_k[al,i,j,be] R[b,be,b'],
//   g[(a,i,b)]           = sum_{c,d} Lf[a,c] F_k[c,i,d] Rf[b,d],
// with L/R the left/right environments of <x, K x> and Lf/Rf those of <x, f>.
// B is symmetric positive definite (K is, the frames are orthonormal); it is
// factored by a blocked right-looking Cholesky (CB-wide panels: the diagonal
// block factored in one wavefront, the panel rows solved against it, the
// forward substitution of g folded into both, an FP64 MFMA trailing update
// deferred over strips), then solved backward.  After the solve the core is
// orthogonalised (QR or LQ) and the environments move one core on.
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "internal.h"

namespace qtt {
namespace {

constexpr int CB = 32;       // Cholesky panel width (<= 64: one wavefront per panel)
constexpr int AWG = 256;

// ---------------------------------------------------------------- envs
// Environments are contracted in three (or two) grid-stride stages, each a
// plain sum over one or two indices; every stage writes its whole result.
//
// left step of <x, A y>: P'[b, be, b'] = sum X[a,i,b] A[al,i,j,be] Y[a',j,b'] P[a,al,a']
// stage 1: W1[a, al, j, b'] = sum_a' P[a, al, a'] Y[a', j, b']
__global__ void k_e3l_1(const double *P, const double *Y, double *W1, int r0, int ra0, int n,
                        int r1) {
  const int64_t ne = (int64_t)r0 * ra0 * n * r1, ra = (int64_t)r0 * ra0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t aal = e % ra, jb = e / ra;
    const double *yc = Y + (int64_t)r0 * jb;
    double acc = 0.0;
    for (int a2 = 0; a2 < r0; ++a2) acc = fma(P[aal + ra * a2], yc[a2], acc);
    W1[e] = acc;
  }
}
// stage 2: W2[a, i, be, b'] = sum_{j, al} W1[a, al, j, b'] A[al, i, j, be]
__global__ void k_e3l_2(const double *W1, const double *A, double *W2, int r0, int ra0, int n,
                        int ra1, int r1) {
  const int64_t ne = (int64_t)r0 * n * ra1 * r1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % r0);
    int64_t t = e / r0;
    const int i = (int)(t % n);
    t /= n;
    const int be = (int)(t % ra1);
    const int64_t b2 = t / ra1;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
      const double *w = W1 + a + (int64_t)r0 * ra0 * (j + (int64_t)n * b2);
      const double *av = A + (int64_t)ra0 * (i + (int64_t)n * (j + (int64_t)n * be));
      for (int al = 0; al < ra0; ++al) acc = fma(w[(int64_t)r0 * al], av[al], acc);
    }
    W2[e] = acc;
  }
}
// stage 3: P'[b, c] = sum_l X[l, b] W[l, c] over l < L (the row pairs (a, i))
__global__ void k_e_close(const double *X, const double *Wm, double *Pn, int L, int r1,
                          int64_t ncol) {
  const int64_t ne = (int64_t)r1 * ncol;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e % r1);
    const int64_t col = e / r1;
    const double *xb = X + (int64_t)L * b, *wc = Wm + (int64_t)L * col;
    double acc = 0.0;
    for (int l = 0; l < L; ++l) acc = fma(xb[l], wc[l], acc);
    Pn[e] = acc;
  }
}

// right step of <x, A y>: P[a, al, a'] from P'[b, be, b']
// stage 1: V1[a, i, c] = sum_b X[a, i, b] P'[b, c] over the column index c
__global__ void k_e_open(const double *X, const double *Pn, double *V1, int r0n, int r1,
                         int64_t ncol) {
  const int64_t ne = (int64_t)r0n * ncol;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ai = e % r0n, c = e / r0n;
    double acc = 0.0;
    for (int b = 0; b < r1; ++b) acc = fma(X[ai + (int64_t)r0n * b], Pn[b + (int64_t)r1 * c], acc);
    V1[e] = acc;
  }
}
// stage 2: V2[a, al, j, b'] = sum_{be, i} V1[a, i, be, b'] A[al, i, j, be]
__global__ void k_e3r_2(const double *V1, const double *A, double *V2, int r0, int ra0, int n,
                        int ra1, int r1) {
  const int64_t ne = (int64_t)r0 * ra0 * n * r1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % r0);
    int64_t t = e / r0;
    const int al = (int)(t % ra0);
    t /= ra0;
    const int j = (int)(t % n);
    const int64_t b2 = t / n;
    double acc = 0.0;
    for (int be = 0; be < ra1; ++be)
      for (int i = 0; i < n; ++i)
        acc = fma(V1[a + (int64_t)r0 * (i + (int64_t)n * (be + (int64_t)ra1 * b2))],
                  A[al + (int64_t)ra0 * (i + (int64_t)n * (j + (int64_t)n * be))], acc);
    V2[e] = acc;
  }
}
// stage 3: P[a, al, a'] = sum_{j, b'} V2[a, al, j, b'] Y[a', j, b']
__global__ void k_e3r_3(const double *V2, const double *Y, double *P, int r0, int ra0, int n,
                        int r1) {
  const int64_t ra = (int64_t)r0 * ra0, ne = ra * r0;
  const int nb = n * r1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t aal = e % ra;
    const int a2 = (int)(e / ra);
    double acc = 0.0;
    for (int jb = 0; jb < nb; ++jb) acc = fma(V2[aal + ra * jb], Y[a2 + (int64_t)r0 * jb], acc);
    P[e] = acc;
  }
}

// left step of <x, f>, stage 1: T[a, i, d] = sum_c Q[a, c] F[c, i, d]
__global__ void k_e2l_1(const double *Q, const double *F, double *Tm, int r0, int rf0, int n,
                        int rf1) {
  const int64_t ne = (int64_t)r0 * n * rf1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % r0);
    const int64_t id = e / r0;
    double acc = 0.0;
    for (int c = 0; c < rf0; ++c) acc = fma(Q[a + (int64_t)r0 * c], F[c + (int64_t)rf0 * id], acc);
    Tm[e] = acc;
  }
}
// right step of <x, f>, stage 2: Q[a, c] = sum_{i, d} T[a, i, d] F[c, i, d]
__global__ void k_e2r_2(const double *Tm, const double *F, double *Q, int r0, int rf0, int n,
                        int rf1) {
  const int64_t ne = (int64_t)r0 * rf0;
  const int nd = n * rf1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % r0), c = (int)(e / r0);
    double acc = 0.0;
    for (int id = 0; id < nd; ++id)
      acc = fma(Tm[a + (int64_t)r0 * id], F[c + (int64_t)rf0 * id], acc);
    Q[e] = acc;
  }
}

// ---------------------------------------------------------------- local system
// T[a, a', i, j, be] = sum_al L[a, al, a'] K[al, i, j, be]
__global__ void k_local_T(const double *L, const double *K, double *T, int r0, int ra0, int n,
                          int ra1) {
  const int64_t ne = (int64_t)r0 * r0 * n * n * ra1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int aa = (int)(e % ((int64_t)r0 * r0));  // a + r0 a'
    const int64_t ijb = e / ((int64_t)r0 * r0);    // i + n (j + n be)
    const int a = aa % r0, a2 = aa / r0;
    double acc = 0.0;
    for (int al = 0; al < ra0; ++al)
      acc = fma(L[a + (int64_t)r0 * (al + (int64_t)ra0 * a2)], K[al + (int64_t)ra0 * ijb], acc);
    T[e] = acc;
  }
}

// B[p, q] = sum_be T[a, a', i, j, be] R[b, be, b'], p = a + r0 (i + n b),
// q = a' + r0 (j + n b'); N = r0 n r1
__global__ void k_local_B(const double *T, const double *R, double *B, int r0, int n, int ra1,
                          int r1) {
  const int64_t N = (int64_t)r0 * n * r1;
  const int64_t ne = N * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e % N, q = e / N;
    const int a = (int)(p % r0);
    const int i = (int)((p / r0) % n);
    const int b = (int)(p / ((int64_t)r0 * n));
    const int a2 = (int)(q % r0);
    const int j = (int)((q / r0) % n);
    const int b2 = (int)(q / ((int64_t)r0 * n));
    const double *t = T + (a + (int64_t)r0 * a2) + (int64_t)r0 * r0 * (i + (int64_t)n * j);
    const int64_t tstride = (int64_t)r0 * r0 * n * n;
    double acc = 0.0;
    for (int be = 0; be < ra1; ++be)
      acc = fma(t[tstride * be], R[b + (int64_t)r1 * (be + (int64_t)ra1 * b2)], acc);
    B[e] = acc;
  }
}

// g[a, i, b] = sum_{c, d} Lf[a, c] F[c, i, d] Rf[b, d]
__global__ void k_local_g(const double *Lf, const double *F, const double *Rf, double *g, int r0,
                          int rf0, int n, int r1, int rf1) {
  const int64_t N = (int64_t)r0 * n * r1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % r0);
    const int i = (int)((e / r0) % n);
    const int b = (int)(e / ((int64_t)r0 * n));
    double acc = 0.0;
    for (int d = 0; d < rf1; ++d) {
      double s = 0.0;
      for (int c = 0; c < rf0; ++c)
        s = fma(Lf[a + (int64_t)r0 * c], F[c + (int64_t)rf0 * (i + (int64_t)n * d)], s);
      acc = fma(s, Rf[b + (int64_t)r1 * d], acc);
    }
    g[e] = acc;
  }
}

// ---------------------------------------------------------------- Cholesky
// Blocked right-looking Cholesky B = L L^T with the forward substitution
// L z = g folded into the panel kernel, then a blocked backward
// substitution L^T y = z.  Panels are CB = 32 columns wide; the trailing
// update is deferred over strips of NB = 256 columns (inner updates touch
// only the strip), so the trailing matrix is read and written once per strip
// by an FP64 MFMA kernel.
constexpr int NB = 256;
typedef double dbl4 __attribute__((ext_vector_type(4)));

// One panel of the factorisation in one launch.  Every workgroup factors
// the diagonal block A[k0:k0+kb, k0:k0+kb] itself (one wavefront, lane i
// holds row i in registers, the active column broadcast through LDS; lanes
// kb..CB-1 carry an identity row, lanes >= CB a zero row) and forms
// z1 = L11^-1 g1, identically in every workgroup.  Workgroup 0 stores L11
// (CB x CB, column-major, in Ls) and z1 (in zs_out[k0..]); the diagonal
// block of A and g1 are only read, so no workgroup waits for another.  Then
// each workgroup solves its 64 rows below the panel (full panels only):
// A21 <- A21 L11^-T, and g2 <- g2 - A21 z1.  *flag becomes 1 when a pivot
// is not positive.
__global__ void __launch_bounds__(64) k_panel(double *A, int64_t N, int k0, int kb, double *g,
                                              double *Ls, double *zs_out, int *flag) {
  __shared__ double col[64];
  __shared__ double Lt[CB][CB + 1];
  __shared__ double zsh[CB], rd[CB];
  const int i = threadIdx.x;
  const bool live = i < kb;
  {
    double x[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j)
      x[j] = (live && j <= i) ? A[(k0 + i) + N * (k0 + j)] : (i == j ? 1.0 : 0.0);
    double gi = live ? g[k0 + i] : 0.0, diag = 1.0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const double piv = __shfl(x[j], j, 64);
      bad = bad || !(piv > 0.0);
      const double sq = sqrt(piv > 0.0 ? piv : 1.0);
      if (i == j) diag = sq;
      x[j] = (i == j) ? sq : (i > j ? x[j] / sq : 0.0);
      col[i] = x[j];
      __syncthreads();
#pragma unroll
      for (int l = j + 1; l < CB; ++l)
        if (i >= l) x[l] = fma(-x[j], col[l], x[l]);
      __syncthreads();
    }
    // forward substitution on the block: lane j finishes z_j, the lanes
    // below subtract its contribution
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const double zj = __shfl(gi / x[j], j, 64);
      if (i == j) gi = zj;
      else if (i > j) gi = fma(-x[j], zj, gi);
    }
    if (i < CB) {
#pragma unroll
      for (int j = 0; j < CB; ++j) Lt[i][j] = (j <= i) ? x[j] : 0.0;
      zsh[i] = gi;
      rd[i] = 1.0 / diag;
    }
    if (blockIdx.x == 0) {
      if (live) {
#pragma unroll
        for (int j = 0; j < CB; ++j) Ls[i + CB * j] = (j <= i) ? x[j] : 0.0;
        zs_out[k0 + i] = gi;
      }
      if (bad && i == 0) flag[0] = 1;
    }
  }
  __syncthreads();
  if (kb < CB) return;  // the last, partial panel has no rows below it
  const int64_t row = (int64_t)k0 + CB + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (row >= N) return;
  double x[CB];
#pragma unroll
  for (int j = 0; j < CB; ++j) x[j] = A[row + N * (k0 + j)];
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    double v = x[j];
#pragma unroll
    for (int l = 0; l < j; ++l) v = fma(-x[l], Lt[j][l], v);
    x[j] = v * rd[j];
  }
  double sg = 0.0;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    A[row + N * (k0 + j)] = x[j];
    sg = fma(x[j], zsh[j], sg);
  }
  g[row] -= sg;
}

// A[m, n] -= sum_{c in [kc0, kc0+kd)} A[m, c] A[n, c] for nb <= n < ne,
// n <= m < N (lower triangle), 64 x 64 output tiles per workgroup; each
// wavefront owns a 32 x 32 quarter as 2 x 2 blocks of
// v_mfma_f64_16x16x4f64 (A operand: lane l holds row l%16, depth l/16; B
// likewise for the column; result: element v of lane l is row l/16 + 4v of
// column l%16).  Depth is staged through LDS in chunks of KC.
constexpr int KC = 32;
__global__ void __launch_bounds__(256) k_syrk_mfma(double *A, int64_t N, int kc0, int kd, int nb,
                                                   int ne) {
  const int64_t m0 = nb + (int64_t)blockIdx.x * 64, n0 = nb + (int64_t)blockIdx.y * 64;
  if (n0 > m0 + 63) return;  // tile strictly above the diagonal
  __shared__ double As[64][KC + 1], Bs[64][KC + 1];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int rr = lane & 15, kq = lane >> 4;
  dbl4 acc00 = {0.0, 0.0, 0.0, 0.0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
  // thread t stages rows t%64 of depth columns t/64 + 4u (u < KC/4); the
  // next chunk is loaded into registers while the current one is multiplied
  constexpr int PER = 64 * KC / 256;
  const int sr = threadIdx.x & 63, sc = threadIdx.x >> 6;
  double pa[PER], pb[PER];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int c = sc + 4 * u;
      const bool cv = c0 + c < kd;
      const int64_t cc = N * (int64_t)(kc0 + c0 + c);
      pa[u] = (cv && m0 + sr < N) ? A[(m0 + sr) + cc] : 0.0;
      pb[u] = (cv && n0 + sr < N) ? A[(n0 + sr) + cc] : 0.0;
    }
  };
  fetch(0);
  for (int c0 = 0; c0 < kd; c0 += KC) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      As[sr][sc + 4 * u] = pa[u];
      Bs[sr][sc + 4 * u] = pb[u];
    }
    __syncthreads();
    if (c0 + KC < kd) fetch(c0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const double a0 = As[wr + rr][kk + kq], a1 = As[wr + 16 + rr][kk + kq];
      const double b0 = Bs[wc + rr][kk + kq], b1 = Bs[wc + 16 + rr][kk + kq];
      acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc01, 0, 0, 0);
      acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc10, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc11, 0, 0, 0);
    }
  }
  const dbl4 accs[2][2] = {{acc00, acc01}, {acc10, acc11}};
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gm = m0 + wr + 16 * bi + kq + 4 * v, gn = n0 + wc + 16 * bj + rr;
        if (gm < N && gn < ne && gm >= gn) A[gm + N * gn] -= accs[bi][bj][v];
      }
}

// backward substitution step for the block [k0, k0+kb): every workgroup
// solves L_bb^T y_b = z_b (one wavefront, shuffles; L_bb as stored by
// k_panel), workgroup 0 stores y_b,
// and each workgroup then updates its 128 entries of z below k0:
// z_i -= sum_j L[k0+j, i] y_j (8 lanes per i reading the CB contiguous
// entries of column i's block row).
constexpr int BWD_COLS = 128;
__global__ void __launch_bounds__(256) k_bwd(const double *A, int64_t N, int k0, int kb,
                                             const double *Lb, double *z, double *y) {
  __shared__ double Ls[CB][CB + 1];
  __shared__ double ys[CB], rd[CB];
  for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) {
    const int i = e % kb, j = e / kb;
    Ls[i][j] = (i >= j) ? Lb[i + CB * j] : 0.0;
  }
  if (threadIdx.x < kb) rd[threadIdx.x] = 1.0 / Lb[threadIdx.x * (CB + 1)];
  __syncthreads();
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    double v = l < kb ? z[k0 + l] : 0.0;
    for (int j = kb - 1; j >= 0; --j) {
      const double yj = __shfl(v, j, 64) * rd[j];
      if (l == j) v = yj;
      else if (l < j) v = fma(-Ls[j][l], yj, v);
    }
    if (l < kb) {
      ys[l] = v;
      if (blockIdx.x == 0) y[k0 + l] = v;
    }
  }
  __syncthreads();
  // 8 lanes per column: lane group q = lane / 8 owns column i, part p = lane % 8
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane >> 3, p = lane & 7;
  const int64_t ibase = (int64_t)blockIdx.x * BWD_COLS;
  for (int c = wave * 8 + q; c < BWD_COLS; c += 32) {
    const int64_t i = ibase + c;
    double s = 0.0;
    if (i < k0)
      for (int j = p; j < kb; j += 8) s = fma(A[(k0 + j) + N * i], ys[j], s);
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 4, 64);
    if (i < k0 && p == 0) z[i] -= s;
  }
}

// ---------------------------------------------------------------- QR
__device__ double blk_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  return t;
}

// Householder QR of W (rows x cols, ld rows, cols <= rows) in global memory
// (one block): R -> Rout (cols x cols), Q (rows x cols) -> W
__global__ void __launch_bounds__(AWG) k_qr_thin(double *W, int rows, int cols, double *Rout,
                                                 double *tau) {
  __shared__ double red[AWG / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = 0; j < cols; ++j) {
    double *wj = W + (int64_t)rows * j;
    double p = 0.0;
    for (int i = j + 1 + threadIdx.x; i < rows; i += blockDim.x) p += wj[i] * wj[i];
    const double xn2 = blk_sum(p, red);
    const double alpha = wj[j];
    double t = 0.0, beta = alpha, scale = 0.0;
    if (xn2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();
    if (t != 0.0)
      for (int i = j + 1 + threadIdx.x; i < rows; i += blockDim.x) wj[i] *= scale;
    if (threadIdx.x == 0) {
      wj[j] = beta;
      tau[j] = t;
    }
    __syncthreads();
    if (t != 0.0) {
      for (int c = j + 1 + wave; c < cols; c += nw) {
        double *wc = W + (int64_t)rows * c;
        double s = (lane == 0) ? wc[j] : 0.0;
        for (int i = j + 1 + lane; i < rows; i += 64) s += wj[i] * wc[i];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        s *= t;
        if (lane == 0) wc[j] -= s;
        for (int i = j + 1 + lane; i < rows; i += 64) wc[i] -= s * wj[i];
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < cols * cols; e += blockDim.x) {
    const int i = e % cols, c = e / cols;
    Rout[e] = (i <= c) ? W[i + (int64_t)rows * c] : 0.0;
  }
  __syncthreads();
  // form Q in place: apply the reflectors to the identity columns, last first;
  // the reflector of column j is kept in a register copy before overwriting
  for (int j = cols - 1; j >= 0; --j) {
    const double t = tau[j];
    double *wj = W + (int64_t)rows * j;
    // columns c > j already hold Q's columns; apply H_j to them
    if (t != 0.0) {
      for (int c = j + 1 + wave; c < cols; c += nw) {
        double *qc = W + (int64_t)rows * c;
        double s = 0.0;
        for (int i = j + 1 + lane; i < rows; i += 64) s += wj[i] * qc[i];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        s *= t;  // qc[j] is 0 before this reflector
        if (lane == 0) qc[j] = -s;
        for (int i = j + 1 + lane; i < rows; i += 64) qc[i] -= s * wj[i];
      }
    }
    __syncthreads();
    // column j of Q: H_j e_j = e_j - t v (v_j = 1)
    for (int i = threadIdx.x; i < rows; i += blockDim.x) {
      const double vi = (i < j) ? 0.0 : (i == j ? 1.0 : wj[i]);
      wj[i] = (i == j ? 1.0 : 0.0) - t * vi;
    }
    __syncthreads();
  }
}

// C (M x N) = A (M x K) B (K x N), or with B transposed; small, column-major
__global__ void k_gemm_small(const double *A, int lda, const double *B, int ldb, int tb, double *C,
                             int ldc, int M, int N, int K) {
  const int64_t ne = (int64_t)M * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(e % M), nn = (int)(e / M);
    double acc = 0.0;
    for (int k = 0; k < K; ++k)
      acc = fma(A[m + (int64_t)lda * k], tb ? B[nn + (int64_t)ldb * k] : B[k + (int64_t)ldb * nn],
                acc);
    C[m + (int64_t)ldc * nn] = acc;
  }
}

// deterministic start values (integer hash, uniform in [-1, 1)), scaled
__global__ void k_hash_fill(double *x, int64_t n, uint64_t seed, double scale) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(e + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[e] = scale * ((double)(z >> 11) * (1.0 / 4503599627370496.0) - 1.0);
  }
}

// out[0] = sum_i a[i] b[i] (one workgroup)
__global__ void __launch_bounds__(AWG) k_vdot(const double *a, const double *b, int64_t n,
                                              double *out) {
  __shared__ double red[AWG / 64];
  double p = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) p = fma(a[i], b[i], p);
  const double t = blk_sum(p, red);
  if (threadIdx.x == 0) out[0] = t;
}

// dst (cols x rows) = src (rows x cols)^T, column-major
__global__ void k_transpose(const double *src, int rows, int cols, double *dst) {
  const int64_t ne = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % rows), c = (int)(e / rows);
    dst[c + (int64_t)cols * r] = src[e];
  }
}

__global__ void k_fill_value(double *x, int64_t n, double v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = v;
}

// dst (r0d x n x r1d) = src (r0s x n x r1s) zero-padded
__global__ void k_pad_core(const double *src, int r0s, int n, int r1s, double *dst, int r0d,
                           int r1d) {
  const int64_t ne = (int64_t)r0d * n * r1d;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % r0d);
    const int i = (int)((e / r0d) % n);
    const int b = (int)(e / ((int64_t)r0d * n));
    dst[e] = (a < r0s && b < r1s) ? src[a + (int64_t)r0s * (i + (int64_t)n * b)] : 0.0;
  }
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t als_env3_left(const double *P, const double *X, const double *A, const double *Y,
                         double *Pn, double *W1, double *W2, int r0, int ra0, int n, int ra1,
                         int r1, hipStream_t s) {
  const int64_t n1 = (int64_t)r0 * ra0 * n * r1, n2 = (int64_t)r0 * n * ra1 * r1;
  hipLaunchKernelGGL(k_e3l_1, dim3(blocks_for(n1)), dim3(256), 0, s, P, Y, W1, r0, ra0, n, r1);
  hipLaunchKernelGGL(k_e3l_2, dim3(blocks_for(n2)), dim3(256), 0, s, W1, A, W2, r0, ra0, n, ra1,
                     r1);
  const int64_t nc = (int64_t)ra1 * r1;
  hipLaunchKernelGGL(k_e_close, dim3(blocks_for(r1 * nc)), dim3(256), 0, s, X, W2, Pn, r0 * n, r1,
                     nc);
  return hipGetLastError();
}
hipError_t als_env3_right(const double *Pn, const double *X, const double *A, const double *Y,
                          double *P, double *W1, double *W2, int r0, int ra0, int n, int ra1,
                          int r1, hipStream_t s) {
  const int64_t nc = (int64_t)ra1 * r1;
  hipLaunchKernelGGL(k_e_open, dim3(blocks_for((int64_t)r0 * n * nc)), dim3(256), 0, s, X, Pn, W1,
                     r0 * n, r1, nc);
  const int64_t n2 = (int64_t)r0 * ra0 * n * r1;
  hipLaunchKernelGGL(k_e3r_2, dim3(blocks_for(n2)), dim3(256), 0, s, W1, A, W2, r0, ra0, n, ra1,
                     r1);
  hipLaunchKernelGGL(k_e3r_3, dim3(blocks_for((int64_t)r0 * ra0 * r0)), dim3(256), 0, s, W2, Y, P,
                     r0, ra0, n, r1);
  return hipGetLastError();
}
hipError_t als_env2_left(const double *Q, const double *X, const double *F, double *Qn,
                         double *Tm, int r0, int rf0, int n, int r1, int rf1, hipStream_t s) {
  hipLaunchKernelGGL(k_e2l_1, dim3(blocks_for((int64_t)r0 * n * rf1)), dim3(256), 0, s, Q, F, Tm,
                     r0, rf0, n, rf1);
  hipLaunchKernelGGL(k_e_close, dim3(blocks_for((int64_t)r1 * rf1)), dim3(256), 0, s, X, Tm, Qn,
                     r0 * n, r1, (int64_t)rf1);
  return hipGetLastError();
}
hipError_t als_env2_right(const double *Qn, const double *X, const double *F, double *Q,
                          double *Tm, int r0, int rf0, int n, int r1, int rf1, hipStream_t s) {
  hipLaunchKernelGGL(k_e_open, dim3(blocks_for((int64_t)r0 * n * rf1)), dim3(256), 0, s, X, Qn, Tm,
                     r0 * n, r1, (int64_t)rf1);
  hipLaunchKernelGGL(k_e2r_2, dim3(blocks_for((int64_t)r0 * rf0)), dim3(256), 0, s, Tm, F, Q, r0,
                     rf0, n, rf1);
  return hipGetLastError();
}

hipError_t als_local_system(const double *L, const double *K, const double *R, const double *Lf,
                            const double *F, const double *Rf, double *T, double *B, double *g,
                            int r0, int ra0, int n, int ra1, int r1, int rf0, int rf1,
                            hipStream_t s) {
  const int64_t nt = (int64_t)r0 * r0 * n * n * ra1;
  hipLaunchKernelGGL(k_local_T, dim3(blocks_for(nt)), dim3(256), 0, s, L, K, T, r0, ra0, n, ra1);
  const int64_t N = (int64_t)r0 * n * r1;
  hipLaunchKernelGGL(k_local_B, dim3(blocks_for(N * N)), dim3(256), 0, s, T, R, B, r0, n, ra1, r1);
  hipLaunchKernelGGL(k_local_g, dim3(blocks_for(N)), dim3(256), 0, s, Lf, F, Rf, g, r0, rf0, n, r1,
                     rf1);
  return hipGetLastError();
}

// B (N x N, SPD) y = g: the part of B below the diagonal blocks is
// overwritten by the Cholesky factor, the diagonal blocks of L go to Lst
// (CB x CB each, ceil(N/CB) of them), z = L^-1 g to z (N), and y receives
// the solution; g is consumed.  zz (may be NULL) receives <z, z> = <y, g>.
hipError_t als_cholesky_solve(double *B, int64_t N, double *g, double *y, double *Lst, double *z,
                              int *flag, double *zz, hipStream_t s) {
  for (int64_t K0 = 0; K0 < N; K0 += NB) {
    const int64_t K1 = std::min<int64_t>(K0 + NB, N);
    for (int64_t k0 = K0; k0 < K1; k0 += CB) {
      const int kb = (int)std::min<int64_t>(CB, N - k0);
      const int64_t rest = N - k0 - kb;  // > 0 implies a full panel (kb == CB)
      const int groups = (int)std::max<int64_t>(1, (rest + 63) / 64);
      hipLaunchKernelGGL(k_panel, dim3(groups), dim3(64), 0, s, B, N, (int)k0, kb, g,
                         Lst + (k0 / CB) * CB * CB, z, flag);
      const int64_t nb = k0 + CB;
      if (rest > 0 && nb < K1)
        hipLaunchKernelGGL(k_syrk_mfma, dim3((int)((N - nb + 63) / 64), (int)((K1 - nb + 63) / 64)),
                           dim3(256), 0, s, B, N, (int)k0, CB, (int)nb, (int)K1);
    }
    if (K1 < N) {
      const int t = (int)((N - K1 + 63) / 64);
      hipLaunchKernelGGL(k_syrk_mfma, dim3(t, t), dim3(256), 0, s, B, N, (int)K0, (int)(K1 - K0),
                         (int)K1, (int)N);
    }
  }
  if (zz) hipLaunchKernelGGL(k_vdot, dim3(1), dim3(AWG), 0, s, z, z, N, zz);
  const int64_t nblk = (N + CB - 1) / CB;
  for (int64_t b = nblk - 1; b >= 0; --b) {
    const int64_t k0 = b * CB;
    const int kb = (int)std::min<int64_t>(CB, N - k0);
    const int groups = (int)std::max<int64_t>(1, (k0 + BWD_COLS - 1) / BWD_COLS);
    hipLaunchKernelGGL(k_bwd, dim3(groups), dim3(256), 0, s, B, N, (int)k0, kb,
                       (const double *)(Lst + b * CB * CB), z, y);
  }
  return hipGetLastError();
}

int64_t als_chol_diag_elems(int64_t N) { return ((N + CB - 1) / CB) * CB * CB; }

hipError_t als_qr(double *W, int rows, int cols, double *R, double *tau, hipStream_t s) {
  hipLaunchKernelGGL(k_qr_thin, dim3(1), dim3(AWG), 0, s, W, rows, cols, R, tau);
  return hipGetLastError();
}

hipError_t als_gemm(const double *A, int lda, const double *B, int ldb, bool tb, double *C, int ldc,
                    int M, int N, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_gemm_small, dim3(blocks_for((int64_t)M * N)), dim3(256), 0, s, A, lda, B,
                     ldb, tb ? 1 : 0, C, ldc, M, N, K);
  return hipGetLastError();
}

hipError_t als_fill(double *x, int64_t n, uint64_t seed, double scale, hipStream_t s) {
  hipLaunchKernelGGL(k_hash_fill, dim3(blocks_for(n)), dim3(256), 0, s, x, n, seed, scale);
  return hipGetLastError();
}

hipError_t als_vdot(const double *a, const double *b, int64_t n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_vdot, dim3(1), dim3(AWG), 0, s, a, b, n, out);
  return hipGetLastError();
}

hipError_t als_transpose(const double *src, int rows, int cols, double *dst, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose, dim3(blocks_for((int64_t)rows * cols)), dim3(256), 0, s, src,
                     rows, cols, dst);
  return hipGetLastError();
}

hipError_t als_fill_value(double *x, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_value, dim3(blocks_for(n)), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}

hipError_t als_pad_core(const double *src, int r0s, int n, int r1s, double *dst, int r0d, int r1d,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_pad_core, dim3(blocks_for((int64_t)r0d * n * r1d)), dim3(256), 0, s, src,
                     r0s, n, r1s, dst, r0d, r1d);
  return hipGetLastError();
}

}  // namespace qtt
