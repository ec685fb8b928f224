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
#include "internal.h"

namespace qtt {

namespace {

constexpr int WG = 1024;           // threads of the one-workgroup kernels
constexpr int NWAVE = WG / 64;
constexpr int JACOBI_MAX_SWEEPS = 40;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

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

// Householder QR of a column-major rows x cols matrix W (ld = rows) in
// place: R above the diagonal, reflectors below, tau[j].  LAPACK-style
// reflectors H = I - tau v v^T with v(0) = 1.
__device__ void householder_qr(double *W, int rows, int cols, double *tau,
                               double *red) {
  const int kmax = rows < cols ? rows : cols;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < kmax; ++j) {
    double *wj = W + (int64_t)rows * j;
    double p = 0.0;
    for (int i = j + 1 + threadIdx.x; i < rows; i += WG) p += wj[i] * wj[i];
    const double xnorm2 = block_sum(p, red);
    const double alpha = wj[j];
    double t = 0.0, beta = alpha, scale = 0.0;
    if (xnorm2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();
    if (t != 0.0) {
      for (int i = j + 1 + threadIdx.x; i < rows; i += WG) wj[i] *= scale;
    }
    if (threadIdx.x == 0) {
      wj[j] = beta;
      tau[j] = t;
    }
    __syncthreads();
    if (t != 0.0) {
      for (int c = j + 1 + wave; c < cols; c += NWAVE) {
        double *wc = W + (int64_t)rows * c;
        double s = (lane == 0) ? wc[j] : 0.0;
        for (int i = j + 1 + lane; i < rows; i += 64) s += wj[i] * wc[i];
        s = wave_sum(s) * t;
        if (lane == 0) wc[j] -= s;
        for (int i = j + 1 + lane; i < rows; i += 64) wc[i] -= s * wj[i];
      }
    }
    __syncthreads();
  }
}

// Q (rows x kq, ld = rows) = H_0 ... H_{kq-1} [I; 0] from the reflectors in W.
__device__ void form_q(const double *W, int rows, int kq, const double *tau,
                       double *Q) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t e = threadIdx.x; e < (int64_t)rows * kq; e += WG) {
    const int i = (int)(e % rows), c = (int)(e / rows);
    Q[e] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = kq - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t != 0.0) {
      const double *wj = W + (int64_t)rows * j;
      for (int c = j + wave; c < kq; c += NWAVE) {
        double *qc = Q + (int64_t)rows * c;
        double s = (lane == 0) ? qc[j] : 0.0;
        for (int i = j + 1 + lane; i < rows; i += 64) s += wj[i] * qc[i];
        s = wave_sum(s) * t;
        if (lane == 0) qc[j] -= s;
        for (int i = j + 1 + lane; i < rows; i += 64) qc[i] -= s * wj[i];
      }
    }
    __syncthreads();
  }
}

// Left sweep, core k: QR of the left unfolding (rows = nr[k]*nm_k,
// cols = rk[k+1]); Q -> slot k, R -> rbuf (ld = r'), nr[k+1] = r'.
__global__ void __launch_bounds__(WG)
    k_qr_step(TTView x, int k, const double *src, double *work, double *rbuf,
              double *tau, int *iwork) {
  __shared__ double red[NWAVE];
  IW w = iw_of(iwork, x.D);
  const int nm = x.n[k] * x.m[k];
  const int rows = w.nr[k] * nm;
  const int cols = x.rk[k + 1];
  const int rq = rows < cols ? rows : cols;
  for (int64_t e = threadIdx.x; e < (int64_t)rows * cols; e += WG) work[e] = src[e];
  __syncthreads();
  householder_qr(work, rows, cols, tau, red);
  // R: rq x cols, upper trapezoid
  for (int64_t e = threadIdx.x; e < (int64_t)rq * cols; e += WG) {
    const int i = (int)(e % rq), c = (int)(e / rq);
    rbuf[e] = (i <= c) ? work[i + (int64_t)rows * c] : 0.0;
  }
  form_q(work, rows, rq, tau, x.data + x.off[k]);
  if (threadIdx.x == 0) w.nr[k + 1] = rq;
}

// Column-major GEMM C = A * B, 64x64 tiles, K step 16, FP64.
constexpr int GT = 64, GK = 16;
__device__ void gemm_tile(const double *A, int lda, const double *B, int ldb,
                          double *C, int ldc, int M, int N, int K, int tm,
                          int tn) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tid = threadIdx.x;  // 256 threads
  const int tr = tid % 16, tc = tid / 16;
  double acc[4][4] = {};
  const int m0 = tm * GT, n0 = tn * GT;
  for (int k0 = 0; k0 < K; k0 += GK) {
    for (int e = tid; e < GK * GT; e += 256) {
      const int mm = e % GT, kk = e / GT;
      const int gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < M && gk < K) ? A[gm + (int64_t)lda * gk] : 0.0;
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

// absorb: carry (nr[k+1] x nm_{k+1} rk[k+2]) = R (nr[k+1] x rk[k+1]) *
// slot k+1 (rk[k+1] x nm_{k+1} rk[k+2])
__global__ void __launch_bounds__(256)
    k_absorb(TTView x, int k, const double *rbuf, double *carry, int *iwork) {
  IW w = iw_of(iwork, x.D);
  const int M = w.nr[k + 1];
  const int K = x.rk[k + 1];
  const int N = x.n[k + 1] * x.m[k + 1] * x.rk[k + 2];
  if (blockIdx.x * GT >= M || blockIdx.y * GT >= N) return;
  gemm_tile(rbuf, M, x.data + x.off[k + 1], K, carry, M, M, N, K, blockIdx.x,
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
  if (blockIdx.x * GT >= M || blockIdx.y * GT >= N) return;
  gemm_tile(x.data + x.off[k - 1], M, F, K, carry, M, M, N, K, blockIdx.x,
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

// One-sided Jacobi (Hestenes) on the columns of B (mb x nb, ld = mb) with V
// (nb x nb) accumulated: B V has mutually orthogonal columns.  Round-robin
// ordering: each round pairs all columns disjointly, one wave per pair.
__device__ void jacobi(double *B, int mb, int nb, double *V, int *flag) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t e = threadIdx.x; e < (int64_t)nb * nb; e += WG)
    V[e] = ((e % nb) == (e / nb)) ? 1.0 : 0.0;
  const int N = nb + (nb & 1);
  const double tol = 1e-15 * sqrt((double)mb);
  for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
    __syncthreads();
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      for (int i = wave; i < N / 2; i += NWAVE) {
        int p = (r + i) % (N - 1);
        int q = (i == 0) ? (N - 1) : (r - i + N - 1) % (N - 1);
        if (p >= nb || q >= nb) continue;
        if (p > q) { int t = p; p = q; q = t; }
        double *bp = B + (int64_t)mb * p, *bq = B + (int64_t)mb * q;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int l = lane; l < mb; l += 64) {
          const double u = bp[l], v = bq[l];
          al = fma(u, u, al);
          be = fma(v, v, be);
          ga = fma(u, v, ga);
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (ga == 0.0 || !(fabs(ga) > tol * sqrt(al * be))) continue;
        const double zeta = (be - al) / (2.0 * ga);
        double t;
        if (fabs(zeta) > 1e150)
          t = 0.5 / zeta;
        else
          t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int l = lane; l < mb; l += 64) {
          const double u = bp[l], v = bq[l];
          bp[l] = c * u - s * v;
          bq[l] = s * u + c * v;
        }
        double *vp = V + (int64_t)nb * p, *vq = V + (int64_t)nb * q;
        for (int l = lane; l < nb; l += 64) {
          const double u = vp[l], v = vq[l];
          vp[l] = c * u - s * v;
          vq[l] = s * u + c * v;
        }
        if (lane == 0) *flag = 1;
      }
      __syncthreads();
    }
    __syncthreads();
    if (*flag == 0) break;
  }
  __syncthreads();
}

// Right sweep, core k: SVD of the right unfolding M (r0 = nr[k] rows,
// nc = nm_k * fr[k+1] columns) held in `carry`; writes V^T-type factor to
// slot k, the fold operand F (r0 x rank) and fr[k] = rank.
__global__ void __launch_bounds__(WG)
    k_svd_step(TTView x, int k, double eps, int rmax, const double *carry,
               double *work, double *vbuf, double *F, double *sig,
               int *iwork, double *scal) {
  __shared__ double red[NWAVE];
  __shared__ int flag;
  __shared__ int rank_s;
  IW w = iw_of(iwork, x.D);
  const int D = x.D;
  const int nm = x.n[k] * x.m[k];
  const int r0 = w.nr[k];
  const int nc = nm * w.fr[k + 1];
  const bool tall = r0 >= nc;
  const int mb = tall ? r0 : nc, nb = tall ? nc : r0;
  // B = M (tall) or M^T (wide), column-major mb x nb
  for (int64_t e = threadIdx.x; e < (int64_t)mb * nb; e += WG) {
    const int i = (int)(e % mb), j = (int)(e / mb);
    work[e] = tall ? carry[e] : carry[j + (int64_t)r0 * i];
  }
  __syncthreads();
  jacobi(work, mb, nb, vbuf, &flag);
  // column norms
  for (int j = threadIdx.x >> 6; j < nb; j += NWAVE) {
    const double *bj = work + (int64_t)mb * j;
    double s = 0.0;
    for (int l = threadIdx.x & 63; l < mb; l += 64) s = fma(bj[l], bj[l], s);
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sig[j] = sqrt(s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // descending order by selection (nb is at most a few hundred)
    for (int j = 0; j < nb; ++j) w.perm[j] = j;
    for (int a = 0; a < nb; ++a) {
      int best = a;
      for (int b = a + 1; b < nb; ++b)
        if (sig[w.perm[b]] > sig[w.perm[best]]) best = b;
      int t = w.perm[a]; w.perm[a] = w.perm[best]; w.perm[best] = t;
    }
    const double delta = (D > 1) ? eps * scal[0] / sqrt((double)(D - 1)) : 0.0;
    // smallest rank with tail <= delta
    double tail2 = 0.0;
    int rank = nb;
    for (int j = nb - 1; j >= 0; --j) {
      const double sj = sig[w.perm[j]];
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
    for (int j = rank; j < nb; ++j) disc += sig[w.perm[j]] * sig[w.perm[j]];
    scal[1] += disc;
    w.fr[k] = rank;
    rank_s = rank;
  }
  __syncthreads();
  const int rank = rank_s;
  double *core = x.data + x.off[k];  // rank x nc
  if (tall) {
    // M V = W: F = W[:, perm[:rank]] (r0 x rank), core = V[:, perm]^T
    for (int64_t e = threadIdx.x; e < (int64_t)r0 * rank; e += WG) {
      const int a = (int)(e % r0), l = (int)(e / r0);
      F[e] = work[a + (int64_t)mb * w.perm[l]];
    }
    for (int64_t e = threadIdx.x; e < (int64_t)rank * nc; e += WG) {
      const int l = (int)(e % rank), col = (int)(e / rank);
      core[e] = vbuf[col + (int64_t)nb * w.perm[l]];
    }
  } else {
    // M^T V = W: M = V W^T; F = V[:, perm] * sigma, core = (W / sigma)^T
    for (int64_t e = threadIdx.x; e < (int64_t)r0 * rank; e += WG) {
      const int a = (int)(e % r0), l = (int)(e / r0);
      F[e] = vbuf[a + (int64_t)nb * w.perm[l]] * sig[w.perm[l]];
    }
    for (int64_t e = threadIdx.x; e < (int64_t)rank * nc; e += WG) {
      const int l = (int)(e % rank), col = (int)(e / rank);
      const double s = sig[w.perm[l]];
      core[e] = (s > 0.0) ? work[col + (int64_t)mb * w.perm[l]] / s
                          : ((col == l) ? 1.0 : 0.0);
    }
  }
}

// slot 0 <- carry (1 x nm_0 x fr[1]), ranks <- fr
__global__ void k_round_finish(TTView x, const double *carry, int *iwork) {
  IW w = iw_of(iwork, x.D);
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
  // SVD matrices are at most cap x (nm cap); V at most (nm cap)^2
  const int64_t sq = (nm * cap) * (nm * cap);
  w.carry_elems = slot;
  w.sq_elems = sq;
  w.carry = (double *)ar.take(sizeof(double) * slot);
  w.work = (double *)ar.take(sizeof(double) * (slot > sq ? slot : sq));
  w.rbuf = (double *)ar.take(sizeof(double) * cap * cap);
  w.vbuf = (double *)ar.take(sizeof(double) * cap * cap);
  w.fold = (double *)ar.take(sizeof(double) * cap * cap * nm);
  w.scal = (double *)ar.take(sizeof(double) * (4 + 2 * nm * cap));
  w.iwork = (int *)ar.take(sizeof(int) * (2 * (x.D + 1) + nm * cap + 8));
  return ar.ok();
}

hipError_t round_tt(const TTView &x, double eps, int rmax, const RoundWs &w,
                    hipStream_t s) {
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
  for (int k = 0; k < D - 1; ++k) {
    const double *src = (k == 0) ? x.data + x.off[0] : w.carry;
    hipLaunchKernelGGL(k_qr_step, dim3(1), dim3(WG), 0, s, x, k, src, w.work,
                       w.rbuf, tau, w.iwork);
    const int mt = (x.cap[k + 1] + GT - 1) / GT;
    const int nt = (x.n[k + 1] * x.m[k + 1] * x.cap[k + 2] + GT - 1) / GT;
    hipLaunchKernelGGL(k_absorb, dim3(mt, nt), dim3(256), 0, s, x, k, w.rbuf,
                       w.carry, w.iwork);
  }
  hipLaunchKernelGGL(k_last_norm, dim3(1), dim3(WG), 0, s, x, w.carry, w.iwork,
                     w.scal);
  for (int k = D - 1; k >= 1; --k) {
    hipLaunchKernelGGL(k_svd_step, dim3(1), dim3(WG), 0, s, x, k, eps, rmax,
                       w.carry, w.work, w.vbuf, w.fold, sig, w.iwork, w.scal);
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
