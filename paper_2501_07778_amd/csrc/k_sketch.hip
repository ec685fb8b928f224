// k_sketch.hip — randomised rounding of a tensor train whose ranks are far
// above the target (the product K p inside the solve), gfx950.
//
// Randomize-then-orthogonalize (Al Daas, Ballard, Cazeaux, Hallman,
// Miedlar, Pasha, Reid, Saibaba, "Randomized algorithms for rounding in the
// tensor-train format", SIAM J. Sci. Comput. 2023):
//   1. a Gaussian TT Omega with ranks l (target + oversampling);
//   2. right-to-left partial contractions W_k = Y_{>=k} Omega_{>=k}^T,
//      W_k = Y_k^{(L)} T_k with T_k[(i, b), l] = sum_l' W_{k+1}[b, l'] Omega_k[l, i, l'];
//   3. left-to-right: S = Z_k W_{k+1}, S = Q R, core k = Q,
//      Z_{k+1} = (Q^T Z_k) Y_{k+1};  the last core is Z_{D-1}.
// The result has ranks <= l and approximates y with error close to the best
// rank-l approximation; the exact rounding then truncates it to the
// requested accuracy.  The work is small GEMMs and (l n) x l QRs instead of
// QRs of the full (R r n) x (R r) unfoldings.
//
// Gaussian numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC 2011) on the counter (element,
// core, call), keyed by the seed, then the Box-Muller transform.
#include <algorithm>
#include <cstdlib>

#include "dev_gemm.h"
#include "dev_qr.h"
#include "dev_reduce.h"
#include "internal.h"

namespace qtt {

namespace {

constexpr int WG = 1024;
constexpr int NWAVE = WG / 64;
constexpr int LDS_DBL = 19200;
constexpr int LDS_TAU = 160;

__device__ __forceinline__ void mulhilo(uint32_t a, uint32_t b, uint32_t &hi, uint32_t &lo) {
  const uint64_t p = (uint64_t)a * (uint64_t)b;
  hi = (uint32_t)(p >> 32);
  lo = (uint32_t)p;
}

__device__ uint4 philox4x32_10(uint4 c, uint2 k) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t h0, l0, h1, l1;
    mulhilo(M0, c.x, h0, l0);
    mulhilo(M1, c.z, h1, l1);
    c = make_uint4(h1 ^ c.y ^ k.x, l1, h0 ^ c.w ^ k.y, l0);
    k.x += W0;
    k.y += W1;
  }
  return c;
}

__device__ __forceinline__ double gauss(uint32_t e, uint32_t core, uint64_t call, uint64_t seed) {
  const uint4 r = philox4x32_10(make_uint4(e, core, (uint32_t)call, (uint32_t)(call >> 32)),
                                make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
  const double u1 = ((double)r.x + 0.5) * (1.0 / 4294967296.0);
  const double u2 = ((double)r.y + 0.5) * (1.0 / 4294967296.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Omega core k: l_k x n_k x l_{k+1} (host-known ranks in om.cap)
__global__ void k_gauss_tt(TTView om, uint64_t seed, uint64_t call) {
  const int k = blockIdx.y;
  const int64_t ne = (int64_t)om.cap[k] * om.n[k] * om.m[k] * om.cap[k + 1];
  double *c = om.data + om.off[k];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x)
    c[e] = gauss((uint32_t)e, (uint32_t)k, call, seed);
}

// true when the ranks around core k exceed the slots the buffers are sized for
__device__ __forceinline__ bool beyond_caps(const TTView &y, int k) {
  for (int j = k; j <= k + 2 && j <= y.D; ++j)
    if (y.rk[j] > y.cap[j]) return true;
  return false;
}

// T_k[(i + n b) + (n a1) l] = sum_l' W_{k+1}[b + a1 l'] Omega_k[l + lk (i + n l')]
__global__ void k_sketch_T(TTView y, TTView om, int k, const double *Wn, double *Tk) {
  if (beyond_caps(y, k)) return;
  const int nm = y.n[k] * y.m[k];
  const int a1 = y.rk[k + 1];
  const int lk = om.cap[k], l1 = om.cap[k + 1];
  const int64_t ne = (int64_t)nm * a1 * lk;
  const double *o = om.data + om.off[k];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % ((int64_t)nm * a1));
    const int l = (int)(e / ((int64_t)nm * a1));
    const int i = row % nm, b = row / nm;
    // operands of eight terms loaded before they are summed (same order),
    // so eight loads are in flight instead of one
    double acc = 0.0;
    int lp = 0;
    for (; lp + 8 <= l1; lp += 8) {
      double wv[8], ov[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        wv[u] = Wn[b + (int64_t)a1 * (lp + u)];
        ov[u] = o[l + (int64_t)lk * (i + (int64_t)nm * (lp + u))];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = fma(wv[u], ov[u], acc);
    }
    for (; lp < l1; ++lp)
      acc = fma(Wn[b + (int64_t)a1 * lp], o[l + (int64_t)lk * (i + (int64_t)nm * lp)], acc);
    Tk[e] = acc;
  }
}

using TN80 = dev::TileN80;  // 64 x 80 tiles: outputs with an l-wide column range
using TM80 = dev::TileM80;  // 80 x 64 tiles: outputs with an l-wide row range

constexpr int KC = 256;   // K range per block of the split-K products
constexpr int KC_S = 64;  // the same for S, whose output is only a few tiles

// Block (0,0,0) of a split-K product publishes the element count of its
// output and the number of K ranges that hold data; the reduction that
// follows on the stream reads them (the sizes live in device memory).
__device__ __forceinline__ void publish_dims(int64_t *dims, int M, int N, int K, int kcmin) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) {
    const int nz = (int)gridDim.z;
    int kc = (K + nz - 1) / nz;
    kc = kc > kcmin ? kc : kcmin;
    const int used = K > 0 ? (K + kc - 1) / kc : 0;
    dims[0] = (int64_t)M * N;
    dims[1] = used < nz ? used : nz;
  }
}

// W_k (a_k x l_k) = Y_k (a_k x nm a_{k+1}) T_k, split over K
__global__ void __launch_bounds__(256) k_sketch_W(TTView y, TTView om, int k, const double *Tk,
                                                  double *Pw, int64_t *dims) {
  const bool bad = beyond_caps(y, k);
  const int M = bad ? 0 : y.rk[k], K = y.n[k] * y.m[k] * y.rk[k + 1], N = om.cap[k];
  publish_dims(dims, M, N, K, KC);
  if (bad || blockIdx.x * TN80::TM >= M || blockIdx.y * TN80::TN >= N) return;
  dev::gemm_tile_k_w<false, TN80>(y.data + y.off[k], M, Tk, K, Pw, M, N, K, blockIdx.x,
                                  blockIdx.y, blockIdx.z, KC);
}

// S ((lz nm) x l_{k+1}) = Z (lz nm x a_{k+1}) W_{k+1}, split over K
__global__ void __launch_bounds__(256) k_sketch_S(TTView y, TTView om, int k, int lz,
                                                  const double *Z, const double *Wn, double *Ps,
                                                  int64_t *dims) {
  const bool bad = beyond_caps(y, k);
  const int M = bad ? 0 : lz * y.n[k] * y.m[k], K = y.rk[k + 1], N = om.cap[k + 1];
  publish_dims(dims, M, N, K, KC_S);
  if (bad || blockIdx.x * TN80::TM >= M || blockIdx.y * TN80::TN >= N) return;
  dev::gemm_tile_k_w<false, TN80>(Z, M, Wn, K, Ps, M, N, K, blockIdx.x, blockIdx.y, blockIdx.z,
                                  KC_S);
}

// Mq (rq x a_{k+1}) = Q^T (rq x lz nm) Z (lz nm x a_{k+1})
__global__ void __launch_bounds__(256) k_sketch_M(TTView y, int k, int lz, int rq,
                                                  const double *Q, const double *Z, double *Mq) {
  if (beyond_caps(y, k)) return;
  const int M = rq, K = lz * y.n[k] * y.m[k], N = y.rk[k + 1];
  if (blockIdx.x * TM80::TM >= M || blockIdx.y * TM80::TN >= N) return;
  dev::gemm_tile_mfma_w<true, TM80::WM, TM80::WN, TM80::BM, TM80::BN>(Q, K, Z, K, Mq, M, M, N, K,
                                                                      blockIdx.x, blockIdx.y);
}

// Z' (rq x nm_{k+1} a_{k+2}) = Mq (rq x a_{k+1}) Y_{k+1}, split over K
__global__ void __launch_bounds__(256) k_sketch_Z(TTView y, int k, int rq, const double *Mq,
                                                  double *Pz, int64_t *dims) {
  const bool bad = beyond_caps(y, k);
  const int M = bad ? 0 : rq, K = y.rk[k + 1], N = y.n[k + 1] * y.m[k + 1] * y.rk[k + 2];
  publish_dims(dims, M, N, K, KC);
  if (bad || blockIdx.x * TM80::TM >= M || blockIdx.y * TM80::TN >= N) return;
  dev::gemm_tile_k_w<false, TM80>(Mq, M, y.data + y.off[k + 1], K, Pz, M, N, K, blockIdx.x,
                                  blockIdx.y, blockIdx.z, KC);
}

// C = sum of the partials of the product launched just before (sizes from
// `dims`, written by that product)
__global__ void k_splitk_reduce(const int64_t *dims, const double *P, double *C) {
  const int64_t ne = dims[0];
  const int used = (int)dims[1];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    // partials loaded eight at a time, summed in order
    double acc = 0.0;
    int z = 0;
    for (; z + 8 <= used; z += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = P[(int64_t)(z + u) * ne + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; z < used; ++z) acc += P[(int64_t)z * ne + e];
    C[e] = acc;
  }
}

// Householder QR of the (rows x cols) sketch S; Q (rows x rq) is formed in
// place of the reflectors and written to `Qout` (ld = rows).  The LDS
// variant needs rows*cols <= LDS_DBL; the other one works in `gw` (rows
// cols doubles of global memory, then the reflector factors).
template <bool LDS>
__global__ void __launch_bounds__(WG) k_sketch_qr(const double *S, int rows, int cols,
                                                  double *Qout, double *gw) {
  __shared__ double lds[LDS ? LDS_DBL : 1];
  __shared__ double tau_l[LDS_TAU];
  const int kmax = rows < cols ? rows : cols;
  double *W = LDS ? lds : gw;
  double *tau = LDS ? tau_l : gw + 2 * rows * cols;
  for (int e = threadIdx.x; e < rows * cols; e += WG) W[e] = S[e];
  __syncthreads();
  dev::householder_qr<NWAVE>(W, rows, cols, tau);
  dev::form_q_inplace<NWAVE>(W, rows, kmax, tau);
  for (int e = threadIdx.x; e < rows * kmax; e += WG) Qout[e] = W[e];
}

__global__ void k_copy(const double *src, double *dst, const int *r1, int mul, int r1cap) {
  if (r1 && *r1 > r1cap) return;
  const int64_t ne = (int64_t)mul * (r1 ? *r1 : 1);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

__global__ void k_fill_one(double *p) { *p = 1.0; }

struct RankArgS {
  int D;
  int r[QTT_MAXD + 1];
};
__global__ void k_set_ranks_s(int *rk, RankArgS a) {
  if ((int)threadIdx.x <= a.D) rk[threadIdx.x] = a.r[threadIdx.x];
}

struct SketchDims {
  std::vector<int> l;    // ranks of Omega
  std::vector<int> lz;   // ranks of the result
};

SketchDims sketch_dims(const TTView &y, int ell) {
  SketchDims d;
  const int D = y.D;
  d.l.assign(D + 1, 1);
  double left = 1.0;
  for (int k = 1; k < D; ++k) {
    left *= (double)y.n[k - 1] * y.m[k - 1];
    double right = 1.0;
    for (int j = k; j < D; ++j) right *= (double)y.n[j] * y.m[j];
    double b = left < right ? left : right;
    b = b < y.cap[k] ? b : y.cap[k];
    d.l[k] = (int)(b < ell ? b : ell);
    if (d.l[k] < 1) d.l[k] = 1;
  }
  d.lz.assign(D + 1, 1);
  for (int k = 0; k < D - 1; ++k) {
    const int rows = d.lz[k] * y.n[k] * y.m[k];
    d.lz[k + 1] = rows < d.l[k + 1] ? rows : d.l[k + 1];
  }
  return d;
}

// split count for a product with K of at most kcap
int split_of(int64_t kcap, int kc = KC) {
  const int64_t s = (kcap + kc - 1) / kc;
  return (int)std::max<int64_t>(1, std::min<int64_t>(s, 32));
}

int red_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048)); }

struct SketchLayout {
  TTView om;
  std::vector<double *> W;
  double *T, *Z[2], *S, *Mq, *Qw, *P;
  int64_t *dims;
  int64_t used;
};

int64_t al32(int64_t x) { return (x + 31) & ~int64_t(31); }

SketchLayout sketch_layout(const TTView &y, const SketchDims &d, double *ws) {
  SketchLayout L;
  const int D = y.D;
  L.om = y;
  int64_t off = 0;
  for (int k = 0; k < D; ++k) {
    L.om.off[k] = off;
    off = al32(off + (int64_t)d.l[k] * y.n[k] * y.m[k] * d.l[k + 1]);
  }
  for (int k = 0; k <= D; ++k) L.om.cap[k] = d.l[k];
  L.om.data = ws;
  L.om.rk = nullptr;
  L.W.assign(D + 1, nullptr);
  for (int k = 1; k <= D; ++k) {
    L.W[k] = ws ? ws + off : nullptr;
    off = al32(off + (int64_t)y.cap[k] * d.l[k] + 1);
  }
  int64_t tmax = 1, zmax = 1, smax = 1, mqmax = 1;
  for (int k = 0; k < D; ++k) {
    tmax = std::max<int64_t>(tmax, (int64_t)y.n[k] * y.m[k] * y.cap[k + 1] * d.l[k]);
    zmax = std::max<int64_t>(zmax, (int64_t)d.lz[k] * y.n[k] * y.m[k] * y.cap[k + 1]);
    smax = std::max<int64_t>(smax, (int64_t)d.lz[k] * y.n[k] * y.m[k] * d.l[k + 1]);
    mqmax = std::max<int64_t>(mqmax, (int64_t)d.lz[k + 1] * y.cap[k + 1]);
  }
  auto take = [&](int64_t n) {
    double *p = ws ? ws + off : nullptr;
    off = al32(off + n);
    return p;
  };
  L.T = take(tmax);
  L.Z[0] = take(zmax);
  L.Z[1] = take(zmax);
  L.S = take(smax);
  L.Mq = take(mqmax);
  L.Qw = take(2 * smax + 1024);
  // split-K partials of the largest product
  int64_t pmax = 1;
  for (int k = 0; k < D; ++k) {
    pmax = std::max<int64_t>(pmax, (int64_t)split_of(y.n[k] * y.m[k] * y.cap[k + 1]) *
                                       y.cap[k] * d.l[k]);
    pmax = std::max<int64_t>(pmax, (int64_t)split_of(y.cap[k + 1], KC_S) * d.lz[k] * y.n[k] * y.m[k] *
                                       d.l[k + 1]);
    if (k + 1 < D)
      pmax = std::max<int64_t>(pmax, (int64_t)split_of(y.cap[k + 1]) * d.lz[k + 1] *
                                         y.n[k + 1] * y.m[k + 1] * y.cap[k + 2]);
  }
  L.P = take(pmax);
  L.dims = (int64_t *)take(4);
  L.used = off;
  return L;
}

}  // namespace

int64_t sketch_ws_elems(const TTView &y, int ell) {
  SketchDims d = sketch_dims(y, ell);
  return sketch_layout(y, d, nullptr).used + 64;
}

hipError_t sketch_tt(const TTView &y, int ell, uint64_t seed, uint64_t call, double *ws,
                     hipStream_t s) {
  const int D = y.D;
  if (D < 2) return hipSuccess;
  SketchDims d = sketch_dims(y, ell);
  SketchLayout L = sketch_layout(y, d, ws);
  // 1. Omega
  {
    int64_t mx = 1;
    for (int k = 0; k < D; ++k)
      mx = std::max<int64_t>(mx, (int64_t)d.l[k] * y.n[k] * y.m[k] * d.l[k + 1]);
    int blocks = (int)std::min<int64_t>((mx + 255) / 256, 1024);
    hipLaunchKernelGGL(k_gauss_tt, dim3(blocks, D), dim3(256), 0, s, L.om, seed, call);
  }
  // 2. right-to-left partial contractions, W_D = 1
  hipLaunchKernelGGL(k_fill_one, dim3(1), dim3(1), 0, s, L.W[D]);
  for (int k = D - 1; k >= 1; --k) {
    const int64_t tn = (int64_t)y.n[k] * y.m[k] * y.cap[k + 1] * d.l[k];
    int blocks = (int)std::min<int64_t>((tn + 255) / 256, 4096);
    hipLaunchKernelGGL(k_sketch_T, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, y, L.om, k,
                       L.W[k + 1], L.T);
    const int mt = (y.cap[k] + TN80::TM - 1) / TN80::TM, nt = (d.l[k] + TN80::TN - 1) / TN80::TN;
    const int ns = split_of(y.n[k] * y.m[k] * y.cap[k + 1]);
    hipLaunchKernelGGL(k_sketch_W, dim3(mt, nt, ns), dim3(256), 0, s, y, L.om, k, L.T, L.P,
                       L.dims);
    hipLaunchKernelGGL(k_splitk_reduce, dim3(red_blocks((int64_t)y.cap[k] * d.l[k])), dim3(256), 0,
                       s, L.dims, L.P, L.W[k]);
  }
  // 3. left-to-right
  {
    const int64_t ne = (int64_t)y.n[0] * y.m[0] * y.cap[1];
    int blocks = (int)std::min<int64_t>((ne + 255) / 256, 1024);
    hipLaunchKernelGGL(k_copy, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s,
                       y.data + y.off[0], L.Z[0], y.rk + 1, y.n[0] * y.m[0], y.cap[1]);
  }
  int cur = 0;
  for (int k = 0; k < D - 1; ++k) {
    const int lz = d.lz[k], rq = d.lz[k + 1];
    const int rows = lz * y.n[k] * y.m[k], cols = d.l[k + 1];
    {
      const int mt = (rows + TN80::TM - 1) / TN80::TM, nt = (cols + TN80::TN - 1) / TN80::TN;
      const int ns = split_of(y.cap[k + 1], KC_S);
      hipLaunchKernelGGL(k_sketch_S, dim3(mt, nt, ns), dim3(256), 0, s, y, L.om, k, lz, L.Z[cur],
                         L.W[k + 1], L.P, L.dims);
      hipLaunchKernelGGL(k_splitk_reduce, dim3(red_blocks((int64_t)rows * cols)), dim3(256), 0, s,
                         L.dims, L.P, L.S);
    }
    double *Q = y.data + y.off[k];
    const int th = ktimer_begin(KT_SKETCH_QR, s);
    if ((int64_t)rows * cols <= LDS_DBL && rq <= LDS_TAU)
      hipLaunchKernelGGL(k_sketch_qr<true>, dim3(1), dim3(WG), 0, s, L.S, rows, cols, Q, L.Qw);
    else
      hipLaunchKernelGGL(k_sketch_qr<false>, dim3(1), dim3(WG), 0, s, L.S, rows, cols, Q, L.Qw);
    ktimer_end(th, s);
    {
      const int mt = (rq + TM80::TM - 1) / TM80::TM, nt = (y.cap[k + 1] + TM80::TN - 1) / TM80::TN;
      hipLaunchKernelGGL(k_sketch_M, dim3(mt, nt), dim3(256), 0, s, y, k, lz, rq, Q, L.Z[cur],
                         L.Mq);
    }
    {
      const int mt = (rq + TM80::TM - 1) / TM80::TM;
      const int nt = (y.n[k + 1] * y.m[k + 1] * y.cap[k + 2] + TM80::TN - 1) / TM80::TN;
      const int ns = split_of(y.cap[k + 1]);
      hipLaunchKernelGGL(k_sketch_Z, dim3(mt, nt, ns), dim3(256), 0, s, y, k, rq, L.Mq, L.P,
                         L.dims);
      hipLaunchKernelGGL(k_splitk_reduce,
                         dim3(red_blocks((int64_t)rq * y.n[k + 1] * y.m[k + 1] * y.cap[k + 2])),
                         dim3(256), 0, s, L.dims, L.P, L.Z[1 - cur]);
    }
    cur = 1 - cur;
  }
  {
    const int64_t ne = (int64_t)d.lz[D - 1] * y.n[D - 1] * y.m[D - 1];
    int blocks = (int)std::min<int64_t>((ne + 255) / 256, 1024);
    hipLaunchKernelGGL(k_copy, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, L.Z[cur],
                       y.data + y.off[D - 1], nullptr, (int)ne, 1);
  }
  RankArgS a;
  a.D = D;
  for (int k = 0; k <= D; ++k) a.r[k] = d.lz[k];
  hipLaunchKernelGGL(k_set_ranks_s, dim3(1), dim3(64), 0, s, y.rk, a);
  return hipGetLastError();
}

}  // namespace qtt
