// k_tt.hip — QTT matrix-vector product and the tensor-train glue used by
// the solver (sums, inner products, packing), gfx950.
//
// The matrix-vector product is the strong Kronecker product of cores
// (Sec. 4): y_k[(a,b), i, (c,d)] = sum_j A_k[a,i,j,c] x_k[b,j,d].  It reads
// two small operand cores and writes an output core that is R*r times larger
// in each rank, so it is bound by HBM writes: the kernel streams the output
// once, fully coalesced along the fastest index b (the rank of x), with the
// operand slices of each output column staged in LDS.
#include <hip/hip_bf16.h>

#include <algorithm>

#include "dev_gemm.h"
#include "internal.h"

namespace qtt {

namespace {

constexpr int MV_TX = 64;   // lanes along b (output rows of one column)
constexpr int MV_TY = 4;    // waves along a
constexpr int MV_MMAX = 8;  // column modes held in registers (wider ones read directly)

template <typename T>
__device__ __forceinline__ float to_compute(double v);
template <>
__device__ __forceinline__ float to_compute<float>(double v) {
  return static_cast<float>(v);
}
template <>
__device__ __forceinline__ float to_compute<__hip_bfloat16>(double v) {
  return __bfloat162float(__float2bfloat16(static_cast<float>(v)));
}

// Blocks loop over the output columns (i, c, d) of core blockIdx.y; the
// P = ra0*rx0 rows of a column are contiguous in memory.  The operand slices
// of a column, A[:, i, :, c] (ra0 x m) and x[:, :, d] (rx0 x m), are staged
// in LDS once, so the output loop reads no global memory and issues one
// 16-byte non-temporal store per lane for two consecutive rows.
// T = double: FP64 throughout; T = float or __hip_bfloat16: operands rounded
// to T when staged, products accumulated in FP32, output written in FP64.
constexpr int MV_SLICE = 2048;  // entries per staged operand slice
template <typename T> struct MvStage { typedef float type; };
template <> struct MvStage<double> { typedef double type; };
template <typename T>
__device__ __forceinline__ typename MvStage<T>::type mv_stage(double v) {
  return to_compute<T>(v);
}
template <>
__device__ __forceinline__ double mv_stage<double>(double v) {
  return v;
}
__device__ __forceinline__ double mv_fma(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float mv_fma(float a, float b, float c) { return fmaf(a, b, c); }

template <typename T>
__device__ __forceinline__ void matvec_staged(const TTView &A, const TTView &x, const TTView &y,
                                              typename MvStage<T>::type *As,
                                              typename MvStage<T>::type *Xs) {
  typedef typename MvStage<T>::type S;
  const int k = blockIdx.y;
  const int ra0 = A.rk[k], ra1 = A.rk[k + 1];
  const int rx0 = x.rk[k], rx1 = x.rk[k + 1];
  if (blockIdx.x == 0 && k == 0 && threadIdx.x <= A.D)
    y.rk[threadIdx.x] = A.rk[threadIdx.x] * x.rk[threadIdx.x];
  const int n = A.n[k], m = A.m[k];
  const int P = ra0 * rx0;
  const int ncols = n * ra1 * rx1;
  // never write past the output slot (its caps bound the product ranks);
  // the host picks this kernel only when the slices fit the LDS arrays
  if (P > y.cap[k] || ra1 * rx1 > y.cap[k + 1]) return;
  if (ra0 * m > MV_SLICE || rx0 * m > MV_SLICE) return;
  const double *Ak = A.data + A.off[k];
  const double *xk = x.data + x.off[k];
  double *yk = y.data + y.off[k];
  const int t = threadIdx.x;
  // output pair e2 = t + 256 s covers rows e = 2 e2, 2 e2 + 1 (a = e / rx0,
  // b = e % rx0); the step of 512 rows is q whole rows plus r
  const int q = 512 / rx0, r = 512 % rx0;
  for (int col = blockIdx.x; col < ncols; col += gridDim.x) {
    const int i = col % n;
    const int s = col / n;
    const int c = s / rx1;
    const int d = s - c * rx1;
    __syncthreads();
    for (int e = t; e < ra0 * m; e += 256) {
      const int a = e % ra0, j = e / ra0;
      As[e] = mv_stage<T>(Ak[a + (int64_t)ra0 * (i + (int64_t)n * (j + (int64_t)m * c))]);
    }
    for (int e = t; e < rx0 * m; e += 256) {
      const int b = e % rx0, j = e / rx0;
      Xs[e] = mv_stage<T>(xk[b + (int64_t)rx0 * (j + (int64_t)m * d)]);
    }
    __syncthreads();
    double *ycol = yk + (int64_t)P * col;
    if ((P & 1) == 0 && (((uintptr_t)ycol) & 15) == 0) {
      int a0 = (2 * t) / rx0, b0 = 2 * t - a0 * rx0;
      for (int e2 = t; e2 < P / 2; e2 += 256) {
        int a1 = a0, b1 = b0 + 1;
        if (b1 == rx0) {
          b1 = 0;
          ++a1;
        }
        S v0 = 0, v1 = 0;
        for (int j = 0; j < m; ++j) {
          v0 = mv_fma(As[a0 + ra0 * j], Xs[b0 + rx0 * j], v0);
          v1 = mv_fma(As[a1 + ra0 * j], Xs[b1 + rx0 * j], v1);
        }
        typedef double d2v __attribute__((ext_vector_type(2)));
        const d2v v = {static_cast<double>(v0), static_cast<double>(v1)};
        __builtin_nontemporal_store(v, reinterpret_cast<d2v *>(ycol) + e2);
        a0 += q;
        b0 += r;
        if (b0 >= rx0) {
          b0 -= rx0;
          ++a0;
        }
      }
    } else {
      for (int e = t; e < P; e += 256) {
        const int a = e / rx0, b = e - a * rx0;
        S v = 0;
        for (int j = 0; j < m; ++j) v = mv_fma(As[a + ra0 * j], Xs[b + rx0 * j], v);
        __builtin_nontemporal_store(static_cast<double>(v), ycol + e);
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_matvec_f64(TTView A, TTView x, TTView y) {
  __shared__ double As[MV_SLICE], Xs[MV_SLICE];
  matvec_staged<double>(A, x, y, As, Xs);
}

template <typename T>
__global__ void __launch_bounds__(256) k_matvec_lp_staged(TTView A, TTView x, TTView y) {
  __shared__ float As[MV_SLICE], Xs[MV_SLICE];
  matvec_staged<T>(A, x, y, As, Xs);
}

// The same product with the operand values read from global memory, for
// slices too large for the LDS arrays of k_matvec_f64.
__global__ void __launch_bounds__(MV_TX *MV_TY)
    k_matvec_f64_direct(TTView A, TTView x, TTView y) {
  const int k = blockIdx.y;
  const int ra0 = A.rk[k], ra1 = A.rk[k + 1];
  const int rx0 = x.rk[k], rx1 = x.rk[k + 1];
  if (blockIdx.x == 0 && k == 0 && threadIdx.x <= A.D)
    y.rk[threadIdx.x] = A.rk[threadIdx.x] * x.rk[threadIdx.x];
  const int n = A.n[k], m = A.m[k];
  const int P = ra0 * rx0;
  const int ncols = n * ra1 * rx1;
  // never write past the output slot (its caps bound the product ranks)
  if (P > y.cap[k] || ra1 * rx1 > y.cap[k + 1]) return;
  const double *Ak = A.data + A.off[k];
  const double *xk = x.data + x.off[k];
  double *yk = y.data + y.off[k];
  const int tx = threadIdx.x % MV_TX, ty = threadIdx.x / MV_TX;
  for (int col = blockIdx.x; col < ncols; col += gridDim.x) {
    const int i = col % n;
    const int s = col / n;
    const int c = s / rx1;
    const int d = s - c * rx1;
    double *ycol = yk + (int64_t)P * col;
    for (int b0 = 0; b0 < rx0; b0 += MV_TX) {
      const int b = b0 + tx;
      const bool act = b < rx0;
      if (m > MV_MMAX) {
        // wide column modes (a subdomain core): operands straight from memory
        for (int a = ty; a < ra0; a += MV_TY) {
          const double *Aa = Ak + a + (int64_t)ra0 * (i + (int64_t)n * m * c);
          double acc = 0.0;
          if (act)
            for (int j = 0; j < m; ++j)
              acc = fma(Aa[(int64_t)ra0 * n * j], xk[b + (int64_t)rx0 * (j + (int64_t)m * d)], acc);
          if (act) __builtin_nontemporal_store(acc, &ycol[a * rx0 + b]);
        }
        continue;
      }
      double xv[MV_MMAX];
#pragma unroll
      for (int j = 0; j < MV_MMAX; ++j)
        xv[j] = (act && j < m) ? xk[b + (int64_t)rx0 * (j + m * d)] : 0.0;
      for (int a = ty; a < ra0; a += MV_TY) {
        const double *Aa = Ak + a + (int64_t)ra0 * (i + (int64_t)n * m * c);
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < MV_MMAX; ++j)
          if (j < m) acc = fma(Aa[(int64_t)ra0 * n * j], xv[j], acc);
        // the product is streamed out once: non-temporal stores keep it
        // from evicting the operand cores from the caches
        if (act) __builtin_nontemporal_store(acc, &ycol[a * rx0 + b]);
      }
    }
  }
}

// Mixed precision: operands rounded to T, products accumulated in FP32.
template <typename T>
__global__ void __launch_bounds__(MV_TX *MV_TY)
    k_matvec_lp(TTView A, TTView x, TTView y) {
  const int k = blockIdx.y;
  const int ra0 = A.rk[k], ra1 = A.rk[k + 1];
  const int rx0 = x.rk[k], rx1 = x.rk[k + 1];
  if (blockIdx.x == 0 && k == 0 && threadIdx.x <= A.D)
    y.rk[threadIdx.x] = A.rk[threadIdx.x] * x.rk[threadIdx.x];
  const int n = A.n[k], m = A.m[k];
  const int P = ra0 * rx0;
  const int ncols = n * ra1 * rx1;
  // never write past the output slot (its caps bound the product ranks)
  if (P > y.cap[k] || ra1 * rx1 > y.cap[k + 1]) return;
  const double *Ak = A.data + A.off[k];
  const double *xk = x.data + x.off[k];
  double *yk = y.data + y.off[k];
  const int tx = threadIdx.x % MV_TX, ty = threadIdx.x / MV_TX;
  for (int col = blockIdx.x; col < ncols; col += gridDim.x) {
    const int i = col % n;
    const int s = col / n;
    const int c = s / rx1;
    const int d = s - c * rx1;
    double *ycol = yk + (int64_t)P * col;
    for (int b0 = 0; b0 < rx0; b0 += MV_TX) {
      const int b = b0 + tx;
      const bool act = b < rx0;
      if (m > MV_MMAX) {
        for (int a = ty; a < ra0; a += MV_TY) {
          const double *Aa = Ak + a + (int64_t)ra0 * (i + (int64_t)n * m * c);
          float acc = 0.0f;
          if (act)
            for (int j = 0; j < m; ++j)
              acc = fmaf(to_compute<T>(Aa[(int64_t)ra0 * n * j]),
                         to_compute<T>(xk[b + (int64_t)rx0 * (j + (int64_t)m * d)]), acc);
          if (act) __builtin_nontemporal_store(static_cast<double>(acc), &ycol[a * rx0 + b]);
        }
        continue;
      }
      float xv[MV_MMAX];
#pragma unroll
      for (int j = 0; j < MV_MMAX; ++j)
        xv[j] = (act && j < m)
                    ? to_compute<T>(xk[b + (int64_t)rx0 * (j + m * d)])
                    : 0.0f;
      for (int a = ty; a < ra0; a += MV_TY) {
        const double *Aa = Ak + a + (int64_t)ra0 * (i + (int64_t)n * m * c);
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < MV_MMAX; ++j)
          if (j < m) acc = fmaf(to_compute<T>(Aa[(int64_t)ra0 * n * j]), xv[j], acc);
        if (act) __builtin_nontemporal_store(static_cast<double>(acc), &ycol[a * rx0 + b]);
      }
    }
  }
}

__device__ __forceinline__ int64_t core_elems(const int *rk, const TTView &v,
                                              int k) {
  return (int64_t)rk[k] * v.n[k] * v.m[k] * rk[k + 1];
}

// packed <-> slotted: block y = core, grid-stride over elements
__global__ void k_pack(TTView v, double *packed, int to_packed) {
  const int k = blockIdx.y;
  if (v.rk[k] > v.cap[k] || v.rk[k + 1] > v.cap[k + 1]) return;
  int64_t off = 0;
  for (int l = 0; l < k; ++l) off += core_elems(v.rk, v, l);
  const int64_t ne = core_elems(v.rk, v, k);
  double *slot = v.data + v.off[k];
  double *pk = packed + off;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (to_packed)
      pk[e] = slot[e];
    else
      slot[e] = pk[e];
  }
}

__global__ void k_copy_tt(TTView a, TTView b) {
  const int k = blockIdx.y;
  if (blockIdx.x == 0 && k == 0 && threadIdx.x <= a.D)
    b.rk[threadIdx.x] = a.rk[threadIdx.x];
  if (a.rk[k] > b.cap[k] || a.rk[k + 1] > b.cap[k + 1]) return;
  const int64_t ne = core_elems(a.rk, a, k);
  const double *src = a.data + a.off[k];
  double *dst = b.data + b.off[k];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// z = a x + b y.  Core k of z has ranks (rx0+ry0, rx1+ry1) except at the
// ends; the scalars multiply the first core only.
__global__ void k_axpby(double a, const double *a_dev, TTView x, double b,
                        const double *b_dev, TTView y, TTView z) {
  const int k = blockIdx.y;
  const int D = x.D;
  const int rx0 = x.rk[k], rx1 = x.rk[k + 1];
  const int ry0 = y.rk[k], ry1 = y.rk[k + 1];
  if (blockIdx.x == 0 && k == 0 && threadIdx.x <= D) {
    const int t = threadIdx.x;
    z.rk[t] = (t == 0 || t == D) ? 1 : x.rk[t] + y.rk[t];
  }
  const double ca = a * (a_dev ? *a_dev : 1.0);
  const double cb = b * (b_dev ? *b_dev : 1.0);
  const int nm = x.n[k] * x.m[k];
  const int rz0 = (k == 0) ? 1 : rx0 + ry0;
  const int rz1 = (k == D - 1) ? 1 : rx1 + ry1;
  if (rz0 > z.cap[k] || rz1 > z.cap[k + 1]) return;
  const int64_t ne = (int64_t)rz0 * nm * rz1;
  const double *xk = x.data + x.off[k];
  const double *yk = y.data + y.off[k];
  double *zk = z.data + z.off[k];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(e % rz0);
    const int64_t rest = e / rz0;
    const int i = (int)(rest % nm);
    const int q = (int)(rest / nm);
    double v;
    if (D == 1) {
      v = ca * xk[i] + cb * yk[i];
    } else if (k == 0) {
      v = (q < rx1) ? ca * xk[i + (int64_t)nm * q]
                    : cb * yk[i + (int64_t)nm * (q - rx1)];
    } else if (k == D - 1) {
      v = (p < rx0) ? xk[p + (int64_t)rx0 * i] : yk[(p - rx0) + (int64_t)ry0 * i];
    } else {
      const bool inx = p < rx0, iny = q >= rx1;
      if (inx && !iny)
        v = xk[p + (int64_t)rx0 * (i + (int64_t)nm * q)];
      else if (!inx && iny)
        v = yk[(p - rx0) + (int64_t)ry0 * (i + (int64_t)nm * (q - rx1))];
      else
        v = 0.0;
    }
    zk[e] = v;
  }
}

// <x, y>: left environment Phi_{k+1} = sum_i x_k(:,i,:)^T Phi_k y_k(:,i,:),
// computed by one block; Phi and the intermediate T live in `ws`.
constexpr int DOT_THREADS = 1024;
// largest intermediate (rx0 n ry1 doubles) the one-workgroup <x, y> takes
constexpr int64_t DOT_ONE_BLOCK_MAX = 64 * 1024;
__global__ void __launch_bounds__(DOT_THREADS)
    k_dot(TTView x, TTView y, double *out, double *ws, int64_t phi_cap) {
  double *phi = ws;
  double *T = ws + phi_cap;
  const int D = x.D;
  if (threadIdx.x == 0) phi[0] = 1.0;
  __syncthreads();
  for (int k = 0; k < D; ++k) {
    const int rx0 = x.rk[k], rx1 = x.rk[k + 1];
    const int ry0 = y.rk[k], ry1 = y.rk[k + 1];
    const int n = x.n[k] * x.m[k];
    const double *xk = x.data + x.off[k];
    const double *yk = y.data + y.off[k];
    // T[a, i, b'] = sum_a' phi[a, a'] y[a', i, b']   (rx0 x n*ry1)
    const int tn = rx0 * n * ry1;
    for (int e = threadIdx.x; e < tn; e += blockDim.x) {
      const int a = e % rx0;
      const int col = e / rx0;  // i + n b'
      const double *ycol = yk + (int64_t)ry0 * col;
      double acc = 0.0;
      for (int a2 = 0; a2 < ry0; ++a2) acc = fma(phi[a + rx0 * a2], ycol[a2], acc);
      T[e] = acc;
    }
    __syncthreads();
    // phi'[b, b'] = sum_{a,i} x[a, i, b] T[a, i, b']   (rx1 x ry1)
    const int pn = rx1 * ry1;
    const int L = rx0 * n;
    for (int e = threadIdx.x; e < pn; e += blockDim.x) {
      const int b = e % rx1, b2 = e / rx1;
      const double *xc = xk + (int64_t)L * b;
      const double *tc = T + (int64_t)L * b2;
      double acc = 0.0;
      for (int l = 0; l < L; ++l) acc = fma(xc[l], tc[l], acc);
      phi[b + rx1 * b2] = acc;  // read of old phi finished before the barrier
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = phi[0];
}

// <x, A y> for TT vectors x, y and a TT matrix A: left environment
// Phi_{k+1}[b, beta, b'] = sum x_k[a,i,b] A_k[alpha,i,j,beta] y_k[a',j,b']
// Phi_k[a, alpha, a'], three contractions per core, one block.  The cost is
// O(r^3 R n + r^2 R^2 n^2) per core instead of the O(r (R r)^2 n) of <x, z>
// with z = A y formed first.  ws: Phi (phi_cap) then W1, W2 (w_cap each).
__global__ void __launch_bounds__(DOT_THREADS)
    k_dot3(TTView x, TTView A, TTView y, double *out, double *ws, int64_t phi_cap,
           int64_t w_cap) {
  double *phi = ws;
  double *W1 = ws + phi_cap;
  double *W2 = W1 + w_cap;
  const int D = x.D;
  for (int k = 0; k <= D; ++k)
    if (x.rk[k] > x.cap[k] || y.rk[k] > y.cap[k] || A.rk[k] > A.cap[k]) {
      if (threadIdx.x == 0) *out = NAN;
      return;
    }
  if (threadIdx.x == 0) phi[0] = 1.0;
  __syncthreads();
  for (int k = 0; k < D; ++k) {
    const int rx0 = x.rk[k], rx1 = x.rk[k + 1];
    const int ry0 = y.rk[k], ry1 = y.rk[k + 1];
    const int ra0 = A.rk[k], ra1 = A.rk[k + 1];
    const int n = x.n[k];
    const double *xk = x.data + x.off[k];
    const double *yk = y.data + y.off[k];
    const double *ak = A.data + A.off[k];
    // W1[a, al, j, b'] = sum_a' Phi[a, al, a'] y[a', j, b']
    const int64_t n1 = (int64_t)rx0 * ra0 * n * ry1;
    for (int64_t e = threadIdx.x; e < n1; e += blockDim.x) {
      const int aal = (int)(e % ((int64_t)rx0 * ra0));
      const int jb = (int)(e / ((int64_t)rx0 * ra0));
      const double *yc = yk + (int64_t)ry0 * jb;
      double acc = 0.0;
      for (int a2 = 0; a2 < ry0; ++a2) acc = fma(phi[aal + (int64_t)rx0 * ra0 * a2], yc[a2], acc);
      W1[e] = acc;
    }
    __syncthreads();
    // W2[a, i, be, b'] = sum_{al, j} W1[a, al, j, b'] A[al, i, j, be]
    const int64_t n2 = (int64_t)rx0 * n * ra1 * ry1;
    for (int64_t e = threadIdx.x; e < n2; e += blockDim.x) {
      const int a = (int)(e % rx0);
      int64_t t = e / rx0;
      const int i = (int)(t % n);
      t /= n;
      const int be = (int)(t % ra1);
      const int b2 = (int)(t / ra1);
      double acc = 0.0;
      for (int j = 0; j < n; ++j) {
        const double *w = W1 + a + (int64_t)rx0 * ra0 * (j + (int64_t)n * b2);
        const double *av = ak + (int64_t)ra0 * (i + (int64_t)n * (j + (int64_t)n * be));
        for (int al = 0; al < ra0; ++al) acc = fma(w[(int64_t)rx0 * al], av[al], acc);
      }
      W2[e] = acc;
    }
    __syncthreads();
    // Phi'[b, be, b'] = sum_{a, i} x[a, i, b] W2[a, i, be, b']
    const int L = rx0 * n;
    const int64_t n3 = (int64_t)rx1 * ra1 * ry1;
    for (int64_t e = threadIdx.x; e < n3; e += blockDim.x) {
      const int b = (int)(e % rx1);
      const int64_t col = e / rx1;  // be + ra1 b'
      const double *xc = xk + (int64_t)L * b;
      const double *wc = W2 + (int64_t)L * col;
      double acc = 0.0;
      for (int l = 0; l < L; ++l) acc = fma(xc[l], wc[l], acc);
      phi[e] = acc;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = phi[0];
}

// core 0 of a TT vector times c (ranks from the device)
__global__ void k_scale_first(TTView v, double c, const double *c_dev) {
  if (v.rk[1] > v.cap[1]) return;
  if (c_dev) c *= *c_dev;
  const int64_t ne = (int64_t)v.n[0] * v.m[0] * v.rk[1];
  double *c0 = v.data + v.off[0];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x)
    c0[e] *= c;
}

__global__ void k_scalar(int op, double *s0, const double *s1,
                         const double *s2, double c) {
  switch (op) {
    case SC_DIV: *s0 = *s1 / *s2; break;
    case SC_NEG: *s0 = -*s1; break;
    case SC_COPY: *s0 = *s1; break;
    case SC_SQRT_DIV: *s0 = sqrt(fmax(*s1, 0.0)) / c; break;
    case SC_SET: *s0 = c; break;
    case SC_DIV_POS: *s0 = (*s2 > 0.0) ? *s1 / *s2 : 0.0; break;
    case SC_NORM2: *s0 = fmax(s1[0] * s1[0] - s1[1], 0.0); break;
    case SC_DIFF_DIV: *s0 = (s2[0] > 0.0) ? (s1[0] - s1[1]) / s2[0] : 0.0; break;
  }
}

int max_cols(const TTView &v) {
  int mx = 1;
  for (int k = 0; k < v.D; ++k) {
    int c = v.n[k] * v.cap[k + 1];
    mx = c > mx ? c : mx;
  }
  return mx;
}

int64_t max_core_cap(const TTView &v) {
  int64_t mx = 1;
  for (int k = 0; k < v.D; ++k) {
    int64_t c = (int64_t)v.cap[k] * v.n[k] * v.m[k] * v.cap[k + 1];
    mx = c > mx ? c : mx;
  }
  return mx;
}

}  // namespace

hipError_t launch_scale(const TTView &v, double c, hipStream_t s, const double *c_dev) {
  const int64_t ne = (int64_t)v.n[0] * v.m[0] * v.cap[1];
  const int blocks = (int)std::min<int64_t>((ne + 255) / 256, 1024);
  hipLaunchKernelGGL(k_scale_first, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, v, c, c_dev);
  return hipGetLastError();
}

hipError_t launch_matvec(const TTView &A, const TTView &x, const TTView &y,
                         qtt_dtype compute, hipStream_t s) {
  int cols = 1;
  for (int k = 0; k < A.D; ++k) {
    int c = A.n[k] * A.cap[k + 1] * x.cap[k + 1];
    cols = c > cols ? c : cols;
  }
  // 1024 blocks per core, each looping over its columns, measured fastest at
  // level 10 (more blocks only add scheduling cost for these short columns)
  cols = cols < 1024 ? cols : 1024;
  dim3 grid(cols, A.D);
  dim3 block(MV_TX * MV_TY);
  bool staged = true;
  for (int k = 0; k < A.D; ++k)
    staged = staged && A.cap[k] * A.m[k] <= MV_SLICE && x.cap[k] * A.m[k] <= MV_SLICE;
  if (staged) {
    if (compute == QTT_F64)
      hipLaunchKernelGGL(k_matvec_f64, grid, dim3(256), 0, s, A, x, y);
    else if (compute == QTT_F32)
      hipLaunchKernelGGL(k_matvec_lp_staged<float>, grid, dim3(256), 0, s, A, x, y);
    else
      hipLaunchKernelGGL(k_matvec_lp_staged<__hip_bfloat16>, grid, dim3(256), 0, s, A, x, y);
  } else if (compute == QTT_F64) {
    hipLaunchKernelGGL(k_matvec_f64_direct, grid, block, 0, s, A, x, y);
  } else if (compute == QTT_F32) {
    hipLaunchKernelGGL(k_matvec_lp<float>, grid, block, 0, s, A, x, y);
  } else {
    hipLaunchKernelGGL(k_matvec_lp<__hip_bfloat16>, grid, block, 0, s, A, x, y);
  }
  return hipGetLastError();
}

hipError_t launch_unpack(const double *packed, const TTView &dst,
                         hipStream_t s) {
  int64_t mc = max_core_cap(dst);
  int blocks = (int)((mc + 255) / 256);
  blocks = blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096;
  hipLaunchKernelGGL(k_pack, dim3(blocks, dst.D), dim3(256), 0, s, dst,
                     const_cast<double *>(packed), 0);
  return hipGetLastError();
}

hipError_t launch_pack(const TTView &src, double *packed, hipStream_t s) {
  int64_t mc = max_core_cap(src);
  int blocks = (int)((mc + 255) / 256);
  blocks = blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096;
  hipLaunchKernelGGL(k_pack, dim3(blocks, src.D), dim3(256), 0, s, src,
                     packed, 1);
  return hipGetLastError();
}

hipError_t launch_copy_tt(const TTView &src, const TTView &dst,
                          hipStream_t s) {
  int64_t mc = max_core_cap(src);
  int blocks = (int)((mc + 255) / 256);
  blocks = blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096;
  hipLaunchKernelGGL(k_copy_tt, dim3(blocks, src.D), dim3(256), 0, s, src,
                     dst);
  return hipGetLastError();
}

hipError_t launch_axpby(double a, const double *a_dev, const TTView &x,
                        double b, const double *b_dev, const TTView &y,
                        const TTView &z, hipStream_t s) {
  int64_t mc = max_core_cap(z);
  int blocks = (int)((mc + 255) / 256);
  blocks = blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096;
  hipLaunchKernelGGL(k_axpby, dim3(blocks, x.D), dim3(256), 0, s, a, a_dev,
                     x, b, b_dev, y, z);
  return hipGetLastError();
}

// <x, y> over the whole chip for wide trains: per core two GEMMs with
// 64 x 64 output tiles (dev_gemm.h), ranks read from the device,
// T = Phi_k y_k (rx0 x n ry1, K = ry0) then Phi_{k+1} = x_k^T T
// (rx1 x ry1, K = rx0 n), Phi ping-ponging between two buffers.
__device__ __forceinline__ bool dot_beyond(const TTView &x, const TTView &y, int k) {
  return x.rk[k] > x.cap[k] || x.rk[k + 1] > x.cap[k + 1] || y.rk[k] > y.cap[k] ||
         y.rk[k + 1] > y.cap[k + 1];
}

__global__ void __launch_bounds__(256) k_dot_T(TTView x, TTView y, int k, const double *phi,
                                               double *T) {
  if (dot_beyond(x, y, k)) return;
  const int rx0 = x.rk[k], ry0 = y.rk[k], ry1 = y.rk[k + 1];
  const int N = x.n[k] * x.m[k] * ry1;
  if (blockIdx.x * dev::GT >= rx0 || blockIdx.y * dev::GT >= N) return;
  dev::gemm_tile<false>(phi, rx0, y.data + y.off[k], ry0, T, rx0, rx0, N, ry0, blockIdx.x,
                        blockIdx.y);
}

__global__ void __launch_bounds__(256) k_dot_P(TTView x, TTView y, int k, const double *T,
                                               double *phin) {
  if (dot_beyond(x, y, k)) return;
  const int rx1 = x.rk[k + 1], ry1 = y.rk[k + 1];
  const int K = x.rk[k] * x.n[k] * x.m[k];
  if (blockIdx.x * dev::GT >= rx1 || blockIdx.y * dev::GT >= ry1) return;
  dev::gemm_tile<true>(x.data + x.off[k], K, T, K, phin, rx1, rx1, ry1, K, blockIdx.x,
                       blockIdx.y);
}

__global__ void k_dot_init(double *phi) { phi[0] = 1.0; }

__global__ void k_dot_out(TTView x, TTView y, const double *phi, double *out) {
  bool bad = false;
  for (int k = 0; k <= x.D; ++k) bad = bad || x.rk[k] > x.cap[k] || y.rk[k] > y.cap[k];
  *out = bad ? NAN : phi[0];
}

hipError_t launch_dot(const TTView &x, const TTView &y, double *out,
                      double *ws, int64_t ws_elems, hipStream_t s) {
  int64_t phi_cap = 1, t_cap = 1;
  for (int k = 0; k <= x.D; ++k) {
    int64_t c = (int64_t)x.cap[k] * y.cap[k];
    phi_cap = c > phi_cap ? c : phi_cap;
  }
  for (int k = 0; k < x.D; ++k) {
    int64_t c = (int64_t)x.cap[k] * x.n[k] * x.m[k] * y.cap[k + 1];
    t_cap = c > t_cap ? c : t_cap;
  }
  if (phi_cap + t_cap > ws_elems) return hipErrorInvalidValue;
  // narrow trains: one workgroup walks all cores (no launch per core);
  // wide ones (a product against a vector): two chip-wide GEMMs per core
  if (t_cap <= DOT_ONE_BLOCK_MAX || 2 * phi_cap + t_cap > ws_elems) {
    hipLaunchKernelGGL(k_dot, dim3(1), dim3(DOT_THREADS), 0, s, x, y, out, ws, phi_cap);
    return hipGetLastError();
  }
  double *phi[2] = {ws, ws + phi_cap};
  double *T = ws + 2 * phi_cap;
  hipLaunchKernelGGL(k_dot_init, dim3(1), dim3(1), 0, s, phi[0]);
  for (int k = 0; k < x.D; ++k) {
    const int nm = x.n[k] * x.m[k];
    const int mt = (x.cap[k] + dev::GT - 1) / dev::GT;
    const int nt = (int)(((int64_t)nm * y.cap[k + 1] + dev::GT - 1) / dev::GT);
    hipLaunchKernelGGL(k_dot_T, dim3(mt, nt), dim3(256), 0, s, x, y, k, phi[k & 1], T);
    const int mt2 = (x.cap[k + 1] + dev::GT - 1) / dev::GT;
    const int nt2 = (y.cap[k + 1] + dev::GT - 1) / dev::GT;
    hipLaunchKernelGGL(k_dot_P, dim3(mt2, nt2), dim3(256), 0, s, x, y, k, T, phi[(k + 1) & 1]);
  }
  hipLaunchKernelGGL(k_dot_out, dim3(1), dim3(1), 0, s, x, y, phi[x.D & 1], out);
  return hipGetLastError();
}

void dot3_caps(const TTView &x, const TTView &A, const TTView &y, int64_t &phi, int64_t &w) {
  phi = 1;
  w = 1;
  for (int k = 0; k <= x.D; ++k) {
    int64_t c = (int64_t)x.cap[k] * A.cap[k] * y.cap[k];
    phi = c > phi ? c : phi;
  }
  for (int k = 0; k < x.D; ++k) {
    const int64_t n = x.n[k];
    int64_t c1 = (int64_t)x.cap[k] * A.cap[k] * n * y.cap[k + 1];
    int64_t c2 = (int64_t)x.cap[k] * n * A.cap[k + 1] * y.cap[k + 1];
    w = c1 > w ? c1 : w;
    w = c2 > w ? c2 : w;
  }
}

int64_t dot3_ws_elems(const TTView &x, const TTView &A, const TTView &y) {
  int64_t phi, w;
  dot3_caps(x, A, y, phi, w);
  return phi + 2 * w;
}

hipError_t launch_dot3(const TTView &x, const TTView &A, const TTView &y, double *out,
                       double *ws, int64_t ws_elems, hipStream_t s) {
  int64_t phi, w;
  dot3_caps(x, A, y, phi, w);
  if (phi + 2 * w > ws_elems) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dot3, dim3(1), dim3(DOT_THREADS), 0, s, x, A, y, out, ws, phi, w);
  return hipGetLastError();
}

int64_t dot_ws_elems(const TTView &x, const TTView &y) {
  int64_t phi_cap = 1, t_cap = 1;
  for (int k = 0; k <= x.D; ++k) {
    int64_t c = (int64_t)x.cap[k] * y.cap[k];
    phi_cap = c > phi_cap ? c : phi_cap;
  }
  for (int k = 0; k < x.D; ++k) {
    int64_t c = (int64_t)x.cap[k] * x.n[k] * x.m[k] * y.cap[k + 1];
    t_cap = c > t_cap ? c : t_cap;
  }
  return 2 * phi_cap + t_cap;   // two environment buffers and T
}

hipError_t launch_scalar(int op, double *s0, const double *s1,
                         const double *s2, double c, hipStream_t s) {
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(1), 0, s, op, s0, s1, s2, c);
  return hipGetLastError();
}

namespace {
struct RankArg {
  int D;
  int r[QTT_MAXD + 1];
};
__global__ void k_set_ranks(int *rk, RankArg a) {
  if ((int)threadIdx.x <= a.D) rk[threadIdx.x] = a.r[threadIdx.x];
}
}  // namespace

// ranks travel as a kernel argument, so the host array may be reused at once
hipError_t upload_ranks(const TTView &v, const int32_t *ranks,
                        hipStream_t s) {
  RankArg a;
  a.D = v.D;
  for (int k = 0; k <= v.D; ++k) a.r[k] = ranks[k];
  hipLaunchKernelGGL(k_set_ranks, dim3(1), dim3(64), 0, s, v.rk, a);
  return hipGetLastError();
}

}  // namespace qtt
