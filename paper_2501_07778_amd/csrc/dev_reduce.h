// dev_reduce.h — FP64 sums across lanes of a 64-wide wavefront (device code
// only), by DPP row moves instead of LDS permutes.
#pragma once

#include <hip/hip_runtime.h>

namespace qtt {
namespace dev {

// One FP64 value from another lane of the same 16-lane row by a DPP move of
// both halves (row-local patterns only, so every source lane is in the row).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of each row: swap neighbours, swap pairs (quad
// permutations [1,0,3,2] and [2,3,0,1]), then mirror within each half row
// and within the row.  Each step adds two partial sums that both lanes of
// a pair form alike, so all 16 lanes end with the same total.  Every lane
// of the row must be active.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return v;
}

// Sum over the whole wavefront, the same value in every lane: the row sums,
// then the four rows read from lanes 0, 16, 32 and 48 and added in that
// order.  Every lane of the wavefront must be active.
__device__ __forceinline__ double wave64_sum(double v) {
  v = row16_sum(v);
  const int lo = __double2loint(v), hi = __double2hiint(v);
  double s = __hiloint2double(__builtin_amdgcn_readlane(hi, 0), __builtin_amdgcn_readlane(lo, 0));
  s += __hiloint2double(__builtin_amdgcn_readlane(hi, 16), __builtin_amdgcn_readlane(lo, 16));
  s += __hiloint2double(__builtin_amdgcn_readlane(hi, 32), __builtin_amdgcn_readlane(lo, 32));
  s += __hiloint2double(__builtin_amdgcn_readlane(hi, 48), __builtin_amdgcn_readlane(lo, 48));
  return s;
}

// Reciprocal and reciprocal square root from the hardware estimates
// (v_rcp_f64, v_rsq_f64, about 23 correct bits) refined by Newton steps:
// one step gives about 46 bits, two about one ulp.  For the positive normal
// arguments of the rotations below.
template <int STEPS>
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int i = 0; i < STEPS; ++i) y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
template <int STEPS>
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < STEPS; ++i) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

}  // namespace dev
}  // namespace qtt

namespace qtt {
namespace dev {

constexpr int REFL_RG = 9;    // reflector rows per lane held in registers (16-lane groups)

// Apply the Householder reflector H = I - t v v^T, v = [1 at row j; vs * wj
// below it] (wj is the reflector's column, rows long, and vs a factor the
// caller has not yet applied to it), to the columns c0 <= c < c1 of Y
// (leading dimension ldy), NW wavefronts.  Each 16-lane group (one DPP row)
// takes one column at a time, so a wavefront works on four columns at once
// and a column's sum takes four DPP steps instead of a 64-lane reduction
// (about a quarter of the instructions per column), when the reflector
// spans at most 16 REFL_RG rows; every lane then keeps its part of it (rows
// j + lane + 16 k) in registers.
template <int NW>
__device__ __forceinline__ void reflect_cols(const double *wj, int j, int rows, double vs,
                                             double t, double *Y, int64_t ldy, int c0, int c1) {
  const int gl = threadIdx.x & 15, grp = threadIdx.x >> 4;
  constexpr int NG = NW * 4;
  if (rows - j <= 16 * REFL_RG) {
    // rows past the end read row j instead (in bounds) with a zero weight
    int iv[REFL_RG];
    double wv[REFL_RG];
#pragma unroll
    for (int k = 0; k < REFL_RG; ++k) {
      const int i = j + gl + 16 * k;
      const bool ok = i < rows;
      iv[k] = ok ? i : j;
      const double w = wj[iv[k]];
      wv[k] = (i == j) ? 1.0 : (ok ? vs * w : 0.0);
    }
    for (int c = c0 + grp; c < c1; c += NG) {
      double *yc = Y + ldy * c;
      double yv[REFL_RG];
#pragma unroll
      for (int k = 0; k < REFL_RG; ++k) yv[k] = yc[iv[k]];
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int k = 0; k < REFL_RG; k += 2) s0 = fma(wv[k], yv[k], s0);
#pragma unroll
      for (int k = 1; k < REFL_RG; k += 2) s1 = fma(wv[k], yv[k], s1);
      const double s = row16_sum(s0 + s1) * t;
#pragma unroll
      for (int k = 0; k < REFL_RG; ++k)
        if (j + gl + 16 * k < rows) yc[iv[k]] = yv[k] - s * wv[k];
    }
    return;
  }
  // longer reflectors: one column per wavefront and a 64-lane sum, so each
  // lane accumulates a quarter as many terms in sequence as a 16-lane group
  // would (the long QRs of the assembly, whose rounding error the solves at
  // high condition numbers see)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = c0 + wave; c < c1; c += NW) {
    double *yc = Y + ldy * c;
    double s = (lane == 0) ? yc[j] : 0.0;
    for (int i = j + 1 + lane; i < rows; i += 64) s = fma(vs * wj[i], yc[i], s);
    s = wave64_sum(s) * t;
    if (lane == 0) yc[j] -= s;
    for (int i = j + 1 + lane; i < rows; i += 64) yc[i] -= s * (vs * wj[i]);
  }
}

}  // namespace dev
}  // namespace qtt
