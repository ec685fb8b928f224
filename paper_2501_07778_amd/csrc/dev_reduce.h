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

}  // namespace dev
}  // namespace qtt
