// Wavefront-level float64 helpers shared by the kernels: lane exchanges on
// the data-parallel-primitive path of the vector ALU and a fixed-order sum
// over the 64 lanes.
#pragma once

#include <hip/hip_runtime.h>

namespace jkc {

// v from another lane of the same row of 16 lanes (DPP control Ctrl), both
// 32-bit halves moved by the data-parallel-primitive path of the VALU (no
// trip through the LDS unit).
template <int Ctrl>
__device__ inline double dpp_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, Ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), Ctrl, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ inline double lane_f64(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes of a wavefront, every lane active: pairs, quads,
// eighths and rows of 16 combine by DPP lane swaps (each step adds two equal
// partial sums in either order, and a + b == b + a exactly, so every lane of
// a row holds the same bits), then the four row sums in the fixed order
// (r0 + r1) + (r2 + r3).  Every lane gets the result; the same lanes combine
// in the same order on every run.  The additions are not contracted: were
// the caller's last product fused into the first one, the two lanes of a
// pair would round differently and the sum would depend on the call site.
__device__ inline double wave_sum(double v) {
#pragma clang fp contract(off)
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
  v += dpp_f64<0x141>(v);   // row_half_mirror: the other quad of the eight
  v += dpp_f64<0x140>(v);   // row_mirror: the other eight of the row
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

}  // namespace jkc
