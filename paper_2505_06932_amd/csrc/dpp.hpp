// dpp.hpp -- cross-lane moves by DPP (data-parallel primitives): a VALU
// operand taken from another lane of the same row of 16 lanes, or from the
// row broadcasts, register to register.  An LDS shuffle (ds_bpermute)
// instead issues an LDS instruction and waits for it, which costs issue
// slots in kernels bound by instruction issue.  Lanes whose source falls
// outside its row, or whose row the row mask leaves out, receive 0.
// Every caller has all 64 lanes of its wavefront active.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ftc {

// Controls used here (GFX9 encoding).
constexpr int kDppSwap1 = 0xB1;        // quad_perm [1,0,3,2]: lane i takes lane i ^ 1
constexpr int kDppSwap2 = 0x4E;        // quad_perm [2,3,0,1]: lane i takes lane i ^ 2
constexpr int kDppHalfMirror = 0x141;  // lane i of each 8 takes lane 7 - i
constexpr int kDppMirror = 0x140;      // lane i of each 16 takes lane 15 - i
constexpr int kDppShr = 0x110;         // + n: row_shr:n, lane i takes lane i - n of its row
constexpr int kDppRor = 0x120;         // + n: row_ror:n, lane i takes lane (i - n) mod 16 of its row
constexpr int kDppBcast15 = 0x142;     // lane 15 of each row into the next row
constexpr int kDppBcast31 = 0x143;     // lane 31 into rows 2 and 3

template <int CTRL, int ROWS = 0xF>
__device__ inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS = 0xF>
__device__ inline float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL, ROWS>(__float_as_int(v)));
}

template <int CTRL, int ROWS = 0xF>
__device__ inline double dpp_d(double v) {
  const int lo = dpp_i<CTRL, ROWS>(__double2loint(v)), hi = dpp_i<CTRL, ROWS>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Inclusive prefix sum over the wavefront's 64 lanes: prefix sums within
// each row by shifts of 1, 2, 4 and 8 lanes, then row 0's total into row 1
// and row 2's into row 3, then rows 0-1's total into rows 2 and 3.
__device__ inline int32_t wave_incl_scan_dpp(int32_t v) {
  v += dpp_i<kDppShr + 1>(v);
  v += dpp_i<kDppShr + 2>(v);
  v += dpp_i<kDppShr + 4>(v);
  v += dpp_i<kDppShr + 8>(v);
  v += dpp_i<kDppBcast15, 0xA>(v);
  v += dpp_i<kDppBcast31, 0xC>(v);
  return v;
}

// Maximum of a non-negative value over the wavefront, in every lane.
__device__ inline int wave_max_dpp(int v) {
  v = max(v, dpp_i<kDppSwap1>(v));
  v = max(v, dpp_i<kDppSwap2>(v));
  v = max(v, dpp_i<kDppHalfMirror>(v));
  v = max(v, dpp_i<kDppMirror>(v));
  v = max(v, dpp_i<kDppBcast15, 0xA>(v));
  v = max(v, dpp_i<kDppBcast31, 0xC>(v));
  return __builtin_amdgcn_readlane(v, 63);
}

}  // namespace ftc
