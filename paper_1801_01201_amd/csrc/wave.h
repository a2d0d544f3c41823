// Wavefront (64-lane) reductions with DPP lane permutations.
//
// Each step is a VALU move with a data-parallel-primitive modifier instead of
// an LDS permute, so a full 64-lane sum costs a handful of short-latency
// instructions.  The lane order of the additions is fixed, so the result is
// bitwise reproducible.  Doubles are moved as two 32-bit halves.
#pragma once

#include <hip/hip_runtime.h>

namespace misdc {

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
    // lanes of disabled rows (or reading outside their row) get 0
    const int rlo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false);
    const int rhi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double(((long long)rhi << 32) | (unsigned)rlo);
}

// Sum of v over the 64 lanes of the wavefront, returned in every lane.
// Must be called by all lanes of the wave (uniform control flow).
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0xB1, 0xf>(v);     // quad_perm [1,0,3,2]
    v += dpp_move<0x4E, 0xf>(v);     // quad_perm [2,3,0,1]
    v += dpp_move<0x141, 0xf>(v);    // row_half_mirror: sum over 8 lanes
    v += dpp_move<0x140, 0xf>(v);    // row_mirror: sum over the 16-lane row
    v += dpp_move<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

}  // namespace misdc
