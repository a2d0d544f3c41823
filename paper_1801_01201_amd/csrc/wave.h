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

// gfx950's cross-row lane swaps on a double held in two 32-bit halves:
// swap_halves exchanges lanes 32-63 of x with lanes 0-31 of y; swap_rows
// exchanges the odd 16-lane rows of x with the even rows of y.
__device__ __forceinline__ double from_halves(unsigned lo, unsigned hi) {
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ void swap_halves(double& x, double& y) {
    const unsigned long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)bx, (unsigned)by, false, false);
    const auto hi =
        __builtin_amdgcn_permlane32_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
    x = from_halves(lo[0], hi[0]);
    y = from_halves(lo[1], hi[1]);
}
__device__ __forceinline__ void swap_rows(double& x, double& y) {
    const unsigned long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)bx, (unsigned)by, false, false);
    const auto hi =
        __builtin_amdgcn_permlane16_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
    x = from_halves(lo[0], hi[0]);
    y = from_halves(lo[1], hi[1]);
}

// Sums over the 64 lanes of the wavefront of K <= 32 values per lane
// (value(s) is this lane's value of slot s), by recursive halving: at each
// step a lane keeps half of its slots, adds its partner's copies of them and
// hands over the other half, the partner differing in lane bit 5, 4, 3, 2,
// then 1; a last step adds lane bit 0's partner.  The total of slot s ends
// in lanes 2s and 2s+1 (returned there; other lanes return the total of
// slot lane / 2, zero beyond K).  About 5 (K + 1) moves and adds instead of
// 20 K for K separate wave_sum calls.  The order of the additions is fixed,
// so the result is bitwise reproducible.  Must be called by all lanes.
template <int K, class F>
__device__ __forceinline__ double wave_sum_slots(F value) {
    static_assert(K >= 1 && K <= 32, "at most 32 slots");
    const int lane = threadIdx.x & 63;
    const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
    // evaluated depth first (each step's pair just before it is combined),
    // so that only a few partial sums are live at once
    auto s1 = [&](int i) -> double {                     // bit 5: slot i or i + 16
        if (i >= K) return 0.0;
        double x = value(i);
        double y = (i + 16 < K) ? value(i + 16) : 0.0;
        swap_halves(x, y);
        return x + y;
    };
    auto s2 = [&](int i) -> double {                     // bit 4: index i or i + 8
        double x = s1(i), y = s1(i + 8);
        swap_rows(x, y);
        return x + y;
    };
    auto s3 = [&](int i) -> double {                     // bit 3: lane ^ 8 = (lane + 8) mod 16
        const double lo = s2(i), hi = s2(i + 4);
        const double send = b3 ? lo : hi, keep = b3 ? hi : lo;
        return keep + dpp_move<0x128, 0xf>(send);        // row_ror:8
    };
    auto s4 = [&](int i) -> double {                     // bit 2: lane ^ 4
        const double lo = s3(i), hi = s3(i + 2);
        const double send = b2 ? lo : hi, keep = b2 ? hi : lo;
        const double from_minus4 = dpp_move<0x124, 0xf>(send);   // row_ror:4: lane - 4
        const double from_plus4 = dpp_move<0x12C, 0xf>(send);    // row_ror:12: lane + 4
        return keep + (b2 ? from_minus4 : from_plus4);
    };
    const double lo = s4(0), hi = s4(1);                 // bit 1: lane ^ 2
    const double send = b1 ? lo : hi, keep = b1 ? hi : lo;
    const double e = keep + dpp_move<0x4E, 0xf>(send);   // quad_perm [2,3,0,1]
    return e + dpp_move<0xB1, 0xf>(e);                   // bit 0: quad_perm [1,0,3,2]
}

}  // namespace misdc
