// wave_ops.h -- wavefront reductions for gfx950 kernels (DPP moves inside rows of
// 16 lanes, readlane across rows); every sum is taken in a fixed order, so equal
// inputs give equal bits.
#pragma once

#include <hip/hip_runtime.h>

#include "amg_internal.h"

namespace amg {
namespace {

// Cross-lane moves inside rows of 16 lanes (DPP, no LDS traffic): exchange with
// lane ^ 1 and lane ^ 2 inside a quad, mirror inside 8 lanes, mirror inside 16.
constexpr int kDppQuadXor1 = 0xB1, kDppQuadXor2 = 0x4E, kDppRowHalfMirror = 0x141, kDppRowMirror = 0x140;
template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// Sum over each row of 16 lanes, received by every lane of the row: each step adds
// the partner's partial sum, and both partners form the same sum (fixed order).
// The lanes of the row must be active.
__device__ inline double row16_sum(double v)
{
    v += dpp_f64<kDppQuadXor1>(v);
    v += dpp_f64<kDppQuadXor2>(v);
    v += dpp_f64<kDppRowHalfMirror>(v);
    v += dpp_f64<kDppRowMirror>(v);
    return v;
}
// v of one lane, as a wavefront-uniform value
__device__ inline double lane_value(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}
// Sum over the wavefront, the same value in every lane (fixed order).  All lanes
// must be active.
__device__ inline double wave_sum(double v)
{
    v = row16_sum(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Sum over each aligned group of G lanes, received by every lane of the group
// (fixed order).  The moves stay inside the group, so lanes of other groups may
// be inactive.
template <int G>
__device__ inline double group_sum(double v)
{
    if (G >= 2) v += dpp_f64<kDppQuadXor1>(v);
    if (G >= 4) v += dpp_f64<kDppQuadXor2>(v);
    if (G >= 8) v += dpp_f64<kDppRowHalfMirror>(v);
    if (G >= 16) v += dpp_f64<kDppRowMirror>(v);
    if (G >= 32) v += __shfl_xor(v, 16, kWave);
    if (G >= 64) v += __shfl_xor(v, 32, kWave);
    return v;
}

}  // namespace
}  // namespace amg
