// lanes.h -- neighbour exchange between the lanes of one wave by DPP
// whole-wave shifts (wave_shl:1 / wave_shr:1): a lane reads a register of
// the next or previous lane without going through LDS.  A 64-bit value moves
// as two 32-bit halves; lanes shifted in from outside the wave read 0.
#pragma once

#include <hip/hip_runtime.h>

namespace sw {

// lane l receives v of lane l+1 (lane 63 receives 0)
__device__ __forceinline__ double from_next_lane(double v)
{
    const long long vi = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)vi, 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(vi >> 32), 0x130, 0xf, 0xf, true);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

__device__ __forceinline__ float from_next_lane(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// lane l receives v of lane l-1 (lane 0 receives 0)
__device__ __forceinline__ double from_prev_lane(double v)
{
    const long long vi = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)vi, 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(vi >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

__device__ __forceinline__ float from_prev_lane(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}

} // namespace sw
