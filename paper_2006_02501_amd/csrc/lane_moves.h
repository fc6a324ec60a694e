// Moves of values between the lanes of one wave64, for sums that travel with
// the body they belong to while a wave sweeps over pairs.  Every lane of the
// wave must be active.
#pragma once

#include <hip/hip_runtime.h>

namespace hermite {

// One lane down the whole wave (DPP wave rotate left by one): lane l receives
// lane l + 1's value, lane 63 receives lane 0's.
__device__ __forceinline__ double lane_down(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x134, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x134, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float lane_down(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x134, 0xF, 0xF, false));
}

// The value of lane addr / 4 (ds_bpermute: it goes through the LDS unit).
__device__ __forceinline__ double lane_from(int addr, double x)
{
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(x));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(x));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float lane_from(int addr, float x)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x)));
}

}  // namespace hermite
