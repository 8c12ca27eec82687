// Cross-lane exchanges of 64-bit values inside a 64-lane wavefront (gfx950):
// 32- and 16-lane swaps (v_permlane32_swap / v_permlane16_swap) and DPP
// permutations inside quads, used by the transposed reductions of the
// Legendre adjoint and of the coefficient rotation.
#pragma once

#include <hip/hip_runtime.h>

namespace psht {

// Swap the upper 32 lanes of x with the lower 32 lanes of y (64-bit values).
__device__ inline void swap32(double &x, double &y) {
    unsigned xl = __double2loint(x), xh = __double2hiint(x), yl = __double2loint(y), yh = __double2hiint(y);
    auto lo = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
    x = __hiloint2double(hi[0], lo[0]);
    y = __hiloint2double(hi[1], lo[1]);
}

// Same at 16-lane granularity inside each half of the wave.
__device__ inline void swap16(double &x, double &y) {
    unsigned xl = __double2loint(x), xh = __double2hiint(x), yl = __double2loint(y), yh = __double2hiint(y);
    auto lo = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    auto hi = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    x = __hiloint2double(hi[0], lo[0]);
    y = __hiloint2double(hi[1], lo[1]);
}

// x from lane i ^ 1 and i ^ 2 of the quad (DPP quad permutations, 64-bit values).
__device__ inline double quad_xor1(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0xB1, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ inline double quad_xor2(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x4E, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x4E, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

}  // namespace psht
