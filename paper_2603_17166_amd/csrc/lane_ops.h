// Cross-lane exchanges of 64-bit values inside a 64-lane wavefront (gfx950):
// 32- and 16-lane swaps (v_permlane32_swap / v_permlane16_swap) and DPP
// permutations (xor 1, 2, 4, 8), used by the transposed reductions of the
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

// x from lane i ^ 4 (DPP: mirror inside each 8-lane half row, then reverse
// each quad) and from lane i ^ 8 (DPP row rotation by 8 inside 16-lane rows).
__device__ inline int lane_xor4_b32(int v) {
    return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false), 0x1B, 0xF, 0xF, false);
}
__device__ inline double lane_xor4(double x) {
    return __hiloint2double(lane_xor4_b32(__double2hiint(x)), lane_xor4_b32(__double2loint(x)));
}
__device__ inline double lane_xor8(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x128, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x128, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

}  // namespace psht
