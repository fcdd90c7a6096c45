// ot_device.hpp -- gfx950 device helpers shared by the kernels: clamping,
// wave-uniform values, wave64 DPP reductions and the XCD-aware work remap.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ot_common.hpp"

namespace ot {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// floor(a / b) for 0 <= a <= 4096 and 1 <= b <= 256 through the hardware
// reciprocal: (a + 1/2) / b lies at least 1/(2b) away from an integer, far
// more than the reciprocal's error (exhaustively checked in the CPU tests,
// with the reciprocal off by up to two ulps).
__device__ __forceinline__ int udiv_small(int a, int b) {
    return (int)(((float)a + 0.5f) * __builtin_amdgcn_rcpf((float)b));
}

// Raw buffer view of a byte plane: loads take 32-bit byte offsets (no 64-bit
// address arithmetic per lane) and return 0 past `bytes`.  `p` and `bytes`
// must be wave-uniform (the descriptor lives in scalar registers).
typedef __amdgpu_buffer_rsrc_t plane_t;

__device__ __forceinline__ plane_t plane_rsrc(const uint8_t* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(p), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ __forceinline__ uint32_t plane_dword(plane_t r, uint32_t off) {
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
}
__device__ __forceinline__ uint32_t plane_byte(plane_t r, uint32_t off) {
    return (uint32_t)(uint8_t)__builtin_amdgcn_raw_buffer_load_b8(r, (int)off, 0, 0);
}

__device__ __forceinline__ float uniform_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// One DPP move of a float across lanes (GFX9 DPP control codes); lanes whose
// source is outside the row, or rows masked off, read 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF, true));
}

// Sum over the 64 lanes of a wave; every lane gets the total.  Within a row
// of 16 lanes: two quad permutes, half-row mirror and row mirror leave the row
// total in every lane; row_bcast:15 and row_bcast:31 then fold the four row
// totals into lane 63, which is broadcast.  All 64 lanes must be active.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<0xB1>(v);       // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);       // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);      // row_half_mirror
    v += dpp_f<0x140>(v);      // row_mirror
    v += dpp_f<0x142, 0xA>(v); // row_bcast:15 -> rows 1, 3
    v += dpp_f<0x143, 0xC>(v); // row_bcast:31 -> rows 2, 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Integer DPP move: rows masked off (and, with bound_ctrl, lanes whose source
// is outside the row) return `old`/0 as the GFX9 DPP rules give.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_u(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xF, true);
}

// Minimum / maximum over the 64 lanes (same DPP pattern as wave_sum; masked
// rows keep their own value).  All 64 lanes must be active.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    v = min(v, dpp_u<0xB1>(v, v));
    v = min(v, dpp_u<0x4E>(v, v));
    v = min(v, dpp_u<0x141>(v, v));
    v = min(v, dpp_u<0x140>(v, v));
    v = min(v, dpp_u<0x142, 0xA>(v, v));
    v = min(v, dpp_u<0x143, 0xC>(v, v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, dpp_u<0xB1>(v, v));
    v = max(v, dpp_u<0x4E>(v, v));
    v = max(v, dpp_u<0x141>(v, v));
    v = max(v, dpp_u<0x140>(v, v));
    v = max(v, dpp_u<0x142, 0xA>(v, v));
    v = max(v, dpp_u<0x143, 0xC>(v, v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Inclusive prefix sum over the 64 lanes: row_shr 1, 2, 4, 8 scan each row of
// 16, row_bcast:15 and row_bcast:31 carry the row totals forward.  All 64
// lanes must be active.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
    v += dpp_u<0x111>(0u, v);
    v += dpp_u<0x112>(0u, v);
    v += dpp_u<0x114>(0u, v);
    v += dpp_u<0x118>(0u, v);
    v += dpp_u<0x142, 0xA>(0u, v);
    v += dpp_u<0x143, 0xC>(0u, v);
    return v;
}

// Workgroup b runs on XCD b % 8; hand each XCD one contiguous range of work
// items so neighbouring points share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
    const int X = 8;
    const int q = G / X, rem = G % X;
    const int xcd = b % X, k = b / X;
    return (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) + k;
}

}  // namespace ot
