// Device helpers shared by the X-stage kernels.
#pragma once

#include "xcorr_internal.h"

namespace xcorr {

constexpr int kRsrcConfig = 0x00020000;    // buffer resource word 3 for gfx9-family raw loads

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel)
{
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// r[k] holds bytes (x0, x1, x2, x3) of sample k; returns o[m] = (sample 0..3)
// of byte column m: a 4x4 byte transpose in eight v_perm_b32.
__device__ __forceinline__ void transpose4(const uint32_t r[4], uint32_t o[4])
{
    const uint32_t p0 = perm(r[1], r[0], 0x05010400u);
    const uint32_t p1 = perm(r[1], r[0], 0x07030602u);
    const uint32_t p2 = perm(r[3], r[2], 0x05010400u);
    const uint32_t p3 = perm(r[3], r[2], 0x07030602u);
    o[0] = perm(p2, p0, 0x05040100u);
    o[1] = perm(p2, p0, 0x07060302u);
    o[2] = perm(p3, p1, 0x05040100u);
    o[3] = perm(p3, p1, 0x07060302u);
}

// Range-checked loads of one wave's channel: samples past the chunk (and a
// channel past n_channels, given range 0) read as zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t channel_rsrc(const LaunchArgs& a, int rb, int ch)
{
    const bool ok = rb >= 0 && ch < a.n_channels;
    const uint8_t* base = a.in + (ok ? (int64_t)ch * a.chan_stride : 0);
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, ok ? a.t_len * a.row_bytes : 0,
                                             kRsrcConfig);
}

__device__ __forceinline__ uint32_t load_b32(__amdgpu_buffer_rsrc_t r, uint32_t ofs)
{
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)ofs, 0, 0);
}

// Column offset of an input, or an offset beyond every valid range.
__device__ __forceinline__ uint32_t column_offset(int input, int n_inputs, int bytes_per_sample)
{
    return input < n_inputs ? (uint32_t)input * (uint32_t)bytes_per_sample : 0x80000000u;
}

__device__ __forceinline__ constexpr bool block_on(int kind, int bi, int bj)
{
    return (kind_mask(kind) >> (4 * bi + bj)) & 1u;
}

// True if the kind owns any block in column bj.
__device__ __forceinline__ constexpr bool column_on(int kind, int bj)
{
    return (kind_mask(kind) & (0x1111u << bj)) != 0;
}

// True if the kind owns any block in row bi.
__device__ __forceinline__ constexpr bool row_on(int kind, int bi)
{
    return (kind_mask(kind) & (0xFu << (4 * bi))) != 0;
}

}  // namespace xcorr
