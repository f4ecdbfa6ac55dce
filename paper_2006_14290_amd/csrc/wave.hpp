// wave.hpp -- cross-lane primitives for 64-lane gfx950 wavefronts.
//
// The subwarp group model follows Section 3.3 of the paper: a subwarp of Size
// contiguous lanes has Rank = lane % Size, LaneOffset = (lane / Size) * Size
// and Mask = (~0 >> (64 - Size)) << LaneOffset over a 64-bit lane mask;
// ballot/any/all restrict the wavefront ballot to that mask.
//
// The reduction is the xor butterfly of the paper's reduction kernel
// (log2(Size) steps, every lane ends with the group sum), but no step goes
// through the LDS crossbar: partners 1 and 2 are DPP quad permutes, partners
// 4 and 8 are the DPP half-row and row mirrors, partner 16 is a ds_swizzle
// xor pattern and partner 32 is v_permlane32_swap. Because every lane of a
// group holds the same value after each step, the mirror steps form exactly
// the pairs the xor butterfly forms, so the sums are bitwise those of the
// butterfly order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spx {

constexpr int kWave = 64;
using lane_mask_t = uint64_t;

__device__ __forceinline__ int lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ lane_mask_t ballot64(bool p)
{
    return __builtin_amdgcn_ballot_w64(p);
}

template <int Size>
struct subwave {
    static_assert(Size >= 1 && Size <= kWave && (Size & (Size - 1)) == 0, "Size must be a power of two <= 64");
    __device__ static int rank() { return lane_id() % Size; }
    __device__ static int lane_offset() { return (lane_id() / Size) * Size; }
    __device__ static lane_mask_t mask()
    {
        return (~lane_mask_t(0) >> (kWave - Size)) << lane_offset();
    }
    __device__ static lane_mask_t ballot(bool p) { return (ballot64(p) & mask()) >> lane_offset(); }
    __device__ static bool any(bool p) { return (ballot64(p) & mask()) != 0; }
    __device__ static bool all(bool p) { return (ballot64(p) & mask()) == mask(); }
};

// ------------------------------------------------------------------ DPP moves
// DPP control words (GFX9 encoding).
enum : int {
    kQuadXor1 = 0xB1,        // quad_perm [1,0,3,2]
    kQuadXor2 = 0x4E,        // quad_perm [2,3,0,1]
    kRowHalfMirror = 0x141,  // lane i <-> 7-i inside each 8 lanes
    kRowMirror = 0x140,      // lane i <-> 15-i inside each 16 lanes
    kRowShr1 = 0x111,
    kRowBcast15 = 0x142,
    kRowBcast31 = 0x143,
};

template <int Ctrl, int RowMask = 0xF, int BankMask = 0xF, bool BoundCtrl = false>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v)
{
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(static_cast<int>(old), static_cast<int>(v), Ctrl,
                                                             RowMask, BankMask, BoundCtrl));
}

template <int Ctrl, int RowMask = 0xF, int BankMask = 0xF, bool BoundCtrl = false>
__device__ __forceinline__ double dpp(double old, double v)
{
    uint64_t o = __builtin_bit_cast(uint64_t, old), b = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = dpp_u32<Ctrl, RowMask, BankMask, BoundCtrl>(uint32_t(o), uint32_t(b));
    uint32_t hi = dpp_u32<Ctrl, RowMask, BankMask, BoundCtrl>(uint32_t(o >> 32), uint32_t(b >> 32));
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

template <int Ctrl, int RowMask = 0xF, int BankMask = 0xF, bool BoundCtrl = false>
__device__ __forceinline__ float dpp(float old, float v)
{
    return __builtin_bit_cast(float, dpp_u32<Ctrl, RowMask, BankMask, BoundCtrl>(__builtin_bit_cast(uint32_t, old),
                                                                                 __builtin_bit_cast(uint32_t, v)));
}

template <int Ctrl, int RowMask = 0xF, int BankMask = 0xF, bool BoundCtrl = false>
__device__ __forceinline__ int dpp(int old, int v)
{
    return static_cast<int>(dpp_u32<Ctrl, RowMask, BankMask, BoundCtrl>(uint32_t(old), uint32_t(v)));
}

// value of lane (lane ^ 16): ds_swizzle in bitmask mode (and 0x1F, xor 0x10)
__device__ __forceinline__ uint32_t swz_xor16_u32(uint32_t v)
{
    return static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(static_cast<int>(v), (0x10 << 10) | 0x1F));
}

// value of lane (lane ^ 32): v_permlane32_swap exchanges the upper half of
// the first operand with the lower half of the second; passing the same value
// twice yields the partner half in both results.
__device__ __forceinline__ uint32_t xor32_u32(uint32_t v)
{
    auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return lane_id() < 32 ? r[1] : r[0];
}

template <typename T>
__device__ __forceinline__ T xor16(T v);
template <typename T>
__device__ __forceinline__ T xor32(T v);

template <>
__device__ __forceinline__ double xor16<double>(double v)
{
    uint64_t b = __builtin_bit_cast(uint64_t, v);
    uint64_t r = (uint64_t(swz_xor16_u32(uint32_t(b >> 32))) << 32) | swz_xor16_u32(uint32_t(b));
    return __builtin_bit_cast(double, r);
}
template <>
__device__ __forceinline__ float xor16<float>(float v)
{
    return __builtin_bit_cast(float, swz_xor16_u32(__builtin_bit_cast(uint32_t, v)));
}
template <>
__device__ __forceinline__ double xor32<double>(double v)
{
    uint64_t b = __builtin_bit_cast(uint64_t, v);
    uint64_t r = (uint64_t(xor32_u32(uint32_t(b >> 32))) << 32) | xor32_u32(uint32_t(b));
    return __builtin_bit_cast(double, r);
}
template <>
__device__ __forceinline__ float xor32<float>(float v)
{
    return __builtin_bit_cast(float, xor32_u32(__builtin_bit_cast(uint32_t, v)));
}

// Sum over each subwarp of Size contiguous lanes; every lane receives its
// group's sum. log2(Size) steps.
template <int Size, typename T>
__device__ __forceinline__ T subwave_sum(T v)
{
    if constexpr (Size >= 2) v = v + dpp<kQuadXor1>(v, v);
    if constexpr (Size >= 4) v = v + dpp<kQuadXor2>(v, v);
    if constexpr (Size >= 8) v = v + dpp<kRowHalfMirror>(v, v);
    if constexpr (Size >= 16) v = v + dpp<kRowMirror>(v, v);
    if constexpr (Size >= 32) v = v + xor16(v);
    if constexpr (Size >= 64) v = v + xor32(v);
    return v;
}

// Runtime-size variant (size is wave-uniform, a power of two <= 64).
template <typename T>
__device__ __forceinline__ T subwave_sum_dyn(T v, int size)
{
    if (size >= 2) v = v + dpp<kQuadXor1>(v, v);
    if (size >= 4) v = v + dpp<kQuadXor2>(v, v);
    if (size >= 8) v = v + dpp<kRowHalfMirror>(v, v);
    if (size >= 16) v = v + dpp<kRowMirror>(v, v);
    if (size >= 32) v = v + xor16(v);
    if (size >= 64) v = v + xor32(v);
    return v;
}

// Inclusive segmented sum across the 64 lanes of a wavefront. A segment
// starts at every lane whose head flag is set (and at lane 0). Hillis-Steele
// combine (v, f) . (v', f') = (f' ? v' : v + v', f | f') using DPP row shifts
// inside each 16-lane row, then the row-15 and row-31 broadcasts across rows.
template <typename T>
__device__ __forceinline__ T wave_segscan(T v, bool head)
{
    int f = head ? 1 : 0;
    const T zero = T(0);
#define SPX_SEG_STEP(CTRL, ROWMASK)                                  \
    {                                                                \
        T pv = dpp<CTRL, ROWMASK, 0xF, true>(zero, v);               \
        int pf = dpp<CTRL, ROWMASK, 0xF, true>(0, f);                \
        T nv = f ? v : v + pv;                                       \
        int nf = f | pf;                                             \
        v = nv;                                                      \
        f = nf;                                                      \
    }
    // row_shr:d leaves lanes < d of each row with bound_ctrl zeros (pv = 0, pf = 0)
    SPX_SEG_STEP(0x111, 0xF)  // shr 1
    SPX_SEG_STEP(0x112, 0xF)  // shr 2
    SPX_SEG_STEP(0x114, 0xF)  // shr 4
    SPX_SEG_STEP(0x118, 0xF)  // shr 8
#undef SPX_SEG_STEP
    // rows 1 and 3 take lane 15 of the row below; rows 2 and 3 then take lane 31.
    {
        T pv = dpp<kRowBcast15, 0xA, 0xF, false>(zero, v);
        int pf = dpp<kRowBcast15, 0xA, 0xF, false>(0, f);
        const int row = lane_id() >> 4;
        if (row & 1) {
            T nv = f ? v : v + pv;
            f = f | pf;
            v = nv;
        }
    }
    {
        T pv = dpp<kRowBcast31, 0xC, 0xF, false>(zero, v);
        int pf = dpp<kRowBcast31, 0xC, 0xF, false>(0, f);
        const int row = lane_id() >> 4;
        if (row >= 2) {
            T nv = f ? v : v + pv;
            f = f | pf;
            v = nv;
        }
    }
    return v;
}

// Whole-wavefront shifts by one lane (DPP wave_shr:1 / wave_shl:1): lane i
// receives lane i-1 (resp. i+1); the lane with no source receives `fill`.
__device__ __forceinline__ int wave_shift_up1(int v, int fill)
{
    const int s = __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true);
    return lane_id() == 0 ? fill : s;
}

__device__ __forceinline__ int wave_shift_down1(int v, int fill)
{
    const int s = __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true);
    return lane_id() == kWave - 1 ? fill : s;
}

// Value held by lane src (wave-uniform src) as a scalar broadcast.
template <typename T>
__device__ __forceinline__ T readlane(T v, int src);

template <>
__device__ __forceinline__ double readlane<double>(double v, int src)
{
    uint64_t b = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(uint32_t(b)), src);
    uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(uint32_t(b >> 32)), src);
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
template <>
__device__ __forceinline__ float readlane<float>(float v, int src)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}
template <>
__device__ __forceinline__ int readlane<int>(int v, int src)
{
    return __builtin_amdgcn_readlane(v, src);
}

// Whole-wavefront sum, result uniform in every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    return subwave_sum<kWave>(v);
}

}  // namespace spx
