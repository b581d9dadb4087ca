// Wavefront-level helpers shared by the kernels: DPP lane shifts and the
// segmented inclusive scan over runs of contiguous lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ba {

// Lane shifts through DPP (data-parallel primitives: the shift rides on a
// VALU move, with no LDS round trip).  CTRL: row_shr:n = 0x110 + n (within
// rows of 16 lanes), row_bcast:15 = 0x142 (lane 15 of each row to the next
// row), row_bcast:31 = 0x143 (lane 31 to rows 2 and 3), wave_shr:1 = 0x138.
// Lanes without a source read 0; rows outside ROWMASK read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_shift(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWMASK, 0xf,
                                                                 true));
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_shift(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWMASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWMASK, 0xf, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// The value of lane - 1 (lane 0 reads `first`).
__device__ __forceinline__ int32_t lane_before(int32_t v, int32_t first)
{
    return __builtin_amdgcn_update_dpp(first, v, 0x138, 0xf, 0xf, false);
}

// Inclusive sums of (a0, a1, a2) over each lane's run [seg_s, lane] of
// contiguous lanes: within rows of 16 by shifts of 1, 2, 4 and 8, then the
// last lane of row r into row r + 1 and lane 31 into rows 2 and 3 (the
// row-carry form of a wave scan).  A step adds the shifted value times 1 where
// its source lies in the lane's run and times 0 elsewhere (exactly an add or
// nothing for finite values).
template <typename T>
__device__ __forceinline__ void run_prefix3(T& a0, T& a1, T& a2, int lane, int seg_s)
{
    const T m1 = lane - 1 >= seg_s ? (T)1 : (T)0;
    const T m2 = lane - 2 >= seg_s ? (T)1 : (T)0;
    const T m4 = lane - 4 >= seg_s ? (T)1 : (T)0;
    const T m8 = lane - 8 >= seg_s ? (T)1 : (T)0;
    const T m16 = (lane & ~15) - 1 >= seg_s ? (T)1 : (T)0;
    const T m32 = (lane > 31 && seg_s <= 31) ? (T)1 : (T)0;
#define BA_RUN_STEP(CTRL, ROWMASK, M)                 \
    a0 = fma(dpp_shift<CTRL, ROWMASK>(a0), M, a0); \
    a1 = fma(dpp_shift<CTRL, ROWMASK>(a1), M, a1); \
    a2 = fma(dpp_shift<CTRL, ROWMASK>(a2), M, a2);
    BA_RUN_STEP(0x111, 0xf, m1)
    BA_RUN_STEP(0x112, 0xf, m2)
    BA_RUN_STEP(0x114, 0xf, m4)
    BA_RUN_STEP(0x118, 0xf, m8)
    BA_RUN_STEP(0x142, 0xa, m16)
    BA_RUN_STEP(0x143, 0xc, m32)
#undef BA_RUN_STEP
}

// FP32: each step is one v_fmac_f32 with the shifted value as its DPP
// source (a += shift(a) * m), where the compiler would emit a DPP move and an
// FMA; the same arithmetic, a third fewer instructions.  s_nop 1 gives the
// two wait states a DPP read needs after the VALU write of its source.
#define BA_FMAC3_DPP(A0, A1, A2, M, DPP)                                                   \
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %3 " DPP "\n\tv_fmac_f32_dpp %1, %1, %3 " DPP \
                 "\n\tv_fmac_f32_dpp %2, %2, %3 " DPP                                       \
                 : "+v"(A0), "+v"(A1), "+v"(A2)                                            \
                 : "v"(M))

template <>
__device__ __forceinline__ void run_prefix3<float>(float& a0, float& a1, float& a2, int lane, int seg_s)
{
    const float m1 = lane - 1 >= seg_s ? 1.0f : 0.0f;
    const float m2 = lane - 2 >= seg_s ? 1.0f : 0.0f;
    const float m4 = lane - 4 >= seg_s ? 1.0f : 0.0f;
    const float m8 = lane - 8 >= seg_s ? 1.0f : 0.0f;
    const float m16 = (lane & ~15) - 1 >= seg_s ? 1.0f : 0.0f;
    const float m32 = (lane > 31 && seg_s <= 31) ? 1.0f : 0.0f;
    BA_FMAC3_DPP(a0, a1, a2, m1, "row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    BA_FMAC3_DPP(a0, a1, a2, m2, "row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    BA_FMAC3_DPP(a0, a1, a2, m4, "row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    BA_FMAC3_DPP(a0, a1, a2, m8, "row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    BA_FMAC3_DPP(a0, a1, a2, m16, "row_bcast:15 row_mask:0xa bank_mask:0xf");
    BA_FMAC3_DPP(a0, a1, a2, m32, "row_bcast:31 row_mask:0xc bank_mask:0xf");
}
#undef BA_FMAC3_DPP

// Inclusive sums of the NV values a[] over each lane's run [seg_s, lane],
// in the same steps as run_prefix3 (an add or nothing for finite values; a
// non-finite value can reach the other runs of its wavefront).
template <typename T, int NV>
__device__ __forceinline__ void run_prefix(T* a, int lane, int seg_s)
{
    const T m1 = lane - 1 >= seg_s ? (T)1 : (T)0;
    const T m2 = lane - 2 >= seg_s ? (T)1 : (T)0;
    const T m4 = lane - 4 >= seg_s ? (T)1 : (T)0;
    const T m8 = lane - 8 >= seg_s ? (T)1 : (T)0;
    const T m16 = (lane & ~15) - 1 >= seg_s ? (T)1 : (T)0;
    const T m32 = (lane > 31 && seg_s <= 31) ? (T)1 : (T)0;
#define BA_RUN_STEP(CTRL, ROWMASK, M)                                      \
    _Pragma("unroll") for (int q = 0; q < NV; ++q) a[q] = fma(dpp_shift<CTRL, ROWMASK>(a[q]), M, a[q]);
    BA_RUN_STEP(0x111, 0xf, m1)
    BA_RUN_STEP(0x112, 0xf, m2)
    BA_RUN_STEP(0x114, 0xf, m4)
    BA_RUN_STEP(0x118, 0xf, m8)
    BA_RUN_STEP(0x142, 0xa, m16)
    BA_RUN_STEP(0x143, 0xc, m32)
#undef BA_RUN_STEP
}

}  // namespace ba
