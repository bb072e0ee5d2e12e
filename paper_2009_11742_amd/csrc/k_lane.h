// Cross-lane moves of the operator-resident kernels (FP32 and FP64 forms):
// DPP partner patterns inside a 16-lane row, the register row order that
// lets a halving row sum keep its registers in place, the row gather, the
// permlane16 / permlane32 swap levels between the 16-lane rows of a wave,
// and lane reads.  gfx950 only (v_permlane16_swap, v_permlane32_swap).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rom {
namespace lane {

// DPP controls (gfx9 encoding)
constexpr int kDppRor8 = 0x128;            // row_ror:8        (p ^ 8)
constexpr int kDppHalfMirror = 0x141;      // row_half_mirror  (p ^ 7)
constexpr int kDppXor2 = 0x4E;             // quad_perm [2,3,0,1]
constexpr int kDppXor1 = 0xB1;             // quad_perm [1,0,3,2]

// Every lane of these patterns has a source lane; bound_ctrl with a zero
// "old" lets the compiler fold the move into the add that consumes it.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xf, 0xf, true));
}

// Partner value at halving level LEVEL (lane pairs p ^ 8, p ^ 7, p ^ 2, p ^ 1).
template <int LEVEL>
__device__ __forceinline__ float level_partner(float x) {
    if constexpr (LEVEL == 0) return dpp_mov<kDppRor8>(x);
    else if constexpr (LEVEL == 1) return dpp_mov<kDppHalfMirror>(x);
    else if constexpr (LEVEL == 2) return dpp_mov<kDppXor2>(x);
    else return dpp_mov<kDppXor1>(x);
}

// Register order of a lane's tile rows: register i holds tile row i ^ s(p).
// With b3 b2 b1 the bits of p: TR = 8: s = 4 b3 + 2 b2 + (b1 ^ b2); TR = 4:
// s = 2 b3 + b2; TR = 2: s = b3.  Level k's partner changes s by exactly
// TR >> (k + 1) while 2 (TR >> (k + 1)) registers are live, and leaves it
// unchanged at the levels after the halving (which then add equal rows).
__host__ __device__ __forceinline__ int row_xor(int TR, int p) {
    const int b3 = (p >> 3) & 1, b2 = (p >> 2) & 1, b1 = (p >> 1) & 1;
    if (TR == 8) return 4 * b3 + 2 * b2 + (b1 ^ b2);
    if (TR == 4) return 2 * b3 + b2;
    return b3;
}

// Sum over the 16 lanes of the DPP row of the row partials acc[0 .. TR):
// afterwards acc[0] holds the sum for tile row s(p).
template <int TR, int LEVEL = 0>
__device__ __forceinline__ void row_sum(float (&acc)[TR]) {
    if constexpr (LEVEL < 4) {
        constexpr int H = TR >> (LEVEL + 1);
        if constexpr (H >= 1) {
#pragma unroll
            for (int t = 0; t < H; ++t) acc[t] = acc[t] + level_partner<LEVEL>(acc[t + H]);
        } else {
            acc[0] = acc[0] + level_partner<LEVEL>(acc[0]);
        }
        row_sum<TR, LEVEL + 1>(acc);
    }
}

// The TR new V values of a lane's row block, in its register order:
// vv[i] = V row TR rb + (i ^ s(p)), i.e. the value of a lane p' of the same
// DPP row with s(p') = s(p) ^ i.  s is linear in the bits of p, so one
// partner pattern per bit of i builds them all by doubling: TR = 8: bit 2 is
// p ^ 8 (row_ror:8), bit 1 p ^ 7 (row_half_mirror), bit 0 p ^ 2 (quad_perm
// xor 2); TR = 4: p ^ 8 and p ^ 7; TR = 2: p ^ 8.
template <int TR>
__device__ __forceinline__ void row_gather(float vh, float (&vv)[TR]) {
    vv[0] = vh;
    if constexpr (TR == 8) {
        vv[4] = dpp_mov<kDppRor8>(vv[0]);
        vv[2] = dpp_mov<kDppHalfMirror>(vv[0]);
        vv[6] = dpp_mov<kDppHalfMirror>(vv[4]);
#pragma unroll
        for (int i = 0; i < 8; i += 2) vv[i + 1] = dpp_mov<kDppXor2>(vv[i]);
    } else if constexpr (TR == 4) {
        vv[2] = dpp_mov<kDppRor8>(vv[0]);
        vv[1] = dpp_mov<kDppHalfMirror>(vv[0]);
        vv[3] = dpp_mov<kDppHalfMirror>(vv[2]);
    } else {
        vv[1] = dpp_mov<kDppRor8>(vv[0]);
    }
}

__device__ __forceinline__ unsigned fbits(float x) { return __builtin_bit_cast(unsigned, x); }
__device__ __forceinline__ float bitsf(unsigned x) { return __builtin_bit_cast(float, x); }

// Sum over the four DPP rows of a wave of the column partials q[0 .. TC):
// afterwards q[0 .. TC/4) of a lane in DPP row rho hold the wave's sums for
// columns TC p + col_off(rho) + j.  v_permlane16_swap exchanges the second
// operand of even DPP rows with the first operand of the odd row above it;
// v_permlane32_swap does the same between the two halves of the wave.
template <int TC>
__device__ __forceinline__ void col_sum_rows(float (&q)[TC]) {
    constexpr int H1 = TC / 2, H2 = TC / 4;
#pragma unroll
    for (int j = 0; j < H1; ++j) {
        const auto r = __builtin_amdgcn_permlane16_swap(fbits(q[j]), fbits(q[j + H1]), false, false);
        q[j] = bitsf(r[0]) + bitsf(r[1]);
    }
#pragma unroll
    for (int j = 0; j < H2; ++j) {
        const auto r = __builtin_amdgcn_permlane32_swap(fbits(q[j]), fbits(q[j + H2]), false, false);
        q[j] = bitsf(r[0]) + bitsf(r[1]);
    }
}

__host__ __device__ __forceinline__ int col_off(int TC, int rho) { return (rho & 1) * (TC / 2) + (rho >> 1) * (TC / 4); }

// FP64 sums of lane pairs.  With both operands of a permlane swap equal to
// x, the two results of a lane are its own x and its partner's, in an order
// that depends on the lane's half, so their sum is the pair sum in every
// lane (a + b == b + a: both lanes get the same bits).
template <bool W32>
__device__ __forceinline__ double swap_sum64(double x) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    unsigned l0, l1, h0, h1;
    if constexpr (W32) {
        const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
    } else {
        const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
    }
    return __builtin_bit_cast(double, ((uint64_t)h0 << 32) | l0) + __builtin_bit_cast(double, ((uint64_t)h1 << 32) | l1);
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov64(double x) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// FP64 sum over the whole wave, in every lane: the DPP row by the four
// halving patterns, then the four rows by the two swaps.
__device__ __forceinline__ double wave_sum64(double x) {
    x = x + dpp_mov64<kDppRor8>(x);
    x = x + dpp_mov64<kDppHalfMirror>(x);
    x = x + dpp_mov64<kDppXor2>(x);
    x = x + dpp_mov64<kDppXor1>(x);
    x = swap_sum64<false>(x);
    return swap_sum64<true>(x);
}

// ---- FP64 forms (the FP64 resident kernel)

template <int LEVEL>
__device__ __forceinline__ double level_partner64(double x) {
    if constexpr (LEVEL == 0) return dpp_mov64<kDppRor8>(x);
    else if constexpr (LEVEL == 1) return dpp_mov64<kDppHalfMirror>(x);
    else if constexpr (LEVEL == 2) return dpp_mov64<kDppXor2>(x);
    else return dpp_mov64<kDppXor1>(x);
}

// row_sum for FP64 partials: afterwards acc[0] holds the sum for tile row
// s(p).
template <int TR, int LEVEL = 0>
__device__ __forceinline__ void row_sum64(double (&acc)[TR]) {
    if constexpr (LEVEL < 4) {
        constexpr int H = TR >> (LEVEL + 1);
        if constexpr (H >= 1) {
#pragma unroll
            for (int t = 0; t < H; ++t) acc[t] = acc[t] + level_partner64<LEVEL>(acc[t + H]);
        } else {
            acc[0] = acc[0] + level_partner64<LEVEL>(acc[0]);
        }
        row_sum64<TR, LEVEL + 1>(acc);
    }
}

// row_gather for FP64 values: vv[i] = row TR rb + (i ^ s(p)).
template <int TR>
__device__ __forceinline__ void row_gather64(double x, double (&vv)[TR]) {
    vv[0] = x;
    if constexpr (TR == 8) {
        vv[4] = dpp_mov64<kDppRor8>(vv[0]);
        vv[2] = dpp_mov64<kDppHalfMirror>(vv[0]);
        vv[6] = dpp_mov64<kDppHalfMirror>(vv[4]);
#pragma unroll
        for (int i = 0; i < 8; i += 2) vv[i + 1] = dpp_mov64<kDppXor2>(vv[i]);
    } else if constexpr (TR == 4) {
        vv[2] = dpp_mov64<kDppRor8>(vv[0]);
        vv[1] = dpp_mov64<kDppHalfMirror>(vv[0]);
        vv[3] = dpp_mov64<kDppHalfMirror>(vv[2]);
    } else {
        vv[1] = dpp_mov64<kDppRor8>(vv[0]);
    }
}

__device__ __forceinline__ unsigned lo32(double x) { return (unsigned)__builtin_bit_cast(uint64_t, x); }
__device__ __forceinline__ unsigned hi32(double x) { return (unsigned)(__builtin_bit_cast(uint64_t, x) >> 32); }
__device__ __forceinline__ double mk64(unsigned lo, unsigned hi) {
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// col_sum_rows for FP64 partials (the low and high words of each double
// take the same exchange): afterwards q[0 .. TC/4) of a lane in row rho hold
// the wave's sums for columns TC p + col_off(rho) + j.
template <int TC>
__device__ __forceinline__ void col_sum_rows64(double (&q)[TC]) {
    constexpr int H1 = TC / 2, H2 = TC / 4;
#pragma unroll
    for (int j = 0; j < H1; ++j) {
        const auto rl = __builtin_amdgcn_permlane16_swap(lo32(q[j]), lo32(q[j + H1]), false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap(hi32(q[j]), hi32(q[j + H1]), false, false);
        q[j] = mk64(rl[0], rh[0]) + mk64(rl[1], rh[1]);
    }
#pragma unroll
    for (int j = 0; j < H2; ++j) {
        const auto rl = __builtin_amdgcn_permlane32_swap(lo32(q[j]), lo32(q[j + H2]), false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(hi32(q[j]), hi32(q[j + H2]), false, false);
        q[j] = mk64(rl[0], rh[0]) + mk64(rl[1], rh[1]);
    }
}

// The value of lane i (wave-uniform i) in every lane.
__device__ __forceinline__ double read_lane64(double x, int i) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    return __builtin_bit_cast(double, ((uint64_t)(unsigned)__builtin_amdgcn_readlane((int)(b >> 32), i) << 32) |
                                          (unsigned)__builtin_amdgcn_readlane((int)b, i));
}

}  // namespace lane
}  // namespace rom
