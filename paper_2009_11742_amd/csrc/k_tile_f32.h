// Device building blocks of the FP32 column-block steppers (forward rank-2
// and its adjoint): packed-operator x LDS-state tile products on
// v_mfma_f32_4x4x1f32 with compensated accumulation, and the double-float
// tile update.
#pragma once

#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace tile {

using dev::f4;
constexpr int NB = kColBlock;     // 4 sample columns per workgroup
constexpr int kChunk = 32;        // k terms per compensated chunk (8 float4 loads)
constexpr int kQ = kChunk / 4;

// Load the kQ float4 operator fragments of chunk `ch` of a panel tile.
__device__ __forceinline__ void load_chunk(f4 (&dst)[kQ], const f4 *ap, int ch) {
    const f4 *src = ap + (size_t)ch * kQ * 64;
#pragma unroll
    for (int q = 0; q < kQ; ++q) dst[q] = src[q * 64];
}

// Load the kChunk state values of chunk `ch` of this lane's LDS column.
__device__ __forceinline__ void lds_chunk(f4 (&dst)[kQ], const float *xcol, int ch) {
    const f4 *src = reinterpret_cast<const f4 *>(xcol + ch * kChunk);
#pragma unroll
    for (int q = 0; q < kQ; ++q) dst[q] = src[q];
}

__device__ __forceinline__ void fold(f4 &hi, f4 &lo, const f4 &acc) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float s, e;
        dev::two_sum(hi[r], acc[r], s, e);
        hi[r] = s;
        lo[r] += e;
    }
}

// Product of one chunk, as two independent MFMA chains (even and odd
// float4 groups) so consecutive MFMAs never wait on each other's result;
// each chain's partial sum (16 terms) is folded into (hi, lo) exactly.
__device__ __forceinline__ void mma_chunk(const f4 (&a)[kQ], const f4 (&x)[kQ], f4 &hi, f4 &lo) {
    f4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < kQ; q += 2) {
        c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(a[q].x, x[q].x, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(a[q + 1].x, x[q + 1].x, c1, 0, 0, 0);
        c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(a[q].y, x[q].y, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(a[q + 1].y, x[q + 1].y, c1, 0, 0, 0);
        c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(a[q].z, x[q].z, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(a[q + 1].z, x[q + 1].z, c1, 0, 0, 0);
        c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(a[q].w, x[q].w, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(a[q + 1].w, x[q + 1].w, c1, 0, 0, 0);
    }
    fold(hi, lo, c0);
    fold(hi, lo, c1);
}

// Compensated 64 x 4 tile of  P[t] * X  where P is a packed operator panel
// (pk[t][k/4][lane][k%4] = P[64 t + lane][k]) and X the 4 LDS-resident
// columns (this lane's column at xcol).  Returns per lane the rows
// 64 t + 4 (lane / 4) + r, r = 0..3, of column lane % 4 as (H, L).
// Only chunks [cb, ce) of the reduction are summed (an even count).
// Operator fragments (from L2) and state values (from LDS) are both fetched
// one chunk ahead of use with branch-free ping-pong buffers, so every wait
// covers an access issued a full chunk earlier.
__device__ __forceinline__ void tile_product(const f4 *__restrict__ pk, int t, int kp, int cb,
                                             int ce, const float *xcol, int lane, f4 &H, f4 &L) {
    const f4 *ap = pk + (size_t)t * (size_t)(kp / 4) * 64 + lane + (size_t)cb * kQ * 64;
    xcol += cb * kChunk;
    f4 hi = {0.f, 0.f, 0.f, 0.f}, lo = {0.f, 0.f, 0.f, 0.f};
    const int nch = ce - cb;
    f4 a0[kQ], a1[kQ], x0[kQ], x1[kQ];
    // sched_barrier(0) keeps each prefetch batch where it is written: the
    // scheduler would otherwise sink the loads next to their first use.
    load_chunk(a0, ap, 0);
    load_chunk(a1, ap, 1);
    lds_chunk(x0, xcol, 0);
    __builtin_amdgcn_sched_barrier(0);
    for (int ch = 0; ch < nch; ch += 2) {
        lds_chunk(x1, xcol, ch + 1);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk(a0, x0, hi, lo);
        __builtin_amdgcn_sched_barrier(0);
        // refill with chunk ch+2 (or re-read the last chunk: in bounds, unused)
        const int n2 = min(ch + 2, nch - 1);
        load_chunk(a0, ap, n2);
        lds_chunk(x0, xcol, n2);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk(a1, x1, hi, lo);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk(a1, ap, min(ch + 3, nch - 1));
        __builtin_amdgcn_sched_barrier(0);
    }
    H = hi;
    L = lo;
}

constexpr int kWaves = 4;                 // one wave per SIMD
constexpr int kThreads = kWaves * 64;

struct Field {
    const f4 *pk;      // packed operator panel of this half-step
    int T;             // row tiles of the updated field
    int kp;            // padded reduction length
    const float *X;    // LDS: the other field's columns (hi words), ld ldx
    int ldx;
    float *Yh, *Yl;    // LDS: the updated field (hi, lo), ld ldy
    int ldy;
};

// Finish one 64 x 4 tile: (Yh, Yl) += dt * ((H + L) + forcing).  With
// FORCED the rows also accumulate the probe partial c^T V.
template <bool FORCED>
__device__ __forceinline__ void finish_tile(const Field &f, int t, f4 H, f4 L, int lane,
                                            const float *bl, const float *cl, float uh, float ul,
                                            float dtf, double &ypart) {
    const int j = lane & 3;
    const int i0 = t * kTileRows + 4 * (lane >> 2);
    f4 yh = *(f4 *)(f.Yh + j * f.ldy + i0);
    f4 yl = *(f4 *)(f.Yl + j * f.ldy + i0);
    f4 bb = {0.f, 0.f, 0.f, 0.f}, cc = {0.f, 0.f, 0.f, 0.f};
    if (FORCED) {
        bb = *(const f4 *)(bl + i0);
        cc = *(const f4 *)(cl + i0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float F = 0.f, Fe = 0.f;
        if (FORCED) {
            F = bb[r] * uh;
            Fe = fmaf(bb[r], uh, -F) + bb[r] * ul;
        }
        float h = yh[r], l = yl[r];
        dev::comp_update(h, l, H[r], L[r], F, Fe, dtf);
        yh[r] = h;
        yl[r] = l;
        if (FORCED) ypart += (double)cc[r] * ((double)h + (double)l);
    }
    *(f4 *)(f.Yh + j * f.ldy + i0) = yh;
    *(f4 *)(f.Yl + j * f.ldy + i0) = yl;
}

}  // namespace tile
}  // namespace rom
