// Device building blocks of the FP32 column-block steppers (forward rank-2
// and its adjoint): packed-operator x LDS-state tile products on
// v_mfma_f32_4x4x1f32, FP32 chains folded into FP64 tile sums, and the FP64
// tile update of the (hi, lo) state pair.
//
// Cost model (measured on gfx950, one wave per SIMD): a 4x4x1 MFMA issues
// about every 4.6 ns, and VALU, LDS and global-load instructions of the same
// SIMD add their own time rather than hiding under the MFMAs.  The product
// loop is therefore built to issue as few non-MFMA instructions per MFMA as
// possible: one float4 operator load and one float4 state read per 4 MFMAs,
// and 2 VALU ops per chain value folded.
#pragma once

#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace tile {

using dev::f4;
constexpr int NB = kColBlock;     // 4 sample columns per column set
constexpr int kChunk = 32;        // k terms per operator chunk (8 float4 loads)
constexpr int kQ = kChunk / 4;

// Column sets: a workgroup owns NS sets of 4 sample columns (NS = 1 or 2).
// Every operator fragment loaded feeds one MFMA per set, so two sets halve
// the operator bytes each CU fetches per flop (the column-block products
// are bound by the L1 fill of the streamed operator, not by the MFMAs).

// Load the kQ float4 operator fragments of chunk `ch` of a panel tile.
__device__ __forceinline__ void load_chunk(f4 (&dst)[kQ], const f4 *ap, int ch) {
    const f4 *src = ap + (size_t)ch * kQ * 64;
#pragma unroll
    for (int q = 0; q < kQ; ++q) dst[q] = src[q * 64];
}

// Load the kChunk state values of chunk `ch` of the lane's LDS column of
// every set (set s: column j + 4 s, ld apart).
template <int NS>
__device__ __forceinline__ void lds_chunk(f4 (&dst)[NS][kQ], const float *xcol, int ld, int ch) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const f4 *src = reinterpret_cast<const f4 *>(xcol + 4 * s * ld + ch * kChunk);
#pragma unroll
        for (int q = 0; q < kQ; ++q) dst[s][q] = src[q];
    }
}

// Exact fold of an FP32 partial sum into a (hi, lo) pair (two-sum); used by
// the low-precision products.
__device__ __forceinline__ void fold(f4 &hi, f4 &lo, const f4 &acc) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float s, e;
        dev::two_sum(hi[r], acc[r], s, e);
        hi[r] = s;
        lo[r] += e;
    }
}

__device__ __forceinline__ f4 mfma4(float a, float x, f4 c) {
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, x, c, 0, 0, 0);
}

// The FP32 products accumulate in two MFMA chains per set and chunk pair
// (c[s][0]: even float4 groups, c[s][1]: odd ones; 32 terms each), and
// every finished chain is folded into FP64 tile sums with one convert and
// one FP64 add per value.  Each chain rounds like a 32-term sequential FP32
// sum; the FP64 sums add nothing measurable to that.  The MFMAs alternate
// between chains (a dependent 4x4x1 MFMA waits about twice its issue
// interval), and a sched_barrier after every group pins that order, which
// the scheduler would otherwise trade for back-to-back dependent MFMAs.

// First chunk of a pair: start fresh chains and fold the previous pair's
// chains p into acc, one fold step per set between two MFMA groups, from
// the third group on (the previous chains have left the pipeline).
template <int NS>
__device__ __forceinline__ void mma_first(const f4 (&a)[kQ], const f4 (&x)[NS][kQ], f4 (&c)[NS][2],
                                          const f4 (&p)[NS][2], double (&acc)[NS][4]) {
#pragma unroll
    for (int s = 0; s < NS; ++s) c[s][0] = c[s][1] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 16; ++i) {          // group i: component i % 4 of float4s 2 (i / 4), +1
        const int q = 2 * (i >> 2), e = i & 3;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            c[s][0] = mfma4(a[q][e], x[s][q][e], c[s][0]);
            c[s][1] = mfma4(a[q + 1][e], x[s][q + 1][e], c[s][1]);
        }
        if (i >= 2 && i < 10) {
            const int k = i - 2;            // fold step k: element k % 4 of chain k / 4
#pragma unroll
            for (int s = 0; s < NS; ++s) acc[s][k & 3] += (double)p[s][k >> 2][k & 3];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Second chunk of a pair: continue the chains.
template <int NS>
__device__ __forceinline__ void mma_next(const f4 (&a)[kQ], const f4 (&x)[NS][kQ], f4 (&c)[NS][2]) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = 2 * (i >> 2), e = i & 3;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            c[s][0] = mfma4(a[q][e], x[s][q][e], c[s][0]);
            c[s][1] = mfma4(a[q + 1][e], x[s][q + 1][e], c[s][1]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int NS>
__device__ __forceinline__ void fold64(double (&acc)[NS][4], const f4 (&p)[NS][2]) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            acc[s][r] += (double)p[s][0][r];
            acc[s][r] += (double)p[s][1][r];
        }
}

constexpr int kWaves = 4;                 // one wave per SIMD
constexpr int kThreads = kWaves * 64;

// LDS of the states (hi, lo) of nb columns, probe partials and source /
// probe vectors.
__host__ __device__ inline size_t state_lds_bytes(int kvp, int ksp, int nb) {
    return sizeof(float) * (size_t)nb * 2 * ((kvp + 4) + (ksp + 4)) + sizeof(double) * kWaves * nb +
           sizeof(float) * 2 * (size_t)kvp;
}

// Register-resident operator: each wave keeps the first res_pairs(NS)
// chunk pairs of its first row tile of each field in registers for the
// whole run (8 chunks = 256 registers per lane with one set, 4 chunks with
// two, whose state buffers and chains take the rest), so those chunks cost
// no load at all; the rest is streamed.  A field keeps at least one
// streamed pair per tile.
__host__ __device__ constexpr int res_pairs(int ns) { return ns == 1 ? 2 : 1; }

__host__ __device__ inline int resident_pairs(int nch, int ns) {
    const int r = nch / 2 - 1;
    return r < res_pairs(ns) ? r : res_pairs(ns);
}

struct Field {
    const f4 *pk;      // packed operator panel of this half-step
    int T;             // row tiles of the updated field
    int kp;            // padded reduction length
    int nch;           // reduction chunks per tile (kp / kChunk, even)
    int rp;            // resident pairs of the wave's first tile (resident_pairs(nch))
    const float *X;    // LDS: the other field's columns (hi words), ld ldx
    int ldx;
    float *Yh, *Yl;    // LDS: the updated field (hi, lo), ld ldy
    int ldy;
};

// Uniform address of chunk c of row tile t of a packed panel (add the lane
// at the load).
__device__ __forceinline__ const f4 *chunk_ptr(const f4 *pk, int kp, int t, int c) {
    return pk + (size_t)t * kp * 16 + (size_t)c * (kQ * 64);
}

// Per-wave operator stream: the chunks of the wave's tiles in the order the
// wave uses them (V-update tiles, S-update tiles, the next step's V-update
// tiles, ...), consumed in pairs.  The operators do not change during a
// run, so the stream runs ahead across tile and half-step boundaries and
// the workgroup barriers never drain it.  `p` (wave-uniform) addresses the
// next pair to load, (f, t, c) names it.
struct Stream {
    const f4 *p;
    int f, t, c;
};

// Value select (the operands are loaded first).  A conditional on lvalues
// selects addresses instead, which keeps the Field structs out of
// registers and in private memory.
template <class T>
__device__ __forceinline__ T sel(bool c, T a, T b) {
    return c ? a : b;
}

// Branch-free (scalar selects only), so the product loop stays one block.
// A wave with no tile in the other field keeps cycling through its own.
// The resident pairs of the wave's first tile (t == w, reached exactly at a
// field start) are skipped.
__device__ __forceinline__ void advance(Stream &s, const Field &fv, const Field &fs, int w) {
    const bool onS = s.f != 0;
    const int c = s.c + 2, t = s.t + kWaves;
    const bool tile_end = c >= sel(onS, fs.nch, fv.nch);
    const bool field_end = tile_end && t >= sel(onS, fs.T, fv.T);
    const bool other = sel(onS, w < fv.T, w < fs.T);
    const bool nS = (field_end && other) ? !onS : onS;
    s.f = nS ? 1 : 0;
    s.t = field_end ? w : (tile_end ? t : s.t);
    s.c = field_end ? 2 * sel(nS, fs.rp, fv.rp) : (tile_end ? 0 : c);
    s.p = chunk_ptr(sel(nS, fs.pk, fv.pk), sel(nS, fs.kp, fv.kp), s.t, s.c);
}

// Point the stream at wave w's first pair and load it into (a0, a1).  A
// wave with no tile leaves them untouched.
__device__ __forceinline__ void stream_start(Stream &s, f4 (&a0)[kQ], f4 (&a1)[kQ], const Field &fv,
                                             const Field &fs, int w, int lane) {
    const bool sv = w < fv.T, ss = w < fs.T;
    s.f = sv ? 0 : 1;
    s.t = w;
    s.c = 2 * sel(sv, fv.rp, fs.rp);
    s.p = chunk_ptr(sel(sv, fv.pk, fs.pk), sel(sv, fv.kp, fs.kp), s.t, s.c);
    if (!sv && !ss) return;
    // keep every a0 load ahead of every a1 load, as in the product loop, so
    // the waits there can count on that order on every path
    __builtin_amdgcn_sched_barrier(0);
    load_chunk(a0, s.p + lane, 0);
    __builtin_amdgcn_sched_barrier(0);
    load_chunk(a1, s.p + lane, 1);
    __builtin_amdgcn_sched_barrier(0);
    advance(s, fv, fs, w);
}

// Load the resident pairs of field F (wave w's first tile) into res.
template <int NS>
__device__ __forceinline__ void load_resident(f4 (&res)[2 * res_pairs(NS)][kQ], const Field &F, int w,
                                              int lane) {
    if (w >= F.T) return;
    const f4 *ap = chunk_ptr(F.pk, F.kp, w, 0) + lane;
#pragma unroll
    for (int c = 0; c < 2 * res_pairs(NS); ++c)
        if (c < 2 * F.rp) load_chunk(res[c], ap, c);
}

// 64 x 4 NS tile product  P[t] * X  of field F (X: this lane's LDS column
// xcol of set 0; set s is 4 s columns further), summed in FP64 into acc.
// The first nres chunk pairs come from the registers `res`, the rest from
// the stream, whose current pair sits in (a0, a1); each pair used is
// replaced by the stream's next one.  State values are fetched one chunk
// ahead with ping-pong buffers.  Per lane acc[s][r] is row
// 64 t + 4 (lane / 4) + r of column 4 s + lane % 4.
template <int NS>
__device__ __forceinline__ void tile_product(const Field &F, const float *xcol,
                                             const f4 (&res)[2 * res_pairs(NS)][kQ], int nres,
                                             f4 (&a0)[kQ], f4 (&a1)[kQ], Stream &s, const Field &fv,
                                             const Field &fs, int w, int lane, double (&acc)[NS][4]) {
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[q][r] = 0.0;
    f4 p[NS][2];
#pragma unroll
    for (int q = 0; q < NS; ++q) p[q][0] = p[q][1] = f4{0.f, 0.f, 0.f, 0.f};
    f4 x0[NS][kQ], x1[NS][kQ];
    // sched_barrier(0) keeps each prefetch batch where it is written: the
    // scheduler would otherwise sink the loads next to their first use.
    lds_chunk<NS>(x0, xcol, F.ldx, 0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int rp = 0; rp < res_pairs(NS); ++rp) {
        if (rp < nres) {
            lds_chunk<NS>(x1, xcol, F.ldx, 2 * rp + 1);
            __builtin_amdgcn_sched_barrier(0);
            f4 c[NS][2];
            mma_first<NS>(res[2 * rp], x0, c, p, acc);
            __builtin_amdgcn_sched_barrier(0);
            lds_chunk<NS>(x0, xcol, F.ldx, 2 * rp + 2);     // a streamed pair always follows
            __builtin_amdgcn_sched_barrier(0);
            mma_next<NS>(res[2 * rp + 1], x1, c);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < NS; ++q) p[q][0] = c[q][0], p[q][1] = c[q][1];
        }
    }
    for (int ch = 2 * nres; ch < F.nch; ch += 2) {
        lds_chunk<NS>(x1, xcol, F.ldx, ch + 1);
        __builtin_amdgcn_sched_barrier(0);
        f4 c[NS][2];
        mma_first<NS>(a0, x0, c, p, acc);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk(a0, s.p + lane, 0);
        lds_chunk<NS>(x0, xcol, F.ldx, min(ch + 2, F.nch - 1));
        __builtin_amdgcn_sched_barrier(0);
        mma_next<NS>(a1, x1, c);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk(a1, s.p + lane, 1);
        __builtin_amdgcn_sched_barrier(0);
        advance(s, fv, fs, w);
#pragma unroll
        for (int q = 0; q < NS; ++q) p[q][0] = c[q][0], p[q][1] = c[q][1];
    }
    fold64<NS>(acc, p);
}

// Finish one 64 x 4 NS tile in FP64: y = (Yh + Yl) + dt (acc + b u), stored
// back as the (hi, lo) pair.  With FORCED the rows also accumulate the
// probe partials c^T V of each set (u[s]: the forcing of the lane's column
// of set s).
template <bool FORCED, int NS>
__device__ __forceinline__ void finish_tile(const Field &f, int t, const double (&acc)[NS][4], int lane,
                                            const float *bl, const float *cl, const double (&u)[NS],
                                            double dt, double (&ypart)[NS]) {
    const int j = lane & 3;
    const int i0 = t * kTileRows + 4 * (lane >> 2);
    f4 bb = {0.f, 0.f, 0.f, 0.f}, cc = {0.f, 0.f, 0.f, 0.f};
    if (FORCED) {
        bb = *(const f4 *)(bl + i0);
        cc = *(const f4 *)(cl + i0);
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        float *yhp = f.Yh + (j + 4 * q) * f.ldy + i0;
        float *ylp = f.Yl + (j + 4 * q) * f.ldy + i0;
        f4 yh = *(f4 *)yhp;
        f4 yl = *(f4 *)ylp;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double inc = acc[q][r];
            if (FORCED) inc = fma((double)bb[r], u[q], inc);
            const double y = fma(dt, inc, (double)yh[r] + (double)yl[r]);
            const float h = (float)y;
            yh[r] = h;
            yl[r] = (float)(y - (double)h);
            if (FORCED) ypart[q] += (double)cc[r] * y;
        }
        *(f4 *)yhp = yh;
        *(f4 *)ylp = yl;
    }
}

}  // namespace tile
}  // namespace rom
