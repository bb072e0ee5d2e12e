// Rank-2 leapfrog stepper with FP64 states at small K: the operator-resident
// schedule in FP64, for skew operator pairs (Asv = -Avs^T exactly) with
// Kv, Ks <= 128 and for other pairs with Kv_pad Ks_pad <= 8192.
//
// Method: Sec. 2.4 eq. (2.5) for the staggered system of Sec. 3.1 eq. (3.3),
//     V <- V + dt (Avs S + b u(t_n; mu))      then      S <- S + dt Asv V
// (for a skew pair Asv V = -Avs^T V, the energy-conserving structure of
// Sec. 3.1, so one operator serves both half-steps), with the probe QoI
// J += dt (c^T V)^2 on the new V of each step.
//
// At these sizes a step is a few thousand FP64 multiply-adds per sample, so
// every schedule that moves operators or states through memory per step is
// bound by latency.  Here one workgroup of four waves steps one sample and
// keeps its operators (at most 128 KB in FP64) in registers for the whole
// run; nothing but two column partials per wave passes through LDS, and one
// workgroup barrier per step is the only wait.  A non-skew pair holds Asv^T
// in a second tile of the same layout (twice the registers: hence the
// smaller size limit).
//
// Layout.  Thread t holds the TR x TC tile of Avs at row block rb = t / 16
// and column block cb = t % 16 (columns TC cb + j): the 16 lanes of a row
// block are one 16-lane (DPP) row of a wave.  Register i of the tile holds
// row TR rb + (i ^ s(cb)), with s the row order below.
//  * Velocity: each lane sums its TC columns for its TR rows; four halving
//    levels of DPP partner moves over the 16 lanes (p ^ 8, p ^ 7, p ^ 2,
//    p ^ 1) leave each lane the full sum of row TR rb + s(p), which it
//    updates in FP64 (the 16 / TR lanes of a row compute bitwise equal
//    values); the TR new rows of the block come back by DPP moves.
//  * Stress: each lane sums its TR rows for its TC columns (of Avs, negated
//    in the update, or of Asv^T); two permlane swap levels between the
//    wave's 16-lane rows leave each lane a quarter of its columns' wave
//    sums, the four waves meet in LDS (double-buffered
//    by step parity, so the barrier of step n + 1 separates the reads of step
//    n from the writes of step n + 2), and every lane reads the four wave
//    sums of its TC columns and updates its own copy of them: S is held
//    redundantly by the 16 row blocks, bitwise equal (same operands, same
//    order), so it needs no second exchange and no second barrier.
//  * Probe: c^T V of each row block from the gathered rows, summed over the
//    wave by swaps and over the waves in LDS.
//  * Forcing: each wave evaluates u(t_n) for the next 64 steps, one step per
//    lane, and reads the step's value from its lane.
#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

constexpr int kR64Threads = 256;

// DPP controls (gfx9 encoding)
constexpr int kDppRor8 = 0x128;            // row_ror:8        (p ^ 8)
constexpr int kDppHalfMirror = 0x141;      // row_half_mirror  (p ^ 7)
constexpr int kDppXor2 = 0x4E;             // quad_perm [2,3,0,1]
constexpr int kDppXor1 = 0xB1;             // quad_perm [1,0,3,2]

// Every lane of these patterns has a source lane (bound_ctrl, zero "old").
template <int CTRL>
__device__ __forceinline__ double dpp_mov64(double x) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Register order of a lane's tile rows: register i holds tile row i ^ s(p).
// With b3 b2 b1 the bits of p: TR = 8: s = 4 b3 + 2 b2 + (b1 ^ b2); TR = 4:
// s = 2 b3 + b2.  Halving level k's partner changes s by exactly
// TR >> (k + 1) while 2 (TR >> (k + 1)) registers are live, and leaves it
// unchanged at the levels after the halving (which then add equal rows).
__device__ __forceinline__ int row_xor(int TR, int p) {
    const int b3 = (p >> 3) & 1, b2 = (p >> 2) & 1, b1 = (p >> 1) & 1;
    return TR == 8 ? 4 * b3 + 2 * b2 + (b1 ^ b2) : 2 * b3 + b2;
}

template <int LEVEL>
__device__ __forceinline__ double level_partner64(double x) {
    if constexpr (LEVEL == 0) return dpp_mov64<kDppRor8>(x);
    else if constexpr (LEVEL == 1) return dpp_mov64<kDppHalfMirror>(x);
    else if constexpr (LEVEL == 2) return dpp_mov64<kDppXor2>(x);
    else return dpp_mov64<kDppXor1>(x);
}

// Sum over the 16 lanes of the DPP row of the row partials acc[0 .. TR):
// afterwards acc[0] holds the sum for tile row s(p).
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

// The TR rows of a lane's row block in its register order: vv[i] = row
// TR rb + (i ^ s(p)), the value of a lane p' of the same DPP row with
// s(p') = s(p) ^ i; one partner pattern per bit of i (TR = 8: p ^ 8, p ^ 7,
// p ^ 2; TR = 4: p ^ 8, p ^ 7).
template <int TR>
__device__ __forceinline__ void row_gather64(double x, double (&vv)[TR]) {
    vv[0] = x;
    if constexpr (TR == 8) {
        vv[4] = dpp_mov64<kDppRor8>(vv[0]);
        vv[2] = dpp_mov64<kDppHalfMirror>(vv[0]);
        vv[6] = dpp_mov64<kDppHalfMirror>(vv[4]);
#pragma unroll
        for (int i = 0; i < 8; i += 2) vv[i + 1] = dpp_mov64<kDppXor2>(vv[i]);
    } else {
        vv[2] = dpp_mov64<kDppRor8>(vv[0]);
        vv[1] = dpp_mov64<kDppHalfMirror>(vv[0]);
        vv[3] = dpp_mov64<kDppHalfMirror>(vv[2]);
    }
}

__device__ __forceinline__ unsigned lo32(double x) { return (unsigned)__builtin_bit_cast(uint64_t, x); }
__device__ __forceinline__ unsigned hi32(double x) { return (unsigned)(__builtin_bit_cast(uint64_t, x) >> 32); }
__device__ __forceinline__ double mk64(unsigned lo, unsigned hi) {
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the four 16-lane rows of a wave of the column partials q[0 ..
// TC): afterwards q[0 .. TC/4) of a lane in row rho hold the wave's sums for
// columns TC p + col_off(rho) + j.  v_permlane16_swap exchanges the second
// operand of even rows with the first operand of the odd row above it,
// v_permlane32_swap does the same between the two halves of the wave; the
// low and high words of each double take the same exchange.
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

__device__ __forceinline__ int col_off(int TC, int rho) { return (rho & 1) * (TC / 2) + (rho >> 1) * (TC / 4); }

// x + (the value of lane l ^ 16 (W32 false) or l ^ 32 (W32 true)), bitwise
// equal in both lanes.  With both operands of a permlane swap equal to x a
// lane receives its own x and its partner's, in an order that depends on its
// half; a + b == b + a.
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

// The value of lane i (wave-uniform i) in every lane.
__device__ __forceinline__ double read_lane64(double x, int i) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, i);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), i);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <int TR, int TC, bool SKEW>
__global__ __launch_bounds__(kR64Threads) void rank2_resident64_kernel(Rank2Args a) {
    constexpr int KSR = 16 * TC;
    constexpr int QW = TC / 4;                          // wave sums each lane holds
    constexpr int DUP = 16 / TR - 1;                    // lanes of equal s(p) differ in these bits of p
    // per-wave column sums of Avs^T V and probe sums, by step parity
    __shared__ __align__(16) double part[2][4][KSR];
    __shared__ double ypart[2][4];

    const int tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rho = l >> 4, cb = l & 15;
    const int rb = 4 * w + rho;
    const int sx = row_xor(TR, cb);
    const int m = blockIdx.x;
    const int kv = a.kv, ks = a.ks;
    const double dt = a.dt;
    const double *Ag = static_cast<const double *>(a.avs);   // column-major kv x ks
    const double *Bg = static_cast<const double *>(a.asv);   // column-major ks x kv (non-skew pairs)
    double *Vg = static_cast<double *>(a.V) + (size_t)m * kv;
    double *Sg = static_cast<double *>(a.S) + (size_t)m * ks;
    const double *bg = static_cast<const double *>(a.b);
    const double *cg = static_cast<const double *>(a.c);
    const bool probe = cg != nullptr;
    const double mu = a.mu[m];

    // op: the Avs tile; opT: the Asv^T tile of a non-skew pair
    double op[TR][TC], opT[SKEW ? 1 : TR][SKEW ? 1 : TC], cr[TR], s[TC];
#pragma unroll
    for (int i = 0; i < TR; ++i) {
        const int r = TR * rb + (i ^ sx);
        const bool ok = r < kv;
#pragma unroll
        for (int j = 0; j < TC; ++j) {
            const int c = TC * cb + j;
            op[i][j] = (ok && c < ks) ? Ag[(size_t)c * kv + r] : 0.0;
            if constexpr (!SKEW) opT[i][j] = (ok && c < ks) ? Bg[(size_t)r * ks + c] : 0.0;
        }
        cr[i] = (ok && probe) ? cg[r] : 0.0;
    }
    // owned row of V: TR rb + s(p) (16 / TR lanes each, bitwise equal)
    const int rv = TR * rb + sx;
    const bool rok = rv < kv;
    double v = rok ? Vg[rv] : 0.0;
    const double br = rok ? bg[rv] : 0.0;
#pragma unroll
    for (int j = 0; j < TC; ++j) {
        const int c = TC * cb + j;
        s[j] = c < ks ? Sg[c] : 0.0;
    }

    double Jacc = 0.0, uw = 0.0;
    for (int64_t k = 0; k < a.nsteps; ++k) {
        const int kw = (int)(k & 63), par = (int)(k & 1);
        if (kw == 0) uw = dev::forcing(a.source, (double)(a.n0 + k + l) * dt, mu);
        const double u = read_lane64(uw, kw);

        // ---- velocity half-step: V += dt (Avs S + b u)
        double acc[TR];
#pragma unroll
        for (int i = 0; i < TR; ++i) {
            double t = op[i][0] * s[0];
#pragma unroll
            for (int j = 1; j < TC; ++j) t = fma(op[i][j], s[j], t);
            acc[i] = t;
        }
        row_sum64<TR>(acc);
        v = v + dt * (acc[0] + br * u);

        // ---- stress half-step: S += dt Asv V (S -= dt Avs^T V for a skew pair)
        double vv[TR];
        row_gather64<TR>(v, vv);
        double q[TC];
#pragma unroll
        for (int j = 0; j < TC; ++j) {
            const auto &B = [&]() -> const double(&)[TR][TC] {
                if constexpr (SKEW) return op; else return opT;
            }();
            double t = B[0][j] * vv[0];
#pragma unroll
            for (int i = 1; i < TR; ++i) t = fma(B[i][j], vv[i], t);
            q[j] = t;
        }
        col_sum_rows64<TC>(q);
#pragma unroll
        for (int j = 0; j < QW; ++j) part[par][w][TC * cb + col_off(TC, rho) + j] = q[j];
        if (probe) {
            double y = cr[0] * vv[0];
#pragma unroll
            for (int i = 1; i < TR; ++i) y = fma(cr[i], vv[i], y);
            y = swap_sum64<true>(swap_sum64<false>(y));    // lane 0: the row blocks of lanes 0, 16, 32, 48 (s = 0)
            if (l == 0) ypart[par][w] = y;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < TC; ++j) {
            const int c = TC * cb + j;
            const double Q = (part[par][0][c] + part[par][1][c]) + (part[par][2][c] + part[par][3][c]);
            s[j] = SKEW ? s[j] - dt * Q : s[j] + dt * Q;
        }
        if (probe && tid == 0) {
            const double y = (ypart[par][0] + ypart[par][1]) + (ypart[par][2] + ypart[par][3]);
            Jacc += dt * (y * y);
            if (a.y) a.y[(size_t)k * a.M + m] = y;
        }
    }

    if ((cb & DUP) == 0 && rok) Vg[rv] = v;
    if (rb == 0) {
#pragma unroll
        for (int j = 0; j < TC; ++j)
            if (TC * cb + j < ks) Sg[TC * cb + j] = s[j];
    }
    if (probe && a.J && tid == 0) a.J[m] += Jacc;
}

}  // namespace

bool rank2_resident64_applies(int kvp, int ksp, bool skew) {
    return kvp <= 128 && ksp <= 128 && (skew || kvp * ksp <= 8192);
}

// a.avs, a.asv: the context's column-major FP64 Avs and Asv (Asv read for
// non-skew pairs only); a.kvp, a.ksp the sizes padded to 64.
hipError_t launch_rank2_resident64(const Rank2Args &a, bool skew, hipStream_t st) {
    if (!rank2_resident64_applies(a.kvp, a.ksp, skew) || a.kvp % 64 || a.ksp % 64 || a.kvp < 64 || a.ksp < 64)
        return hipErrorInvalidValue;
    const dim3 g(a.M), b(kR64Threads);
    const int shape = (a.kvp == 128) * 2 + (a.ksp == 128);
    if (skew) {
        switch (shape) {
        case 0: hipLaunchKernelGGL((rank2_resident64_kernel<4, 4, true>), g, b, 0, st, a); break;
        case 1: hipLaunchKernelGGL((rank2_resident64_kernel<4, 8, true>), g, b, 0, st, a); break;
        case 2: hipLaunchKernelGGL((rank2_resident64_kernel<8, 4, true>), g, b, 0, st, a); break;
        default: hipLaunchKernelGGL((rank2_resident64_kernel<8, 8, true>), g, b, 0, st, a); break;
        }
    } else {
        switch (shape) {
        case 0: hipLaunchKernelGGL((rank2_resident64_kernel<4, 4, false>), g, b, 0, st, a); break;
        case 1: hipLaunchKernelGGL((rank2_resident64_kernel<4, 8, false>), g, b, 0, st, a); break;
        default: hipLaunchKernelGGL((rank2_resident64_kernel<8, 4, false>), g, b, 0, st, a); break;
        }
    }
    return hipGetLastError();
}

}  // namespace rom
