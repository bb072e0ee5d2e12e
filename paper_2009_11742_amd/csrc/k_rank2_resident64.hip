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
#include "k_lane.h"
#include "rom_internal.h"

namespace rom {
namespace {

constexpr int kR64Threads = 256;

using namespace lane;

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
