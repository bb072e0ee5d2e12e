// Rank-2 leapfrog stepper for skew operator pairs (Asv = -Avs^T exactly),
// FP32 operators and states: the operator-resident schedule.
//
// Method: Sec. 2.4 eq. (2.5) for the staggered system of Sec. 3.1 eq. (3.3),
//     V <- V + dt (Avs S + b u(t_n; mu)^T)      then      S <- S + dt Asv V,
// where for a skew pair the stress half-step is S <- S - dt Avs^T V: both
// half-steps use the one matrix Avs (the energy-conserving structure of the
// staggered operators, Sec. 3.1).
//
// Why this schedule.  A skew pair with Kv, Ks <= 256 is at most 256 KB of
// FP32, half of one CU's register file.  Each workgroup (8 waves, a whole
// CU) keeps all of Avs in registers for the whole run and steps ONE sample:
// no operator byte moves after the start and no workgroup ever waits for
// another, so M samples occupy M CUs.  (The column-block kernels give a CU
// four samples and stream the operator through it every step, so M = 256
// samples fill only 64 CUs; the row-split kernels exchange states between
// CUs every half-step.)  One sample's products are matrix-vector products,
// which the matrix cores would run at a quarter of their rate (one useful
// column of the narrowest FP32 MFMA), so they run as FP32 FMAs on the vector
// ALUs, at half the FP32 MFMA peak.
//
// Lane layout.  Lane L = 64 w + l (wave w, lane l, DPP row rho = l / 16,
// position p = l % 16) holds the TR x TC tile of Avs at row block
// rb = 4 w + rho (rows TR rb ..) and column block p (columns TC p ..);
// TR in {2, 4, 8}, TC in {4, 8, 12, 16}, so 32 TR >= Kv and 16 TC >= Ks
// (zero padded).  The 16 lanes of a DPP row hold one row block across all
// column blocks, the 32 row blocks of one column block are spread over the
// four DPP rows of every wave.
//  * Velocity half-step: each lane sums its TC columns for its TR rows; the
//    16 lanes of the DPP row combine by recursive halving with the DPP
//    patterns row_ror:8, row_half_mirror, quad_perm xor 2 and xor 1 (lane
//    pairs p ^ 8, p ^ 7, p ^ 2, p ^ 1).  A lane stores its tile rows in the
//    register order i -> tile row i ^ s(p) (row_xor), chosen so that every
//    halving step keeps registers 0 .. H-1 in every lane and adds the
//    partner's H .. 2H-1, which then hold the same rows: no selects.  The
//    sum of tile row s(p) ends in the 16 / TR lanes of equal s(p), which all
//    update that row of V identically (a + b == b + a); one writes it out.
//    The stress half-step multiplies the TR new V rows of the lane's own row
//    block, all held in its DPP row: three more DPP patterns gather them into
//    every lane, so V need not pass through LDS (two workgroup barriers per
//    step, both for S; the largest tile keeps the LDS path, which measures
//    faster there).
//  * Stress half-step: each lane sums its TR rows for its TC columns; the
//    four DPP rows of a wave combine with v_permlane16_swap and
//    v_permlane32_swap (each lane keeps a quarter of its columns), the eight
//    waves through LDS, where two lanes per column add four wave partials
//    each in FP64 and meet with one more swap.
// States: the FP32 (hi, lo) pair of each row of V and column of S stays in
// its owners' registers and is updated in FP64; only the hi words of S pass
// through LDS to the lanes that multiply them.  The forcing u(t_n) of the
// next 64 steps is evaluated once per wave, one step per lane.
#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

using dev::f4;

constexpr int kWavesR = 8;                 // waves per workgroup
constexpr int kThreadsR = 64 * kWavesR;    // threads per workgroup

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

// LDS position of state entry k of a field held in column blocks of TC:
// blocks padded to TC + 4 floats, so the 16 column blocks read by one wave
// instruction fall on different banks.
template <int TC>
__device__ __forceinline__ int spos(int k) { return (k / TC) * (TC + 4) + k % TC; }

template <int TR, int TC>
__global__ __launch_bounds__(kThreadsR) __attribute__((amdgpu_waves_per_eu(2, 2)))
void rank2_resident_kernel(Rank2Args a) {
    constexpr int KVR = 32 * TR, KSR = 16 * TC;
    constexpr int DUP = 16 / TR - 1;                   // lanes of equal s(p) differ in these bits of p
    // V gather for the stress half-step: in-row DPP moves and no workgroup
    // barrier, except for the 8 x 16 tile (K = 256), which runs faster with
    // the V rows through LDS behind a barrier (measured, M = 256, us per
    // step: K = 64 0.60 -> 0.51, K = 128 0.79 -> 0.71, K = 192 1.16 -> 1.10;
    // K = 256 1.28 with LDS and barrier, 1.35 with DPP moves or LDS without
    // the barrier, 1.40 with both DPP moves and the barrier)
    constexpr bool kDppGather = TC < 16;
    __shared__ __align__(16) float Ss[16 * (TC + 4)];  // S hi words, padded column blocks
    __shared__ __align__(16) float Vs[kDppGather ? 1 : KVR];   // V hi words (LDS gather)
    __shared__ __align__(16) float part[kWavesR][KSR]; // per-wave column partials of Avs^T V
    __shared__ double yrow[KVR];                       // probe terms c_r V_r of the step

    const int tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rho = l >> 4, p = l & 15;
    const int rb = 4 * w + rho;
    const int sx = row_xor(TR, p);
    const int m = blockIdx.x;
    const int kv = a.kv, ks = a.ks;
    const double dt = a.dt;
    float *Vg = static_cast<float *>(a.V);
    float *Sg = static_cast<float *>(a.S);
    const float *bg = static_cast<const float *>(a.b);
    const float *cg = static_cast<const float *>(a.c);
    const bool probe = cg != nullptr;

    // ---- operator tile, registers for the whole run: pack[q][tid] (float4),
    // q over the tile's TR x TC entries in (register row, column) order
    float op[TR][TC];
    {
        const f4 *pk = static_cast<const f4 *>(a.avs) + tid;
#pragma unroll
        for (int q = 0; q < TR * TC / 4; ++q) {
            const f4 v = pk[(size_t)q * kThreadsR];
#pragma unroll
            for (int e = 0; e < 4; ++e) op[(4 * q + e) / TC][(4 * q + e) % TC] = v[e];
        }
    }

    // ---- owned state: row rv of V (all lanes), column ko of S (two lanes
    // per column: l and l ^ 32 of wave w own column 32 w + l % 32)
    const int rv = TR * rb + sx;
    const bool vwriter = (p & DUP) == 0;
    const bool rok = rv < kv;
    float vh = rok ? Vg[(size_t)m * kv + rv] : 0.f, vl = 0.f;
    const double br = rok ? (double)bg[rv] : 0.0;
    const double cr = (probe && rok) ? (double)cg[rv] : 0.0;
    const int ko = 32 * w + (l & 31), kh = l >> 5;     // column, half of the wave partials summed
    const bool sown = ko < KSR;
    const bool kok = ko < ks;
    float sh = kok ? Sg[(size_t)m * ks + ko] : 0.f, sl = 0.f;
    if (sown && kh == 0) Ss[spos<TC>(ko)] = sh;
    const double mu = a.mu[m];
    __syncthreads();

    double utab = 0.0, Jacc = 0.0;
    for (int64_t k = 0; k < a.nsteps; ++k) {
        if ((k & 63) == 0) utab = dev::forcing(a.source, (double)(a.n0 + k + l) * dt, mu);
        const int ul = (int)(k & 63);
        const uint64_t ub = __builtin_bit_cast(uint64_t, utab);
        const double u = __builtin_bit_cast(
            double, ((uint64_t)(unsigned)__builtin_amdgcn_readlane((int)(ub >> 32), ul) << 32) |
                        (unsigned)__builtin_amdgcn_readlane((int)ub, ul));

        // ---- velocity half-step: row sums of Avs S
        float acc[TR];
        {
            float sv[TC];
            const float *sp = Ss + p * (TC + 4);
#pragma unroll
            for (int q = 0; q < TC / 4; ++q) {
                const f4 v = *reinterpret_cast<const f4 *>(sp + 4 * q);
#pragma unroll
                for (int e = 0; e < 4; ++e) sv[4 * q + e] = v[e];
            }
#pragma unroll
            for (int i = 0; i < TR; ++i) {
                float s = op[i][0] * sv[0];
#pragma unroll
                for (int j = 1; j < TC; ++j) s = fmaf(op[i][j], sv[j], s);
                acc[i] = s;
            }
        }
        row_sum<TR>(acc);
        {
            const double inc = fma(br, u, (double)acc[0]);
            const double yv = fma(dt, inc, (double)vh + (double)vl);
            vh = (float)yv;
            vl = (float)(yv - (double)vh);
            if (vwriter) {
                if constexpr (!kDppGather) Vs[rv] = vh;
                if (probe) yrow[rv] = cr * yv;
            }
        }

        if constexpr (!kDppGather) __syncthreads();

        // ---- stress half-step: column sums of Avs^T V, S -= dt (Avs^T V).
        // The V rows a lane multiplies are those of its own row block, all
        // updated within its DPP row.
        float q[TC];
        {
            float vv[TR];
            if constexpr (kDppGather) {
                row_gather<TR>(vh, vv);
            } else {
#pragma unroll
                for (int i = 0; i < TR; ++i) vv[i] = Vs[TR * rb + (i ^ sx)];
            }
#pragma unroll
            for (int j = 0; j < TC; ++j) {
                float s = op[0][j] * vv[0];
#pragma unroll
                for (int i = 1; i < TR; ++i) s = fmaf(op[i][j], vv[i], s);
                q[j] = s;
            }
        }
        col_sum_rows<TC>(q);
        {
            float *dst = &part[w][TC * p + col_off(TC, rho)];
#pragma unroll
            for (int j = 0; j < TC / 4; ++j) dst[j] = q[j];
        }
        __syncthreads();
        if (probe && w == 0) {
            // one wave sums the probe terms (the other waves' VALUs stay on
            // the products): lane l adds rows l, l + 64, .. then the wave tree
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < KVR / 64; ++i) t += yrow[l + 64 * i];
            const double yv = wave_sum64(t);
            if (l == 0) {
                Jacc = fma(dt, yv * yv, Jacc);
                if (a.y) a.y[(size_t)k * a.M + m] = yv;
            }
        }
        if (sown) {
            double Q = (double)part[4 * kh][ko];
#pragma unroll
            for (int v = 1; v < 4; ++v) Q += (double)part[4 * kh + v][ko];
            Q = swap_sum64<true>(Q);
            const double yv = fma(dt, -Q, (double)sh + (double)sl);
            sh = (float)yv;
            sl = (float)(yv - (double)sh);
            if (kh == 0) Ss[spos<TC>(ko)] = sh;
        }
        __syncthreads();
    }

    if (vwriter && rok) Vg[(size_t)m * kv + rv] = vh + vl;
    if (sown && kh == 0 && kok) Sg[(size_t)m * ks + ko] = sh + sl;
    if (probe && a.J && tid == 0) a.J[m] += Jacc;
}

// Resident pack of a column-major FP32 Avs (kv x ks): pk[q][t] (float4) for
// thread t of the workgroup, entries 4 q .. 4 q + 3 of its tile in
// (register row i, column j) order: Avs[TR rb + (i ^ s(p))][TC p + j].
__global__ void resident_pack_kernel(const float *__restrict__ A, int kv, int ks, int TR, int TC, f4 *__restrict__ pk) {
    const int nq = TR * TC / 4;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nq * kThreadsR; idx += gridDim.x * blockDim.x) {
        const int q = idx / kThreadsR, t = idx % kThreadsR;
        const int w = t >> 6, l = t & 63, rho = l >> 4, p = l & 15;
        const int rb = 4 * w + rho, s = row_xor(TR, p);
        f4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int flat = 4 * q + e, i = flat / TC, j = flat % TC;
            const int r = TR * rb + (i ^ s), c = TC * p + j;
            v[e] = (r < kv && c < ks) ? A[r + (size_t)c * kv] : 0.f;
        }
        pk[(size_t)q * kThreadsR + t] = v;
    }
}

// Tile shape of padded sizes: TR = kvp / 32 rounded up to a power of two
// (2, 4, 8), TC = ksp / 16; 0 if the schedule does not apply.
void resident_shape(int kvp, int ksp, int &TR, int &TC) {
    TR = TC = 0;
    if (kvp < 64 || kvp > 256 || ksp < 64 || ksp > 256 || kvp % 64 || ksp % 64) return;
    TR = kvp <= 64 ? 2 : (kvp <= 128 ? 4 : 8);
    TC = ksp / 16;
}

template <int TR>
hipError_t launch_tr(const Rank2Args &a, int TC, hipStream_t st) {
    switch (TC) {
    case 4: hipLaunchKernelGGL((rank2_resident_kernel<TR, 4>), dim3(a.M), dim3(kThreadsR), 0, st, a); break;
    case 8: hipLaunchKernelGGL((rank2_resident_kernel<TR, 8>), dim3(a.M), dim3(kThreadsR), 0, st, a); break;
    case 12: hipLaunchKernelGGL((rank2_resident_kernel<TR, 12>), dim3(a.M), dim3(kThreadsR), 0, st, a); break;
    case 16: hipLaunchKernelGGL((rank2_resident_kernel<TR, 16>), dim3(a.M), dim3(kThreadsR), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool rank2_resident_applies(int kvp, int ksp) {
    int TR, TC;
    resident_shape(kvp, ksp, TR, TC);
    return TR > 0;
}

size_t rank2_resident_pack_bytes(int kvp, int ksp) {
    int TR, TC;
    resident_shape(kvp, ksp, TR, TC);
    return (size_t)TR * TC * kThreadsR * sizeof(float);
}

hipError_t launch_resident_pack(const float *A, int kv, int ks, int kvp, int ksp, void *pk, hipStream_t st) {
    int TR, TC;
    resident_shape(kvp, ksp, TR, TC);
    if (TR == 0) return hipErrorInvalidValue;
    const int total = TR * TC / 4 * kThreadsR;
    hipLaunchKernelGGL(resident_pack_kernel, dim3((total + 255) / 256), dim3(256), 0, st, A, kv, ks, TR, TC,
                       static_cast<f4 *>(pk));
    return hipGetLastError();
}

hipError_t launch_rank2_resident(const Rank2Args &a, hipStream_t st) {
    int TR, TC;
    resident_shape(a.kvp, a.ksp, TR, TC);
    if (TR == 8) return launch_tr<8>(a, TC, st);
    if (TR == 4) return launch_tr<4>(a, TC, st);
    if (TR == 2) return launch_tr<2>(a, TC, st);
    return hipErrorInvalidValue;
}

}  // namespace rom
