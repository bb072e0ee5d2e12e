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
#include "k_lane.h"
#include "rom_internal.h"

namespace rom {
namespace {

using dev::f4;
using namespace lane;

constexpr int kWavesR = 8;                 // waves per workgroup
constexpr int kThreadsR = 64 * kWavesR;    // threads per workgroup

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
        const double u = read_lane64(utab, ul);

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
