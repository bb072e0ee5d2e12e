// Rank-2 leapfrog stepper, FP32 operators and states, MFMA products.
//
// Method: Sec. 2.4 eq. (2.5) for the staggered system of Sec. 3.1 eq. (3.3);
// one step is
//     V <- V + dt (Avs S + b u(t_n; mu)^T)      then      S <- S + dt Asv V .
//
// Decomposition (MI355X): the sample columns are independent, so each
// workgroup owns kColBlock (4) columns for the WHOLE run and never talks to
// another workgroup: no grid or group barrier is needed (a cross-workgroup
// barrier costs about 1 us on this part, more than the products of one
// half-step).  The workgroup keeps its V and S columns, plus a compensation
// word per entry, resident in LDS; every half-step it streams the packed
// operator panels from L2 (the operators stay L2 resident across steps) and
// multiplies them with v_mfma_f32_4x4x1f32, whose 16 blocks cover a 64-row
// tile x 4 columns per instruction (lane l holds operator row l of the tile,
// the B operand is the state column l % 4 broadcast from LDS).
//
// Accuracy: MFMA FP32 rounds like sequential FP32 addition, which over 10^4
// steps at K = 256 drifts above 1e-5 relative.  Each wave therefore sums the
// reduction in chunks of kChunk terms into a fresh accumulator and folds
// every chunk into a (hi, lo) pair with an error-free two-sum; the state
// update itself is done in double-float (hi + lo) arithmetic.
#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

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

// One half-step of one field: wave w owns row tiles w, w + 4, ...  Ends
// with a barrier (the other half-step reads every row of this field).
template <bool FORCED>
__device__ __forceinline__ void half_step(const Field &f, int lane, int w, const float *bl,
                                          const float *cl, float uh, float ul, float dtf,
                                          double &ypart) {
    const int j = lane & 3;
    for (int t = w; t < f.T; t += kWaves) {
        f4 H, L;
        tile_product(f.pk, t, f.kp, 0, f.kp / kChunk, f.X + j * f.ldx, lane, H, L);
        finish_tile<FORCED>(f, t, H, L, lane, bl, cl, uh, ul, dtf, ypart);
    }
    __syncthreads();
}

// One workgroup per CU, one wave per SIMD: the compiler may use the whole
// register file for the prefetch buffers instead of trading them for
// occupancy.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void rank2_f32_mfma_kernel(Rank2Args a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int kvp = a.kvp, ksp = a.ksp;
    const int ldv = kvp + 4, lds_ = ksp + 4;     // +4 floats: spread columns over banks
    float *Vh = reinterpret_cast<float *>(smem);
    float *Vl = Vh + NB * ldv;
    float *Sh = Vl + NB * ldv;
    float *Sl = Sh + NB * lds_;
    double *yp = reinterpret_cast<double *>(Sl + NB * lds_);   // [kWaves][NB]
    float *bl = reinterpret_cast<float *>(yp + kWaves * NB);    // source, kvp
    float *cl = bl + kvp;                                         // probe, kvp (0 if none)

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int col0 = blockIdx.x * NB;
    const float *Vin = static_cast<const float *>(a.V);
    const float *Sin = static_cast<const float *>(a.S);
    const float *bv = static_cast<const float *>(a.b);
    const float *cv = static_cast<const float *>(a.c);

    for (int idx = tid; idx < NB * kvp; idx += kThreads) {
        int jj = idx / kvp, i = idx - jj * kvp, mm = col0 + jj;
        Vh[jj * ldv + i] = (mm < a.M && i < a.kv) ? Vin[(size_t)mm * a.kv + i] : 0.f;
        Vl[jj * ldv + i] = 0.f;
    }
    for (int idx = tid; idx < NB * ksp; idx += kThreads) {
        int jj = idx / ksp, i = idx - jj * ksp, mm = col0 + jj;
        Sh[jj * lds_ + i] = (mm < a.M && i < a.ks) ? Sin[(size_t)mm * a.ks + i] : 0.f;
        Sl[jj * lds_ + i] = 0.f;
    }
    for (int i = tid; i < kvp; i += kThreads) {
        bl[i] = bv[i];
        cl[i] = (cv != nullptr && i < a.kv) ? cv[i] : 0.f;
    }

    const int j = lane & 3;            // column of this lane in the MFMA output
    const int m = col0 + j;
    const bool mok = m < a.M;
    const double muj = mok ? a.mu[m] : 1.0;
    const float dtf = (float)a.dt;
    const bool probe = cv != nullptr;
    double Jacc = 0.0;
    const Field fv = {static_cast<const f4 *>(a.avs), kvp / kTileRows, ksp, Sh, lds_, Vh, Vl, ldv};
    const Field fs = {static_cast<const f4 *>(a.asv), ksp / kTileRows, kvp, Vh, ldv, Sh, Sl, lds_};
    __syncthreads();

    for (int64_t k = 0; k < a.nsteps; ++k) {
        const double t = (double)(a.n0 + k) * a.dt;
        const double u64 = mok ? dev::ricker(t, muj) : 0.0;
        const float uh = (float)u64;
        const float ul = (float)(u64 - (double)uh);

        // ---- velocity half-step: V += dt (Avs S + b u^T)
        double ypart = 0.0;
        half_step<true>(fv, lane, w, bl, cl, uh, ul, dtf, ypart);
        if (probe) {
            // sum over the 16 lanes that share column j (lane bits 2..5)
            for (int off = 4; off < 64; off <<= 1) ypart += __shfl_xor(ypart, off, 64);
            if (lane < NB) yp[w * NB + lane] = ypart;
        }
        // ---- stress half-step: S += dt Asv V   (its barrier also publishes
        // yp before it is read below)
        double dummy = 0.0;
        half_step<false>(fs, lane, w, bl, cl, 0.f, 0.f, dtf, dummy);
        if (probe && tid < NB) {
            double yv = 0.0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) yv += yp[q * NB + tid];
            Jacc += a.dt * (yv * yv);
            if (a.y && col0 + tid < a.M) a.y[(size_t)k * a.M + col0 + tid] = yv;
        }
    }

    float *Vout = static_cast<float *>(a.V);
    float *Sout = static_cast<float *>(a.S);
    for (int idx = tid; idx < NB * kvp; idx += kThreads) {
        int jj = idx / kvp, i = idx - jj * kvp, mm = col0 + jj;
        if (mm < a.M && i < a.kv) Vout[(size_t)mm * a.kv + i] = Vh[jj * ldv + i] + Vl[jj * ldv + i];
    }
    for (int idx = tid; idx < NB * ksp; idx += kThreads) {
        int jj = idx / ksp, i = idx - jj * ksp, mm = col0 + jj;
        if (mm < a.M && i < a.ks) Sout[(size_t)mm * a.ks + i] = Sh[jj * lds_ + i] + Sl[jj * lds_ + i];
    }
    if (probe && a.J && tid < NB && col0 + tid < a.M) a.J[col0 + tid] += Jacc;
}

}  // namespace

size_t rank2_f32_mfma_lds_bytes(int kvp, int ksp) {
    return sizeof(float) * (size_t)NB * 2 * ((kvp + 4) + (ksp + 4)) + sizeof(double) * kWaves * NB +
           sizeof(float) * 2 * (size_t)kvp;
}

hipError_t launch_rank2_f32_mfma(const Rank2Args &a, hipStream_t st) {
    const int blocks = (a.M + NB - 1) / NB;
    const size_t lds = rank2_f32_mfma_lds_bytes(a.kvp, a.ksp);
    hipLaunchKernelGGL(rank2_f32_mfma_kernel, dim3(blocks), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t rank2_f32_mfma_configure() {
    return hipFuncSetAttribute((const void *)rank2_f32_mfma_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

}  // namespace rom
