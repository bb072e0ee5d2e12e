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

// Compensated 64 x 4 tile of  P[t] * X  where P is a packed operator panel
// (pk[t][k/4][lane][k%4] = P[64 t + lane][k]) and X the 4 LDS-resident
// columns (column j at xcol_base + j * ld).  Returns per lane the rows
// 64 t + 4 (lane / 4) + r, r = 0..3, of column lane % 4 as (H, L).
__device__ __forceinline__ void tile_product(const f4 *__restrict__ pk, int t, int kp,
                                             const float *xcol, int lane, f4 &H, f4 &L) {
    const f4 *ap = pk + (size_t)t * (size_t)(kp / 4) * 64 + lane;
    f4 hi = {0.f, 0.f, 0.f, 0.f}, lo = {0.f, 0.f, 0.f, 0.f};
    f4 cur[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) cur[q] = ap[q * 64];
    const int nch = kp / kChunk;
    for (int ch = 0; ch < nch; ++ch) {
        f4 nxt[kQ];
        const bool more = ch + 1 < nch;
        if (more) {
            const f4 *an = ap + (size_t)(ch + 1) * kQ * 64;
#pragma unroll
            for (int q = 0; q < kQ; ++q) nxt[q] = an[q * 64];
        }
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        const float *xb = xcol + ch * kChunk;
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            f4 bv = *(const f4 *)(xb + 4 * q);
            acc = __builtin_amdgcn_mfma_f32_4x4x1f32(cur[q].x, bv.x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_4x4x1f32(cur[q].y, bv.y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_4x4x1f32(cur[q].z, bv.z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_4x4x1f32(cur[q].w, bv.w, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float s, e;
            dev::two_sum(hi[r], acc[r], s, e);
            hi[r] = s;
            lo[r] += e;
        }
        if (more) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) cur[q] = nxt[q];
        }
    }
    H = hi;
    L = lo;
}

__global__ __launch_bounds__(256) void rank2_f32_mfma_kernel(Rank2Args a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int kvp = a.kvp, ksp = a.ksp;
    const int ldv = kvp + 4, lds_ = ksp + 4;     // +4 floats: spread columns over banks
    float *Vh = reinterpret_cast<float *>(smem);
    float *Vl = Vh + NB * ldv;
    float *Sh = Vl + NB * ldv;
    float *Sl = Sh + NB * lds_;
    double *yp = reinterpret_cast<double *>(Sl + NB * lds_);   // [4 waves][NB]

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int col0 = blockIdx.x * NB;
    const float *Vin = static_cast<const float *>(a.V);
    const float *Sin = static_cast<const float *>(a.S);
    const float *bv = static_cast<const float *>(a.b);
    const float *cv = static_cast<const float *>(a.c);
    const f4 *avs = static_cast<const f4 *>(a.avs);
    const f4 *asv = static_cast<const f4 *>(a.asv);

    for (int idx = tid; idx < NB * kvp; idx += 256) {
        int j = idx / kvp, i = idx - j * kvp, m = col0 + j;
        Vh[j * ldv + i] = (m < a.M && i < a.kv) ? Vin[(size_t)m * a.kv + i] : 0.f;
        Vl[j * ldv + i] = 0.f;
    }
    for (int idx = tid; idx < NB * ksp; idx += 256) {
        int j = idx / ksp, i = idx - j * ksp, m = col0 + j;
        Sh[j * lds_ + i] = (m < a.M && i < a.ks) ? Sin[(size_t)m * a.ks + i] : 0.f;
        Sl[j * lds_ + i] = 0.f;
    }

    const int j = lane & 3;            // column of this lane in the MFMA output
    const int rq = 4 * (lane >> 2);    // first of the lane's 4 rows inside a tile
    const int m = col0 + j;
    const bool mok = m < a.M;
    const double muj = mok ? a.mu[m] : 1.0;
    const float dtf = (float)a.dt;
    const int TV = kvp / kTileRows, TS = ksp / kTileRows;
    const bool probe = cv != nullptr;
    double Jacc = 0.0;
    __syncthreads();

    for (int64_t k = 0; k < a.nsteps; ++k) {
        const double t = (double)(a.n0 + k) * a.dt;
        const double u64 = mok ? dev::ricker(t, muj) : 0.0;
        const float uh = (float)u64;
        const float ul = (float)(u64 - (double)uh);

        // ---- velocity half-step: V += dt (Avs S + b u^T)
        double ypart = 0.0;
        for (int tt = w; tt < TV; tt += 4) {
            f4 H, L;
            tile_product(avs, tt, ksp, Sh + j * lds_, lane, H, L);
            const int i0 = tt * kTileRows + rq;
            f4 vh = *(f4 *)(Vh + j * ldv + i0);
            f4 vl = *(f4 *)(Vl + j * ldv + i0);
            f4 bb = *(const f4 *)(bv + i0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float F = bb[r] * uh;
                float Fe = fmaf(bb[r], uh, -F) + bb[r] * ul;
                float h = vh[r], l = vl[r];
                dev::comp_update(h, l, H[r], L[r], F, Fe, dtf);
                vh[r] = h;
                vl[r] = l;
                if (probe && i0 + r < a.kv) ypart += (double)cv[i0 + r] * ((double)h + (double)l);
            }
            *(f4 *)(Vh + j * ldv + i0) = vh;
            *(f4 *)(Vl + j * ldv + i0) = vl;
        }
        if (probe) {
            // sum over the 16 lanes that share column j (lane bits 2..5)
            for (int off = 4; off < 64; off <<= 1) ypart += __shfl_xor(ypart, off, 64);
            if (lane < NB) yp[w * NB + lane] = ypart;
        }
        __syncthreads();

        if (probe && tid < NB) {
            double yv = yp[0 * NB + tid] + yp[1 * NB + tid] + yp[2 * NB + tid] + yp[3 * NB + tid];
            Jacc += a.dt * (yv * yv);
            if (a.y && col0 + tid < a.M) a.y[(size_t)k * a.M + col0 + tid] = yv;
        }

        // ---- stress half-step: S += dt Asv V
        for (int tt = w; tt < TS; tt += 4) {
            f4 H, L;
            tile_product(asv, tt, kvp, Vh + j * ldv, lane, H, L);
            const int i0 = tt * kTileRows + rq;
            f4 sh = *(f4 *)(Sh + j * lds_ + i0);
            f4 sl = *(f4 *)(Sl + j * lds_ + i0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float h = sh[r], l = sl[r];
                dev::comp_update(h, l, H[r], L[r], 0.f, 0.f, dtf);
                sh[r] = h;
                sl[r] = l;
            }
            *(f4 *)(Sh + j * lds_ + i0) = sh;
            *(f4 *)(Sl + j * lds_ + i0) = sl;
        }
        __syncthreads();
    }

    float *Vout = static_cast<float *>(a.V);
    float *Sout = static_cast<float *>(a.S);
    for (int idx = tid; idx < NB * kvp; idx += 256) {
        int jj = idx / kvp, i = idx - jj * kvp, mm = col0 + jj;
        if (mm < a.M && i < a.kv) Vout[(size_t)mm * a.kv + i] = Vh[jj * ldv + i] + Vl[jj * ldv + i];
    }
    for (int idx = tid; idx < NB * ksp; idx += 256) {
        int jj = idx / ksp, i = idx - jj * ksp, mm = col0 + jj;
        if (mm < a.M && i < a.ks) Sout[(size_t)mm * a.ks + i] = Sh[jj * lds_ + i] + Sl[jj * lds_ + i];
    }
    if (probe && a.J && tid < NB && col0 + tid < a.M) a.J[col0 + tid] += Jacc;
}

}  // namespace

size_t rank2_f32_mfma_lds_bytes(int kvp, int ksp) {
    return sizeof(float) * (size_t)NB * 2 * ((kvp + 4) + (ksp + 4)) + sizeof(double) * 4 * NB;
}

hipError_t launch_rank2_f32_mfma(const Rank2Args &a, hipStream_t st) {
    const int blocks = (a.M + NB - 1) / NB;
    const size_t lds = rank2_f32_mfma_lds_bytes(a.kvp, a.ksp);
    hipLaunchKernelGGL(rank2_f32_mfma_kernel, dim3(blocks), dim3(256), lds, st, a);
    return hipGetLastError();
}

hipError_t rank2_f32_mfma_configure() {
    return hipFuncSetAttribute((const void *)rank2_f32_mfma_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

}  // namespace rom
