// Rank-2 leapfrog stepper, FP32 operators and states, MFMA products.
//
// Method: Sec. 2.4 eq. (2.5) for the staggered system of Sec. 3.1 eq. (3.3);
// one step is
//     V <- V + dt (Avs S + b u(t_n; mu)^T)      then      S <- S + dt Asv V .
//
// Decomposition (MI355X): the sample columns are independent, so each
// workgroup owns 4 or 8 columns (one or two column sets) for the WHOLE run
// and never talks to another workgroup: no grid or group barrier is needed (a cross-workgroup
// barrier costs about 1 us on this part, more than the products of one
// half-step).  The workgroup keeps its V and S columns, plus a compensation
// word per entry, resident in LDS; every half-step it streams the packed
// operator panels from L2 (the operators stay L2 resident across steps) and
// multiplies them with v_mfma_f32_4x4x1f32, whose 16 blocks cover a 64-row
// tile x 4 columns per instruction (lane l holds operator row l of the tile,
// the B operand is the state column l % 4 broadcast from LDS).  The
// streamed operator bytes per CU, not the MFMAs, bound a 4-column block;
// an 8-column block reuses each operator fragment for two MFMAs and pays
// off wherever there are more blocks than CUs.
//
// The same kernel, in adjoint mode, runs the discrete adjoint of that step
// backwards in time (see the adjoint entry point): the adjoint state (P, Q)
// obeys a leapfrog of the same shape with the transposed operators, the
// probe row c as source, 2 (c^T V+) as the per-sample amplitude and the
// source vector b as probe.
//
// Accuracy: MFMA FP32 rounds like sequential FP32 addition, which over 10^4
// steps at K = 256 drifts above 1e-5 relative.  Each wave therefore sums the
// reduction in chunks of kChunk terms into a fresh accumulator and folds
// every chunk into a (hi, lo) pair with an error-free two-sum; the state
// update itself is done in double-float (hi + lo) arithmetic.
#include "k_tile_f32.h"

namespace rom {
namespace {

using namespace tile;
using dev::f4;

enum Mode { kForward = 0, kAdjoint = 1, kInverse = 2 };

// One half-step of one field: wave w owns row tiles w, w + 4, ...  Ends
// with a barrier (the other half-step reads every row of this field).
template <bool FORCED, int NS>
__device__ __forceinline__ void half_step(const Field &f, const f4 (&res)[2 * res_pairs(NS)][kQ],
                                          f4 (&a0)[kQ], f4 (&a1)[kQ], Stream &s,
                                          const Field &fv, const Field &fs, int lane, int w,
                                          const float *bl, const float *cl, const double (&u)[NS],
                                          double dt, double (&ypart)[NS]) {
    const int j = lane & 3;
    for (int t = w; t < f.T; t += kWaves) {
        double acc[NS][4];
        tile_product<NS>(f, f.X + j * f.ldx, res, t == w ? f.rp : 0, a0, a1, s, fv, fs, w, lane, acc);
        finish_tile<FORCED, NS>(f, t, acc, lane, bl, cl, u, dt, ypart);
    }
    __syncthreads();
}

// Copy the (hi + lo) LDS columns (nb of them) of this workgroup to a K x M
// global matrix.  The (column, element) pairs are spread over all threads
// (each stored once, the waves evenly loaded), as float4 where the matrix is
// 16-byte aligned and K a multiple of 4 (every column then starts aligned).
__device__ __forceinline__ void store_cols(float *dst, const float *hi, const float *lo, int ld, int K, int col0,
                                           int M, int nb, int tid) {
    const int ncol = min(nb, M - col0);
    if ((K & 3) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        const int q4 = K >> 2;
        f4 *d = reinterpret_cast<f4 *>(dst) + (size_t)col0 * q4;
        for (int idx = tid; idx < ncol * q4; idx += kThreads) {
            const int c = idx / q4, q = idx - c * q4;
            d[(size_t)c * q4 + q] = reinterpret_cast<const f4 *>(hi + c * ld)[q] +
                                    reinterpret_cast<const f4 *>(lo + c * ld)[q];
        }
    } else {
        float *d = dst + (size_t)col0 * K;
        for (int idx = tid; idx < ncol * K; idx += kThreads) {
            const int c = idx / K, i = idx - c * K;
            d[(size_t)c * K + i] = hi[c * ld + i] + lo[c * ld + i];
        }
    }
}

// Kernel variants: without state traces (every plain run), or writing them
// every step (the adjoint's recompute and reverse sweeps, receiver runs),
// which always come with a probe (c with its trace y forward, b in the
// adjoint), so their per-step probe epilogue needs no branch.
enum Traces { kNoTraces = 0, kTraces = 1 };

// One workgroup per CU, one wave per SIMD: the compiler may use the whole
// register file for the prefetch buffers instead of trading them for
// occupancy.
//
// Forward: (V, S) = (a.V, a.S), operators (Avs, Asv) packed, source b,
//   probe c; optional state traces a.vtr / a.str (entry k = state after k
//   steps, k = 0..nsteps).
// Adjoint (NS = 1): (P, Q) = (a.V, a.S), operators (Asv^T, Avs^T) packed,
//   source c with amplitude 2 y (y = the forward probe trace a.ytr), probe
//   b; step n = n0 + nsteps - 1 - k at iteration k; writes
//   a.qtr[n - n0] = Q before and a.wtr[n - n0] = P after the P update, and
//   adds dt (b^T P) du/dmu(t_n) to a.dmu.
// Inverse (NS = 1, traces): the forward step undone, which the leapfrog
//   allows exactly in exact arithmetic (it is time-reversible): from the
//   state after step n0 + nsteps - 1, iteration k takes step
//   n = n0 + nsteps - 1 - k back, S <- S - dt Asv V, then
//   V <- V - dt (Avs S + b u(t_n)), and stores the state before step n at
//   trace entry n - n0 (entry nsteps: the state given), so the traces come
//   out in the forward layout.  No probe.
template <int MODE, int NS, int TR>
__device__ __forceinline__ void run_block(const Rank2Args &a, int col0, unsigned char *smem) {
    constexpr int NC = NB * NS;                  // columns of this workgroup
    const int kvp = a.kvp, ksp = a.ksp;
    const int ldv = kvp + 4, lds_ = ksp + 4;     // +4 floats: spread columns over banks
    float *Vh = reinterpret_cast<float *>(smem);
    float *Vl = Vh + NC * ldv;
    float *Sh = Vl + NC * ldv;
    float *Sl = Sh + NC * lds_;
    double *yp = reinterpret_cast<double *>(Sl + NC * lds_);   // [kWaves][NC]
    float *bl = reinterpret_cast<float *>(yp + kWaves * NC);    // source, kvp
    float *cl = bl + kvp;                                         // probe, kvp (0 if none)

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index, uniform
    const float *Vin = static_cast<const float *>(a.V);
    const float *Sin = static_cast<const float *>(a.S);
    const float *bv = static_cast<const float *>(a.b);
    const float *cv = static_cast<const float *>(a.c);

    for (int idx = tid; idx < NC * kvp; idx += kThreads) {
        int jj = idx / kvp, i = idx - jj * kvp, mm = col0 + jj;
        Vh[jj * ldv + i] = (mm < a.M && i < a.kv) ? Vin[(size_t)mm * a.kv + i] : 0.f;
        Vl[jj * ldv + i] = 0.f;
    }
    for (int idx = tid; idx < NC * ksp; idx += kThreads) {
        int jj = idx / ksp, i = idx - jj * ksp, mm = col0 + jj;
        Sh[jj * lds_ + i] = (mm < a.M && i < a.ks) ? Sin[(size_t)mm * a.ks + i] : 0.f;
        Sl[jj * lds_ + i] = 0.f;
    }
    // forward: source b, probe c;  adjoint: source c, probe b;  inverse:
    // source b, no probe
    const float *src = MODE == kAdjoint ? cv : bv;
    const float *prb = MODE == kForward ? cv : (MODE == kAdjoint ? bv : nullptr);
    for (int i = tid; i < kvp; i += kThreads) {
        bl[i] = (src != nullptr && i < a.kv) ? src[i] : 0.f;
        cl[i] = (prb != nullptr && i < a.kv) ? prb[i] : 0.f;
    }

    const int j = lane & 3;            // column of this lane in the MFMA output
    int m[NS];
    bool mok[NS];
    double muj[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        m[q] = col0 + j + 4 * q;
        mok[q] = m[q] < a.M;
        muj[q] = mok[q] ? a.mu[m[q]] : 1.0;
    }
    const bool probe = prb != nullptr;
    double Jacc = 0.0;
    // With traces (recompute and adjoint launches, probe always present)
    // every thread takes part in the per-step probe epilogue for a valid
    // column pc (threads past the block's columns repeat the last one), so
    // that epilogue has no branch either; pc == tid for the threads that
    // write J / dmu.
    const int pc = min(tid % NC, min(NC, a.M - col0) - 1);
    const double mupc = a.mu[col0 + pc];
    const Field fv = {static_cast<const f4 *>(a.avs), kvp / kTileRows, ksp, ksp / kChunk,
                      resident_pairs(ksp / kChunk, NS), Sh, lds_, Vh, Vl, ldv};
    const Field fs = {static_cast<const f4 *>(a.asv), ksp / kTileRows, kvp, kvp / kChunk,
                      resident_pairs(kvp / kChunk, NS), Vh, ldv, Sh, Sl, lds_};
    f4 resv[2 * res_pairs(NS)][kQ], ress[2 * res_pairs(NS)][kQ];
    load_resident<NS>(resv, fv, w, lane);
    load_resident<NS>(ress, fs, w, lane);
    // Let the resident loads land before the time loop: otherwise the
    // wait-count analysis merges "maybe still loading" into the loop header
    // and waits before every use of a resident register, which (counters
    // retire in order) also waits out the operator stream's prefetch.
    __builtin_amdgcn_s_waitcnt(dev::kWaitVm0);
    f4 a0[kQ], a1[kQ];
    Stream str;
    if constexpr (MODE == kInverse) {
        // S half-steps first: the operator stream starts with (and then
        // alternates from) the S-update tiles
        stream_start(str, a0, a1, fs, fv, w, lane);
        __syncthreads();
        store_cols(a.vtr + (size_t)a.nsteps * a.M * a.kv, Vh, Vl, ldv, a.kv, col0, a.M, NC, tid);
        store_cols(a.str + (size_t)a.nsteps * a.M * a.ks, Sh, Sl, lds_, a.ks, col0, a.M, NC, tid);
        double zero[NS], dummy[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) zero[q] = dummy[q] = 0.0;
        for (int64_t k = 0; k < a.nsteps; ++k) {
            const int64_t n = a.n0 + a.nsteps - 1 - k;
            const double t = (double)n * a.dt;
            double u64[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) u64[q] = mok[q] ? dev::forcing(a.source, t, muj[q]) : 0.0;
            half_step<false, NS>(fs, ress, a0, a1, str, fs, fv, lane, w, bl, cl, zero, -a.dt, dummy);
            half_step<true, NS>(fv, resv, a0, a1, str, fs, fv, lane, w, bl, cl, u64, -a.dt, dummy);
            store_cols(a.vtr + (size_t)(n - a.n0) * a.M * a.kv, Vh, Vl, ldv, a.kv, col0, a.M, NC, tid);
            store_cols(a.str + (size_t)(n - a.n0) * a.M * a.ks, Sh, Sl, lds_, a.ks, col0, a.M, NC, tid);
        }
        store_cols(static_cast<float *>(a.V), Vh, Vl, ldv, a.kv, col0, a.M, NC, tid);
        store_cols(static_cast<float *>(a.S), Sh, Sl, lds_, a.ks, col0, a.M, NC, tid);
        return;
    }
    stream_start(str, a0, a1, fv, fs, w, lane);
    __syncthreads();
    if (MODE == kForward && TR == kTraces) {
        store_cols(a.vtr, Vh, Vl, ldv, a.kv, col0, a.M, NC, tid);
        store_cols(a.str, Sh, Sl, lds_, a.ks, col0, a.M, NC, tid);
    }

    for (int64_t k = 0; k < a.nsteps; ++k) {
        const int64_t n = MODE == kForward ? a.n0 + k : a.n0 + a.nsteps - 1 - k;
        const int64_t r = n - a.n0;                    // trace row of step n
        const double t = (double)n * a.dt;
        double u64[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            if (MODE == kForward)
                u64[q] = mok[q] ? dev::forcing(a.source, t, muj[q]) : 0.0;
            else   // clamped column: the load is unconditional, the value selected
                u64[q] = mok[q] ? 2.0 * a.ytr[(size_t)r * a.M + min(m[q], a.M - 1)] : 0.0;
        }
        if (MODE == kAdjoint)   // q^{n+1}, paired with V^{n+1} in the dAsv product
            store_cols(a.qtr + (size_t)r * a.M * a.ks, Sh, Sl, lds_, a.ks, col0, a.M, NC, tid);

        // ---- first half-step: V += dt (Avs S + b u^T)   |   P += dt (Asv^T Q + 2 y c)
        double ypart[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) ypart[q] = 0.0;
        half_step<true, NS>(fv, resv, a0, a1, str, fv, fs, lane, w, bl, cl, u64, a.dt, ypart);
        if (probe) {
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                // sum over the 16 lanes that share column j (lane bits 2..5)
                double v = ypart[q];
                for (int off = 4; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
                if (lane < NB) yp[w * NC + 4 * q + lane] = v;
            }
        }
        if (MODE == kAdjoint)   // w^n, paired with S^n in the dAvs product
            store_cols(a.wtr + (size_t)r * a.M * a.kv, Vh, Vl, ldv, a.kv, col0, a.M, NC, tid);
        // ---- second half-step: S += dt Asv V   |   Q += dt Avs^T P
        // (its barrier also publishes yp before it is read below)
        double zero[NS], dummy[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) zero[q] = dummy[q] = 0.0;
        half_step<false, NS>(fs, ress, a0, a1, str, fv, fs, lane, w, bl, cl, zero, a.dt, dummy);
        if (TR == kTraces) {
            double yv = 0.0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) yv += yp[q * NC + pc];
            if (MODE == kForward) {
                Jacc += a.dt * (yv * yv);
                a.y[(size_t)k * a.M + col0 + pc] = yv;
            } else {
                Jacc += a.dt * yv * dev::forcing_dmu(a.source, t, mupc);
            }
        } else if (probe && tid < NC && col0 + tid < a.M) {
            double yv = 0.0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) yv += yp[q * NC + tid];
            if (MODE == kForward) {
                Jacc += a.dt * (yv * yv);
                if (a.y) a.y[(size_t)k * a.M + col0 + tid] = yv;
            } else {
                Jacc += a.dt * yv * dev::forcing_dmu(a.source, t, a.mu[col0 + tid]);
            }
        }
        if (MODE == kForward && TR == kTraces) {
            store_cols(a.vtr + (size_t)(k + 1) * a.M * a.kv, Vh, Vl, ldv, a.kv, col0, a.M, NC, tid);
            store_cols(a.str + (size_t)(k + 1) * a.M * a.ks, Sh, Sl, lds_, a.ks, col0, a.M, NC, tid);
        }
    }

    store_cols(static_cast<float *>(a.V), Vh, Vl, ldv, a.kv, col0, a.M, NC, tid);
    store_cols(static_cast<float *>(a.S), Sh, Sl, lds_, a.ks, col0, a.M, NC, tid);
    if (probe && tid < NC && col0 + tid < a.M) {
        if (MODE == kForward && a.J) a.J[col0 + tid] += Jacc;
        if (MODE == kAdjoint && a.dmu) a.dmu[col0 + tid] += Jacc;
    }
}

template <int MODE, int NS, int TR>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void rank2_f32_mfma_kernel(Rank2Args a) {
    extern __shared__ __align__(16) unsigned char smem[];
    run_block<MODE, NS, TR>(a, blockIdx.x * NB * NS, smem);
}

// Grouped forward run: workgroup i advances the column block of instance
// items[i].x that starts at column items[i].y, with the instance's column
// sets (a.nset); items are ordered by decreasing cost by the host, so the
// largest blocks are dispatched first.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void grouped_f32_mfma_kernel(const Rank2Args *__restrict__ inst, const int2 *__restrict__ items,
                             int64_t n0, int64_t nsteps) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 it = items[blockIdx.x];
    Rank2Args a = inst[it.x];
    a.n0 = n0;
    a.nsteps = nsteps;
    if (a.nset == 2)
        run_block<kForward, 2, kNoTraces>(a, it.y, smem);
    else
        run_block<kForward, 1, kNoTraces>(a, it.y, smem);
}

}  // namespace

size_t rank2_f32_mfma_lds_bytes(int kvp, int ksp, int nset) {
    return state_lds_bytes(kvp, ksp, NB * nset);
}

// Traced launches need the probe of their branch-free epilogue.
static bool traces_probe_ok(const Rank2Args &a, bool adjoint) {
    return adjoint ? (a.b != nullptr && a.ytr != nullptr) : (a.c != nullptr && a.y != nullptr);
}

hipError_t launch_rank2_f32_mfma(const Rank2Args &a, int nset, hipStream_t st) {
    const int nc = NB * nset;
    const int blocks = (a.M + nc - 1) / nc;
    const size_t lds = rank2_f32_mfma_lds_bytes(a.kvp, a.ksp, nset);
    if (a.vtr) {   // state traces: one column set
        if (!traces_probe_ok(a, false) || nset != 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL((rank2_f32_mfma_kernel<kForward, 1, kTraces>), dim3(blocks), dim3(kThreads), lds, st, a);
    } else if (nset == 2) {
        hipLaunchKernelGGL((rank2_f32_mfma_kernel<kForward, 2, kNoTraces>), dim3(blocks), dim3(kThreads), lds, st,
                           a);
    } else {
        hipLaunchKernelGGL((rank2_f32_mfma_kernel<kForward, 1, kNoTraces>), dim3(blocks), dim3(kThreads), lds, st,
                           a);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_f32_mfma(const Rank2Args &a, hipStream_t st) {
    const int blocks = (a.M + NB - 1) / NB;
    const size_t lds = rank2_f32_mfma_lds_bytes(a.kvp, a.ksp, 1);
    if (!traces_probe_ok(a, true)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((rank2_f32_mfma_kernel<kAdjoint, 1, kTraces>), dim3(blocks), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_inverse_f32_mfma(const Rank2Args &a, hipStream_t st) {
    const int blocks = (a.M + NB - 1) / NB;
    const size_t lds = rank2_f32_mfma_lds_bytes(a.kvp, a.ksp, 1);
    if (!a.vtr || !a.str) return hipErrorInvalidValue;
    hipLaunchKernelGGL((rank2_f32_mfma_kernel<kInverse, 1, kTraces>), dim3(blocks), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_grouped_f32_mfma(const Rank2Args *inst_dev, const int2 *items_dev, int nitems,
                                   size_t lds_bytes, int64_t n0, int64_t nsteps, hipStream_t st) {
    if (nitems <= 0 || nsteps <= 0) return hipSuccess;
    hipLaunchKernelGGL(grouped_f32_mfma_kernel, dim3(nitems), dim3(kThreads), lds_bytes, st, inst_dev,
                       items_dev, n0, nsteps);
    return hipGetLastError();
}

hipError_t rank2_f32_mfma_configure() {
    const void *fns[] = {(const void *)grouped_f32_mfma_kernel,
                         (const void *)rank2_f32_mfma_kernel<kForward, 1, kNoTraces>,
                         (const void *)rank2_f32_mfma_kernel<kForward, 2, kNoTraces>,
                         (const void *)rank2_f32_mfma_kernel<kForward, 1, kTraces>,
                         (const void *)rank2_f32_mfma_kernel<kAdjoint, 1, kTraces>,
                         (const void *)rank2_f32_mfma_kernel<kInverse, 1, kTraces>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rom
