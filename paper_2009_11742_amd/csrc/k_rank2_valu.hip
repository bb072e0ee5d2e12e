// Rank-2 leapfrog stepper on the vector ALUs, any state type (used for FP64
// states: on MI355X FP64 vector FMA runs at the FP64 matrix rate).
//
// Same decomposition as the FP32 MFMA kernel: a workgroup owns 4 sample
// columns for the whole run, its states live in LDS, no cross-workgroup
// communication.  Thread (wave w, lane) computes rows 64 t + lane for row
// tiles t = w, w + 4, ... and all 4 columns, summing the reduction in
// increasing k with fused multiply-adds.  When both operators fit in LDS next
// to the states they are staged there once; otherwise they are read from L2.
#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

constexpr int NB = kColBlock;
constexpr size_t kLdsBudget = 150 * 1024;
constexpr int kUWinV = 256 / NB;        // forcing window: one (step, column) value per thread
static_assert(NB * 64 == 256, "one wave of the 256 threads per column (probe sums)");

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c);
template <>
__device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return fma(a, b, c); }
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return fmaf(a, b, c); }

// RPL > 0 (Kv, Ks <= 64 RPL): wave w computes column w, each lane rows
// lane + 64 r (r < RPL), so all four waves work at small K; RPL = 0: thread
// (w, lane) computes rows 64 t + lane (t = w, w + 4, ..) of all 4 columns.
// Both sum each entry's terms in increasing k with the same FMAs, so they
// agree bitwise.  (Four interleaved FMA chains per entry measured no faster
// at K = 64 and slower at K = 128.)
template <typename T, int RPL>
__global__ __launch_bounds__(256) void rank2_valu_kernel(Rank2Args a, int ops_in_lds) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int kv = a.kv, ks = a.ks, kvp = a.kvp, ksp = a.ksp;
    T *V = reinterpret_cast<T *>(smem);                // [NB][kvp]
    T *S = V + NB * kvp;                                // [NB][ksp]
    double *uw = reinterpret_cast<double *>(S + NB * ksp);   // [kUWinV][NB] forcing window
    T *opA = reinterpret_cast<T *>(uw + kUWinV * NB);   // Avs (kv x ks) if staged
    T *opB = opA + (size_t)kv * ks;                     // Asv (ks x kv) if staged
    const T *gA = static_cast<const T *>(a.avs);
    const T *gB = static_cast<const T *>(a.asv);
    const T *A = gA, *B = gB;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int col0 = blockIdx.x * NB;
    const T *Vin = static_cast<const T *>(a.V);
    const T *Sin = static_cast<const T *>(a.S);
    const T *bv = static_cast<const T *>(a.b);
    const T *cv = static_cast<const T *>(a.c);

    for (int idx = tid; idx < NB * kvp; idx += 256) {
        int j = idx / kvp, i = idx - j * kvp, m = col0 + j;
        V[idx] = (m < a.M && i < kv) ? Vin[(size_t)m * kv + i] : T(0);
    }
    for (int idx = tid; idx < NB * ksp; idx += 256) {
        int j = idx / ksp, i = idx - j * ksp, m = col0 + j;
        S[idx] = (m < a.M && i < ks) ? Sin[(size_t)m * ks + i] : T(0);
    }
    if (ops_in_lds) {
        for (int idx = tid; idx < kv * ks; idx += 256) {
            opA[idx] = gA[idx];
            opB[idx] = gB[idx];
        }
        A = opA;
        B = opB;
    }
    double Jacc = 0.0;
    const T dt = (T)a.dt;
    __syncthreads();

    for (int64_t k = 0; k < a.nsteps; ++k) {
        // the forcing of the next kUWinV steps, one value per thread, once
        // per window (the previous step's last barrier protects the window)
        if (k % kUWinV == 0) {
            const int s = tid / NB, j = tid % NB;
            uw[tid] = (col0 + j < a.M) ? dev::forcing(a.source, (double)(a.n0 + k + s) * a.dt, a.mu[col0 + j]) : 0.0;
            __syncthreads();
        }
        const double *ur = uw + (k % kUWinV) * NB;
        // ---- velocity half-step
        if constexpr (RPL > 0) {
            T acc[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) acc[r] = T(0);
#pragma unroll 8
            for (int q = 0; q < ks; ++q) {
                const T sq = S[w * ksp + q];
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    acc[r] = fma_t<T>(A[min(lane + 64 * r, kv - 1) + (size_t)q * kv], sq, acc[r]);
            }
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                if (i < kv) V[w * kvp + i] = V[w * kvp + i] + dt * (acc[r] + bv[i] * (T)ur[w]);
            }
        }
        for (int i = w * 64 + lane; RPL == 0 && i < kv; i += 256) {
            T acc[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[j] = T(0);
            // unrolled so several operator loads (from L2 when the operators
            // are not staged in LDS) are in flight at once
#pragma unroll 8
            for (int q = 0; q < ks; ++q) {
                T aq = A[i + (size_t)q * kv];
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = fma_t<T>(aq, S[j * ksp + q], acc[j]);
            }
            const T bi = bv[i];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                T f = bi * (T)ur[j];
                V[j * kvp + i] = V[j * kvp + i] + dt * (acc[j] + f);
            }
        }
        __syncthreads();
        if (cv != nullptr) {
            // probe of column w (one wave per column): lane partials over
            // rows lane, lane + 64, .., then the wave's tree
            double yv = 0.0;
            for (int i = lane; i < kv; i += 64) yv = fma((double)cv[i], (double)V[w * kvp + i], yv);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) yv += __shfl_xor(yv, off, 64);
            if (lane == 0) {
                Jacc += a.dt * (yv * yv);
                if (a.y && col0 + w < a.M) a.y[(size_t)k * a.M + col0 + w] = yv;
            }
        }
        // ---- stress half-step
        if constexpr (RPL > 0) {
            T acc[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) acc[r] = T(0);
#pragma unroll 8
            for (int q = 0; q < kv; ++q) {
                const T vq = V[w * kvp + q];
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    acc[r] = fma_t<T>(B[min(lane + 64 * r, ks - 1) + (size_t)q * ks], vq, acc[r]);
            }
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                if (i < ks) S[w * ksp + i] = S[w * ksp + i] + dt * acc[r];
            }
        }
        for (int i = w * 64 + lane; RPL == 0 && i < ks; i += 256) {
            T acc[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[j] = T(0);
#pragma unroll 8
            for (int q = 0; q < kv; ++q) {
                T bq = B[i + (size_t)q * ks];
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = fma_t<T>(bq, V[j * kvp + q], acc[j]);
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) S[j * ksp + i] = S[j * ksp + i] + dt * acc[j];
        }
        __syncthreads();
    }

    T *Vout = static_cast<T *>(a.V);
    T *Sout = static_cast<T *>(a.S);
    for (int idx = tid; idx < NB * kvp; idx += 256) {
        int j = idx / kvp, i = idx - j * kvp, m = col0 + j;
        if (m < a.M && i < kv) Vout[(size_t)m * kv + i] = V[idx];
    }
    for (int idx = tid; idx < NB * ksp; idx += 256) {
        int j = idx / ksp, i = idx - j * ksp, m = col0 + j;
        if (m < a.M && i < ks) Sout[(size_t)m * ks + i] = S[idx];
    }
    if (cv != nullptr && a.J && lane == 0 && col0 + w < a.M) a.J[col0 + w] += Jacc;
}

template <typename T>
size_t valu_lds(int kv, int ks, int kvp, int ksp, bool ops) {
    size_t base = sizeof(T) * (size_t)NB * (kvp + ksp) + sizeof(double) * kUWinV * NB;
    base = (base + 15) / 16 * 16;
    return ops ? base + 2 * sizeof(T) * (size_t)kv * ks : base;
}

}  // namespace

template <typename T>
hipError_t launch_rank2_valu(const Rank2Args &a, hipStream_t st) {
    const int blocks = (a.M + NB - 1) / NB;
    bool ops = valu_lds<T>(a.kv, a.ks, a.kvp, a.ksp, true) <= kLdsBudget;
    size_t lds = valu_lds<T>(a.kv, a.ks, a.kvp, a.ksp, ops);
    if (lds > kLdsBudget) return hipErrorInvalidValue;
    const int kmax = a.kv > a.ks ? a.kv : a.ks;
    if (kmax <= 64)
        hipLaunchKernelGGL((rank2_valu_kernel<T, 1>), dim3(blocks), dim3(256), lds, st, a, ops ? 1 : 0);
    else if (kmax <= 128)
        hipLaunchKernelGGL((rank2_valu_kernel<T, 2>), dim3(blocks), dim3(256), lds, st, a, ops ? 1 : 0);
    else
        hipLaunchKernelGGL((rank2_valu_kernel<T, 0>), dim3(blocks), dim3(256), lds, st, a, ops ? 1 : 0);
    return hipGetLastError();
}

template hipError_t launch_rank2_valu<double>(const Rank2Args &, hipStream_t);
template hipError_t launch_rank2_valu<float>(const Rank2Args &, hipStream_t);

size_t rank2_valu_lds_bytes(rom_dtype st, int kv, int ks, int kvp, int ksp) {
    return st == ROM_F64 ? valu_lds<double>(kv, ks, kvp, ksp, false)
                         : valu_lds<float>(kv, ks, kvp, ksp, false);
}

hipError_t rank2_valu_configure() {
    const void *fns[] = {(const void *)rank2_valu_kernel<double, 0>, (const void *)rank2_valu_kernel<double, 1>,
                         (const void *)rank2_valu_kernel<double, 2>, (const void *)rank2_valu_kernel<float, 0>,
                         (const void *)rank2_valu_kernel<float, 1>, (const void *)rank2_valu_kernel<float, 2>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rom
