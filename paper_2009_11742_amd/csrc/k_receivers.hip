// Seismograms at R receivers and their ensemble statistics, from the state
// traces of a stepped chunk.
//
// Method: the velocity at a target point is reconstructed from a single row
// of the velocity basis, so a receiver is a row c_r of length Kv and its
// seismogram for sample m after step n is  Y[n][r][m] = c_r . V_m^(n+1)
// (Sec. 4.5).  Over the ensemble of M samples each (step, receiver) gets
// the mean, the population variance and the nearest-rank 5th / 50th / 95th
// percentiles (the ceil(p M / 100)-th smallest value), the statistics the
// paper plots for its ensemble.
//
// One workgroup per step of the chunk.  Thread t owns sample columns
// t, t + 256, ... and accumulates the dot products of up to kRcRows
// receivers at a time in FP64, reading its column of the trace once per
// pass (contiguous in k) and the receiver rows from LDS, where they sit
// k-major so the kRcRows values of one k are a broadcast read.  The
// statistics use fixed-shape reductions (deterministic) and a bitonic sort
// of each receiver's M values in LDS.
#include <math.h>

#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

constexpr int kRcThreads = 256;
constexpr int kRcRows = 16;        // receivers per accumulation pass

// Ascending bitonic sort of P (a power of two) doubles in LDS; every thread
// of the block calls it.
__device__ void bitonic_sort(double *x, int P, int tid) {
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P; i += kRcThreads) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const double a = x[i], b = x[l];
                    if ((a > b) == up) {
                        x[i] = b;
                        x[l] = a;
                    }
                }
            }
            __syncthreads();
        }
}

// Sum over the block in a fixed tree (the same order on every run).
__device__ double block_sum(double v, double *red, int tid) {
    red[tid] = v;
    __syncthreads();
    for (int s = kRcThreads / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// vtr: (L + 1) x M x Kv FP32 states, entry n + 1 = after step n of the
// chunk; C: R x Kv row-major FP32; Y: L x R x M FP64 (or null); stats:
// L x R x 5 FP64 (or null): mean, variance, p0, p1, p2 percentiles at the
// 0-based sorted positions i0, i1, i2.
__global__ __launch_bounds__(kRcThreads) void receivers_kernel(const float *__restrict__ vtr, int kv, int M,
                                                               const float *__restrict__ C, int R, int P,
                                                               double *__restrict__ Y, double *__restrict__ stats,
                                                               int i0, int i1, int i2) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *ys = reinterpret_cast<double *>(smem);              // [R][M]
    double *buf = ys + (size_t)R * M;                            // [P]
    double *red = buf + P;                                       // [kRcThreads]
    float *ct = reinterpret_cast<float *>(red + kRcThreads);     // [Kv][Rp], Rp = R rounded up to kRcRows
    const int Rp = (R + kRcRows - 1) / kRcRows * kRcRows;
    const int n = blockIdx.x, tid = threadIdx.x;
    const float *V = vtr + (size_t)(n + 1) * M * kv;

    for (int idx = tid; idx < kv * Rp; idx += kRcThreads) {
        const int k = idx / Rp, r = idx - k * Rp;
        ct[idx] = r < R ? C[(size_t)r * kv + k] : 0.f;
    }
    __syncthreads();

    for (int m0 = 0; m0 < M; m0 += kRcThreads) {
        const int m = m0 + tid;
        const float *col = V + (size_t)min(m, M - 1) * kv;
        for (int r0 = 0; r0 < R; r0 += kRcRows) {
            double acc[kRcRows];
#pragma unroll
            for (int i = 0; i < kRcRows; ++i) acc[i] = 0.0;
            for (int k = 0; k < kv; ++k) {
                const double v = (double)col[k];
                const float *ck = ct + (size_t)k * Rp + r0;
#pragma unroll
                for (int i = 0; i < kRcRows; ++i) acc[i] = fma((double)ck[i], v, acc[i]);
            }
            if (m < M) {
#pragma unroll
                for (int i = 0; i < kRcRows; ++i)
                    if (r0 + i < R) ys[(size_t)(r0 + i) * M + m] = acc[i];
            }
        }
    }
    __syncthreads();
    if (Y) {
        double *Yn = Y + (size_t)n * R * M;
        for (int idx = tid; idx < R * M; idx += kRcThreads) Yn[idx] = ys[idx];
    }
    if (!stats) return;
    for (int r = 0; r < R; ++r) {
        const double *yr = ys + (size_t)r * M;
        double s = 0.0;
        for (int m = tid; m < M; m += kRcThreads) s += yr[m];
        const double mean = block_sum(s, red, tid) / M;
        double q = 0.0;
        for (int m = tid; m < M; m += kRcThreads) {
            const double d = yr[m] - mean;
            q += d * d;
        }
        const double var = block_sum(q, red, tid) / M;
        for (int i = tid; i < P; i += kRcThreads) buf[i] = i < M ? yr[i] : HUGE_VAL;
        __syncthreads();
        bitonic_sort(buf, P, tid);
        if (tid == 0) {
            double *o = stats + ((size_t)n * R + r) * 5;
            o[0] = mean;
            o[1] = var;
            o[2] = buf[i0];
            o[3] = buf[i1];
            o[4] = buf[i2];
        }
        __syncthreads();
    }
}

int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

size_t receivers_lds_bytes(int kv, int M, int R) {
    const int P = pow2_at_least(M);
    const int Rp = (R + kRcRows - 1) / kRcRows * kRcRows;
    return sizeof(double) * ((size_t)R * M + P + kRcThreads) + sizeof(float) * (size_t)kv * Rp;
}

static int pct_index(int p, int M) {
    const int k = (p * M + 99) / 100;
    return (k < 1 ? 1 : k) - 1;
}

hipError_t launch_receivers(const float *vtr, int kv, int M, int L, const float *C, int R, double *Y,
                            double *stats, hipStream_t st) {
    if (L <= 0) return hipSuccess;
    const size_t lds = receivers_lds_bytes(kv, M, R);
    hipLaunchKernelGGL(receivers_kernel, dim3(L), dim3(kRcThreads), lds, st, vtr, kv, M, C, R, pow2_at_least(M), Y,
                       stats, pct_index(5, M), pct_index(50, M), pct_index(95, M));
    return hipGetLastError();
}

hipError_t receivers_configure() {
    return hipFuncSetAttribute((const void *)receivers_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024);
}

}  // namespace rom
