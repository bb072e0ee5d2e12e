// Rank-1 leapfrog step (Sec. 2.2 eq. (2.3) with the staggered form of
// Sec. 3.1): one sample, two matrix-vector products per step, the operators
// re-read from device memory by every call (the memory-bound formulation the
// paper contrasts with the rank-2 one, Sec. 2.3).
//
// Each half-step is one launch (the stress update needs the whole new
// velocity).  A workgroup computes 64 rows; its 4 waves split the reduction,
// lane = row, so every wave load of an operator column segment is 256
// contiguous bytes.  FP32 sums use the same compensated chunking as the
// rank-2 kernel and a double-float increment, so the state is rounded once
// per half-step.
#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

constexpr int kChunk = 32;

template <bool FORCED>
__global__ __launch_bounds__(256) void gemv_half_f32(const float *__restrict__ A, int rows, int cols,
                                                     const float *__restrict__ x, float *__restrict__ y,
                                                     const float *__restrict__ b, double dt, double t,
                                                     double mu, int src) {
    __shared__ float ph[4][64], pl[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int kq = (cols + 3) / 4;
    const int k0 = w * kq, k1 = min(cols, k0 + kq);
    float hi = 0.f, lo = 0.f;
    if (i < rows) {
        for (int c0 = k0; c0 < k1; c0 += kChunk) {
            const int c1 = min(k1, c0 + kChunk);
            float acc = 0.f;
            for (int k = c0; k < c1; ++k) acc = fmaf(A[i + (size_t)k * rows], x[k], acc);
            float s, e;
            dev::two_sum(hi, acc, s, e);
            hi = s;
            lo += e;
        }
    }
    ph[w][lane] = hi;
    pl[w][lane] = lo;
    __syncthreads();
    if (w == 0 && i < rows) {
        float H = ph[0][lane], L = pl[0][lane];
        for (int q = 1; q < 4; ++q) {
            float s, e;
            dev::two_sum(H, ph[q][lane], s, e);
            H = s;
            L += e + pl[q][lane];
        }
        float F = 0.f, Fe = 0.f;
        if (FORCED) {
            double u = dev::forcing(src, t, mu);
            float uh = (float)u, ul = (float)(u - (double)uh);
            F = b[i] * uh;
            Fe = fmaf(b[i], uh, -F) + b[i] * ul;
        }
        float h = y[i], l = 0.f;
        dev::comp_update(h, l, H, L, F, Fe, (float)dt);
        y[i] = h + l;
    }
}

__global__ __launch_bounds__(256) void gemv_half_f64(const double *__restrict__ A, int rows, int cols,
                                                     const double *__restrict__ x, double *__restrict__ y,
                                                     const double *__restrict__ b, double dt, double t,
                                                     double mu, int forced, int src) {
    __shared__ double part[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int kq = (cols + 3) / 4;
    const int k0 = w * kq, k1 = min(cols, k0 + kq);
    double acc = 0.0;
    if (i < rows)
        for (int k = k0; k < k1; ++k) acc = fma(A[i + (size_t)k * rows], x[k], acc);
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0 && i < rows) {
        double r = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        double f = forced ? b[i] * dev::forcing(src, t, mu) : 0.0;
        y[i] = y[i] + dt * (r + f);
    }
}

// Rank-1 formulation for many samples in one launch: workgroup m advances
// sample m through all its steps, and every half-step is a matrix-vector
// product that reads the operator from device memory again -- the rank-1
// cost model of Sec. 2.3 (no reuse of an operator entry within a step),
// with the whole chip busy and no launch per step.  Thread t owns rows t,
// t + 256, ... of both fields (at most kRank1Rows each); the state hi words
// pass through LDS to the other half-step.  The arithmetic per row is the
// single-sample kernel's: compensated chunks of kChunk terms in increasing
// k, then the double-float update.
constexpr int kRank1Rows = 4;

__device__ __forceinline__ void rank1_row(const float *__restrict__ A, int rows, int cols, int i,
                                          const float *__restrict__ x, float &H, float &L) {
    float hi = 0.f, lo = 0.f;
    for (int c0 = 0; c0 < cols; c0 += kChunk) {
        const int c1 = min(cols, c0 + kChunk);
        float acc = 0.f;
        for (int k = c0; k < c1; ++k) acc = fmaf(A[i + (size_t)k * rows], x[k], acc);
        float s, e;
        dev::two_sum(hi, acc, s, e);
        hi = s;
        lo += e;
    }
    H = hi;
    L = lo;
}

__global__ __launch_bounds__(256) void rank1_batch_f32(const float *__restrict__ Avs, const float *__restrict__ Asv,
                                                       const float *__restrict__ b, const double *__restrict__ mu,
                                                       int kv, int ks, double dt, int64_t n0, int64_t nsteps,
                                                       int src, float *__restrict__ V, float *__restrict__ S) {
    extern __shared__ float xsh[];
    float *xs = xsh, *xv = xsh + ks;           // S and V hi words
    const int m = blockIdx.x, tid = threadIdx.x;
    float vh[kRank1Rows], vl[kRank1Rows], sh[kRank1Rows], sl[kRank1Rows];
#pragma unroll
    for (int q = 0; q < kRank1Rows; ++q) {
        const int iv = tid + 256 * q, is = tid + 256 * q;
        vh[q] = iv < kv ? V[(size_t)m * kv + iv] : 0.f;
        sh[q] = is < ks ? S[(size_t)m * ks + is] : 0.f;
        vl[q] = sl[q] = 0.f;
        if (is < ks) xs[is] = sh[q];
    }
    const double mum = mu[m];
    __syncthreads();
    for (int64_t k = 0; k < nsteps; ++k) {
        const double u = dev::forcing(src, (double)(n0 + k) * dt, mum);
        const float uh = (float)u, ul = (float)(u - (double)uh);
#pragma unroll
        for (int q = 0; q < kRank1Rows; ++q) {
            const int i = tid + 256 * q;
            if (i < kv) {
                float H, L;
                rank1_row(Avs, kv, ks, i, xs, H, L);
                const float F = b[i] * uh;
                const float Fe = fmaf(b[i], uh, -F) + b[i] * ul;
                dev::comp_update(vh[q], vl[q], H, L, F, Fe, (float)dt);
                vh[q] = vh[q] + vl[q];      // rounded once per half-step, as the single-sample kernel
                vl[q] = 0.f;
                xv[i] = vh[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kRank1Rows; ++q) {
            const int i = tid + 256 * q;
            if (i < ks) {
                float H, L;
                rank1_row(Asv, ks, kv, i, xv, H, L);
                dev::comp_update(sh[q], sl[q], H, L, 0.f, 0.f, (float)dt);
                sh[q] = sh[q] + sl[q];
                sl[q] = 0.f;
                xs[i] = sh[q];     // xs is read only by the velocity half-step
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kRank1Rows; ++q) {
        const int i = tid + 256 * q;
        if (i < kv) V[(size_t)m * kv + i] = vh[q];
        if (i < ks) S[(size_t)m * ks + i] = sh[q];
    }
}

}  // namespace

hipError_t launch_rank1_batch(const Rank2Args &a, hipStream_t st) {
    if (a.kv > 256 * kRank1Rows || a.ks > 256 * kRank1Rows) return hipErrorInvalidValue;
    const size_t lds = sizeof(float) * (size_t)(a.kv + a.ks);
    hipLaunchKernelGGL(rank1_batch_f32, dim3(a.M), dim3(256), lds, st, static_cast<const float *>(a.avs),
                       static_cast<const float *>(a.asv), static_cast<const float *>(a.b), a.mu, a.kv, a.ks, a.dt,
                       a.n0, a.nsteps, a.source, static_cast<float *>(a.V), static_cast<float *>(a.S));
    return hipGetLastError();
}

template <>
hipError_t launch_rank1_step<float>(const void *avs_cm, const void *asv_cm, const void *b, int kv,
                                    int ks, double dt, int64_t n, double mu, int source, void *v, void *s,
                                    hipStream_t st) {
    const double t = (double)n * dt;
    hipLaunchKernelGGL(gemv_half_f32<true>, dim3((kv + 63) / 64), dim3(256), 0, st,
                       (const float *)avs_cm, kv, ks, (const float *)s, (float *)v,
                       (const float *)b, dt, t, mu, source);
    hipLaunchKernelGGL(gemv_half_f32<false>, dim3((ks + 63) / 64), dim3(256), 0, st,
                       (const float *)asv_cm, ks, kv, (const float *)v, (float *)s,
                       (const float *)nullptr, dt, t, mu, source);
    return hipGetLastError();
}

template <>
hipError_t launch_rank1_step<double>(const void *avs_cm, const void *asv_cm, const void *b, int kv,
                                     int ks, double dt, int64_t n, double mu, int source, void *v, void *s,
                                     hipStream_t st) {
    const double t = (double)n * dt;
    hipLaunchKernelGGL(gemv_half_f64, dim3((kv + 63) / 64), dim3(256), 0, st,
                       (const double *)avs_cm, kv, ks, (const double *)s, (double *)v,
                       (const double *)b, dt, t, mu, 1, source);
    hipLaunchKernelGGL(gemv_half_f64, dim3((ks + 63) / 64), dim3(256), 0, st,
                       (const double *)asv_cm, ks, kv, (const double *)v, (double *)s,
                       (const double *)nullptr, dt, t, mu, 0, source);
    return hipGetLastError();
}

}  // namespace rom
