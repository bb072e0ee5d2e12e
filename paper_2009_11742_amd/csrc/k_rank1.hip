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

}  // namespace

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
