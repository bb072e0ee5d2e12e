// Modified discrete energy of the leapfrog, per sample, in FP64:
//   E_m = |v_m|^2 + |s_m|^2 + dt v_m^T Avs s_m .
// For a skew pair (Asv = -Avs^T) the unforced step conserves it exactly and
// dt sigma_max(Avs) < 2 makes it positive definite, so its drift over a long
// run measures the arithmetic, and its size bounds the state (stability).
#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void energy_kernel(const double *__restrict__ A, int kv, int ks, double dt,
                                                     const T *__restrict__ V, const T *__restrict__ S,
                                                     double *__restrict__ E) {
    const int m = blockIdx.x;
    const T *v = V + (size_t)m * kv;
    const T *s = S + (size_t)m * ks;
    double acc_vv = 0.0, acc_ss = 0.0, acc_vas = 0.0;
    for (int i = threadIdx.x; i < kv; i += 256) {
        double r = 0.0;
        for (int j = 0; j < ks; ++j) r = fma(A[i + (size_t)j * kv], (double)s[j], r);
        const double vi = (double)v[i];
        acc_vas = fma(vi, r, acc_vas);
        acc_vv = fma(vi, vi, acc_vv);
    }
    for (int j = threadIdx.x; j < ks; j += 256) acc_ss = fma((double)s[j], (double)s[j], acc_ss);
    double x = acc_vv + acc_ss + dt * acc_vas;
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) E[m] = ((part[0] + part[1]) + part[2]) + part[3];
}

}  // namespace

hipError_t launch_energy(const double *A64, int kv, int ks, double dt, rom_dtype st_type, const void *V,
                         const void *S, int M, double *E, hipStream_t st) {
    if (st_type == ROM_F64)
        hipLaunchKernelGGL(energy_kernel<double>, dim3(M), dim3(256), 0, st, A64, kv, ks, dt,
                           static_cast<const double *>(V), static_cast<const double *>(S), E);
    else
        hipLaunchKernelGGL(energy_kernel<float>, dim3(M), dim3(256), 0, st, A64, kv, ks, dt,
                           static_cast<const float *>(V), static_cast<const float *>(S), E);
    return hipGetLastError();
}

}  // namespace rom
