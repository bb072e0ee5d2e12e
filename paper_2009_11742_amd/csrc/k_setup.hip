// Setup kernels run once per context: FP64 staging copies of the operators
// and source are converted to the state type and packed into the panels the
// rank-2 MFMA kernel streams (the time-independent terms are prepared once,
// as the paper does for its precomputed reduced operators, Sec. 2.2).
#include <algorithm>

#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

__global__ void convert_kernel(const double *__restrict__ src, void *__restrict__ dst, int64_t n,
                               int to) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        if (to == ROM_F64) static_cast<double *>(dst)[i] = src[i];
        else static_cast<float *>(dst)[i] = (float)src[i];
    }
}

// pk[t][k/4][lane][k%4] = A[64 t + lane][k] (A column-major rows x cols),
// zero outside rows x cols; panel sizes rowsp x colsp (multiples of 64).
__global__ void pack_f32_kernel(const double *__restrict__ A, int rows, int cols, int rowsp,
                                int colsp, float *__restrict__ pk) {
    int64_t total = (int64_t)rowsp * colsp;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; idx < total; idx += stride) {
        int64_t r = idx;
        int k4 = (int)(r % 4); r /= 4;
        int lane = (int)(r % 64); r /= 64;
        int kq = (int)(r % (colsp / 4)); r /= (colsp / 4);
        int t = (int)r;
        int row = t * kTileRows + lane, col = kq * 4 + k4;
        pk[idx] = (row < rows && col < cols) ? (float)A[row + (int64_t)col * rows] : 0.f;
    }
}

__global__ void f32_to_f64_kernel(const float *__restrict__ s, double *__restrict__ d, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (double)s[i];
}

}  // namespace

hipError_t launch_convert_f32_to_f64(const float *src, double *dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(f32_to_f64_kernel, dim3(blocks), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_convert(const double *src, void *dst, int64_t n, rom_dtype to, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(convert_kernel, dim3(blocks), dim3(256), 0, st, src, dst, n, (int)to);
    return hipGetLastError();
}

hipError_t launch_pack_f32(const double *A, int rows, int cols, int rowsp, int colsp, float *pk,
                           hipStream_t st) {
    int64_t total = (int64_t)rowsp * colsp;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(pack_f32_kernel, dim3(blocks), dim3(256), 0, st, A, rows, cols, rowsp, colsp, pk);
    return hipGetLastError();
}

}  // namespace rom

namespace rom {
namespace {

// out[i] = sum_q theta[q] terms[q n + i], terms added in turn (q = 0, 1, ...;
// product then sum, each rounded: the build does not contract).
__global__ void affine_combine_kernel(const double *__restrict__ terms, int Q, int64_t n, AffineCoeffs th,
                                      double *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = th.c[0] * terms[i];
        for (int q = 1; q < Q; ++q) acc = acc + th.c[q] * terms[(size_t)q * n + i];
        out[i] = acc;
    }
}

}  // namespace

hipError_t launch_affine_combine(const double *terms, int Q, int64_t n, const AffineCoeffs &th, double *out,
                                 hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(affine_combine_kernel, dim3((unsigned)blocks), dim3(256), 0, st, terms, Q, n, th, out);
    return hipGetLastError();
}

namespace {

// flag |= 1 if any of the n values (FP64 if f64, else FP32) is NaN or
// infinite.
__global__ void nonfinite_kernel(const void *__restrict__ x, int64_t n, int f64, int *__restrict__ flag) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = f64 ? static_cast<const double *>(x)[i] : (double)static_cast<const float *>(x)[i];
        bad |= !isfinite(v);
    }
    if (bad) __hip_atomic_fetch_or(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

hipError_t launch_nonfinite(const void *x, int64_t n, bool f64, int *flag, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, n, f64 ? 1 : 0, flag);
    return hipGetLastError();
}

}  // namespace rom
