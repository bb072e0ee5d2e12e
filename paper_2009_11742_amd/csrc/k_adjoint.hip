// Support kernels of the discrete adjoint: the operator-gradient products
// dAvs += dt * W * S^T and dAsv += dt * Q * V^T over all (step, sample)
// pairs of a checkpoint segment, packing of the transposed operators for the
// reverse sweep, and the final FP64 -> FP32 conversion.
//
// The gradient product reduces over segment_length * M terms (~1.8e4 at the
// adjoint workload, ~1.3e6 over a whole run), so it accumulates in FP64 on
// the vector ALUs (FP64 FMA runs at the FP64 matrix rate on MI355X): the
// FP32 inputs are exact in FP64 and the reduction adds no visible error.
#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

using dev::f4;
constexpr int kTile = 64;   // output tile (rows x cols) per workgroup
constexpr int kRb = 32;     // reduction block staged in LDS

// dA[r0:r0+64, c0:c0+64] += alpha * X[r0:, :] * Y[c0:, :]^T.  Thread (tx, ty)
// of a 16 x 16 grid owns a 4 x 4 block of the output.
__global__ __launch_bounds__(256) void gemm_nt_acc64_kernel(const float *__restrict__ X,
                                                            const float *__restrict__ Y, int rows,
                                                            int cols, int64_t R, double alpha,
                                                            double *__restrict__ dA) {
    __shared__ __align__(16) float Xs[kRb][kTile + 4];
    __shared__ __align__(16) float Ys[kRb][kTile + 4];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int r0 = blockIdx.x * kTile, c0 = blockIdx.y * kTile;
    double acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
    for (int64_t kb = 0; kb < R; kb += kRb) {
        for (int e = threadIdx.x; e < kRb * kTile; e += 256) {
            const int kk = e / kTile, i = e - kk * kTile;
            const int64_t kc = kb + kk;
            const int row = r0 + i, col = c0 + i;
            Xs[kk][i] = (row < rows && kc < R) ? X[row + kc * rows] : 0.f;
            Ys[kk][i] = (col < cols && kc < R) ? Y[col + kc * cols] : 0.f;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < kRb; ++kk) {
            const f4 xv = *reinterpret_cast<const f4 *>(&Xs[kk][4 * tx]);
            const f4 yv = *reinterpret_cast<const f4 *>(&Ys[kk][4 * ty]);
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] = fma((double)xv[p], (double)yv[q], acc[p][q]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = r0 + 4 * tx + p, col = c0 + 4 * ty + q;
            if (row < rows && col < cols) dA[row + (int64_t)col * rows] += alpha * acc[p][q];
        }
}

__global__ void f64_to_f32_kernel(const double *__restrict__ s, float *__restrict__ d, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (float)s[i];
}

// pk[t][k/4][lane][k%4] = T[64 t + lane][k], T = A or A^T (A column-major
// rows x cols), zero outside T; padded T sizes prow x pcol.
__global__ void pack_from_f32_kernel(const float *__restrict__ A, int rows, int cols, int tr,
                                     int prow, int pcol, float *__restrict__ pk) {
    const int tR = tr ? cols : rows, tC = tr ? rows : cols;
    const int64_t total = (int64_t)prow * pcol;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = idx;
        const int k4 = (int)(r % 4); r /= 4;
        const int lane = (int)(r % 64); r /= 64;
        const int kq = (int)(r % (pcol / 4)); r /= (pcol / 4);
        const int i = (int)r * kTileRows + lane, k = kq * 4 + k4;
        float v = 0.f;
        if (i < tR && k < tC) v = tr ? A[k + (int64_t)i * rows] : A[i + (int64_t)k * rows];
        pk[idx] = v;
    }
}

int grid_for(int64_t n, int cap) {
    int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

hipError_t launch_gemm_nt_acc64(const float *X, const float *Y, int rows, int cols, int64_t R,
                                double alpha, double *dA, hipStream_t st) {
    if (R <= 0) return hipSuccess;
    dim3 grid((rows + kTile - 1) / kTile, (cols + kTile - 1) / kTile);
    hipLaunchKernelGGL(gemm_nt_acc64_kernel, grid, dim3(256), 0, st, X, Y, rows, cols, R, alpha, dA);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double *src, float *dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(f64_to_f32_kernel, dim3(grid_for(n, 4096)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_pack_f32_from_f32(const float *A, int rows, int cols, bool transpose, int prow,
                                    int pcol, float *pk, hipStream_t st) {
    const int64_t total = (int64_t)prow * pcol;
    hipLaunchKernelGGL(pack_from_f32_kernel, dim3(grid_for(total, 8192)), dim3(256), 0, st, A, rows,
                       cols, transpose ? 1 : 0, prow, pcol, pk);
    return hipGetLastError();
}

}  // namespace rom
