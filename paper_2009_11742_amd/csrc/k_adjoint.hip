// Support kernels of the discrete adjoint: the operator-gradient products
// dAvs += dt * W * S^T and dAsv += dt * Q * V^T over all (step, sample)
// pairs of a checkpoint segment, packing of the transposed operators for the
// reverse sweep, and the final FP64 -> FP32 conversion.
//
// The gradient product reduces over segment_length * M terms (~1.8e4 at the
// adjoint workload, ~1.3e6 over a whole run).  It runs on
// v_mfma_f32_16x16x4f32: the FP32 trace values multiply exactly, each MFMA
// chain sums kChainSteps * 4 = 64 terms in FP32, and every chain is folded
// into FP64 sums, so the result keeps ~1e-7 relative accuracy over any
// reduction length.  The reduction is split over waves and workgroups; the
// FP64 partials are summed in a fixed order by a second kernel, so the
// gradient is deterministic.
#include <algorithm>

#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

using dev::f4;
constexpr int kTile = 64;         // output rows and columns per wave (and per workgroup)
constexpr int kChainSteps = 16;   // MFMA k-steps (4 terms each) per FP32 chain
constexpr int kDepth = 4;         // k-steps of operand loads in flight

// Four consecutive rows r .. r+3 of column k of a column-major matrix with
// `ld` rows, read at an address clamped into the matrix (column ke - 1 past
// the end of the reduction, row 0 past the last row), so the load is always
// in bounds and never has to be waited for before its use.  Values of rows
// past the end only reach output rows that are never stored; values past
// the end of the reduction are zeroed where they are used.  VEC: ld and r
// are multiples of 4 (one aligned float4).
template <bool VEC>
__device__ __forceinline__ f4 load_rows4(const float *__restrict__ A, int r, int ld, int64_t k, int64_t ke) {
    const float *col = A + (k < ke ? k : ke - 1) * ld;
    if (VEC) return *reinterpret_cast<const f4 *>(col + (r < ld ? r : 0));
    f4 v;
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = col[r + s < ld ? r + s : ld - 1];
    return v;
}

// part[split][col][row] = sum over k in split's range of X[row][k] Y[col][k]
// for the 64 x 64 output tile (blockIdx.x, blockIdx.y); split = 4 blockIdx.z
// + wave.  Lane l loads rows r0 + 4 (l % 16) + s (s = 0..3) of reduction
// index k0 + l / 16, which makes s the row phase of four 16-row MFMA A
// fragments (and likewise four B fragments for the columns): 2 loads feed 16
// MFMAs.  MFMA output register r of fragment pair (s, s') in lane l is row
// r0 + 16 (l / 16) + 4 r + s, column c0 + 4 (l % 16) + s'.
template <bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_nt_mfma_kernel(const float *__restrict__ X, const float *__restrict__ Y, int rows, int cols,
                         int64_t R, int64_t kper, double *__restrict__ part) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int r0 = blockIdx.x * kTile, c0 = blockIdx.y * kTile;
    const int split = blockIdx.z * 4 + w;
    const int64_t kb = (int64_t)split * kper;
    const int64_t ke = kb + kper < R ? kb + kper : R;
    const int rr = r0 + 4 * li, cc = c0 + 4 * li;
    double acc[4][4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[s][t][r] = 0.0;
    // operands of k-step j sit in ring slot j % kDepth, loaded kDepth steps
    // before their MFMAs
    f4 ra[kDepth], rb[kDepth];
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
        ra[d] = load_rows4<VEC>(X, rr, rows, kb + 4 * d + lk, ke);
        rb[d] = load_rows4<VEC>(Y, cc, cols, kb + 4 * d + lk, ke);
    }
    for (int64_t k0 = kb; k0 < ke; k0 += 4 * kChainSteps) {
        f4 ch[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < 4; ++t) ch[s][t] = f4{0.f, 0.f, 0.f, 0.f};
        // the ring is carried by this (rolled) loop, so the compiler cannot
        // sink a prefetch next to its use
#pragma unroll 1
        for (int g = 0; g < kChainSteps; g += kDepth) {
#pragma unroll
            for (int d = 0; d < kDepth; ++d) {
                // k-step k0/4 + g + d; zero the A operand past the reduction
                const bool kin = k0 + 4 * (g + d) + lk < ke;
                f4 a;
#pragma unroll
                for (int s = 0; s < 4; ++s) a[s] = kin ? ra[d][s] : 0.f;
                const f4 b = rb[d];
                const int64_t kn = k0 + 4 * (g + d + kDepth) + lk;
                ra[d] = load_rows4<VEC>(X, rr, rows, kn, ke);
                rb[d] = load_rows4<VEC>(Y, cc, cols, kn, ke);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        ch[s][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[t], ch[s][t], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[s][t][r] += (double)ch[s][t][r];
    }
    double *P = part + (size_t)split * rows * cols;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + 16 * lk + 4 * r + s, col = cc + t;
                if (row < rows && col < cols) P[row + (size_t)col * rows] = acc[s][t][r];
            }
}

// dA[i] += alpha * sum_p part[p][i], p = 0 .. nsplit - 1 in order.
__global__ void reduce_parts_kernel(const double *__restrict__ part, int nsplit, int64_t n, double alpha,
                                    double *__restrict__ dA) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int p = 0; p < nsplit; ++p) v += part[(size_t)p * n + i];
        dA[i] += alpha * v;
    }
}

// ytr[k M + m] = c . (state m at trace entry k + 1) for k < len: the forward
// probe trace of a segment recovered from its state traces (one wave per
// value, lanes striding over the rows, FP64 sums).
__global__ __launch_bounds__(256) void probe_trace_kernel(const float *__restrict__ vtr, const float *__restrict__ c,
                                                          int kv, int M, int64_t len, double *__restrict__ ytr) {
    const int lane = threadIdx.x & 63;
    const int64_t nval = len * M;
    for (int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); idx < nval; idx += (int64_t)gridDim.x * 4) {
        const float *v = vtr + (size_t)(idx + M) * kv;      // entry k + 1, column m: (k + 1) M + m = idx + M
        double acc = 0.0;
        for (int i = lane; i < kv; i += 64) acc += (double)c[i] * (double)v[i];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) ytr[idx] = acc;
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

// Workgroups along the reduction: enough tiles x splits to cover the CUs
// (at most 8, at least 1).
static int gemm_nt_zsplit(int rows, int cols) {
    const int tiles = ((rows + kTile - 1) / kTile) * ((cols + kTile - 1) / kTile);
    int z = (256 + tiles - 1) / tiles;
    return z < 1 ? 1 : (z > 8 ? 8 : z);
}

int gemm_nt_splits(int rows, int cols) { return 4 * gemm_nt_zsplit(rows, cols); }

hipError_t launch_gemm_nt_acc64(const float *X, const float *Y, int rows, int cols, int64_t R,
                                double alpha, double *dA, double *part, hipStream_t st) {
    if (R <= 0) return hipSuccess;
    const int z = gemm_nt_zsplit(rows, cols), nsplit = 4 * z;
    const int64_t kper = ((R + nsplit - 1) / nsplit + 3) / 4 * 4;
    dim3 grid((rows + kTile - 1) / kTile, (cols + kTile - 1) / kTile, z);
    if (rows % 4 == 0 && cols % 4 == 0)
        hipLaunchKernelGGL(gemm_nt_mfma_kernel<true>, grid, dim3(256), 0, st, X, Y, rows, cols, R, kper, part);
    else
        hipLaunchKernelGGL(gemm_nt_mfma_kernel<false>, grid, dim3(256), 0, st, X, Y, rows, cols, R, kper, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)rows * cols;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(grid_for(n, 4096)), dim3(256), 0, st, part, nsplit, n, alpha, dA);
    return hipGetLastError();
}

hipError_t launch_probe_trace(const float *vtr, const float *c, int kv, int M, int64_t len, double *ytr,
                              hipStream_t st) {
    const int64_t nval = len * M;
    if (nval <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((nval + 3) / 4, 16384);
    hipLaunchKernelGGL(probe_trace_kernel, dim3((unsigned)blocks), dim3(256), 0, st, vtr, c, kv, M, len, ytr);
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
