// Full-order side of the method: the rank-2 FOM stepper over sparse CSR
// operators and the dense products of the offline stage (Galerkin
// projection, POD by Cholesky QR).
//
// FOM (Sec. 3, eq. (3.2)): dV/dt = Av S + f u(t; mu)^T, dS/dt = As V with
// sparse Av (Nv x Ns, about four entries per row) and As (Ns x Nv, about
// two), the leapfrog of the ROM.  States are row-major (element (r, m) at
// r M + m, one DOF's M samples contiguous, the layout of the paper's rank-2
// FOM runs): consecutive threads take consecutive samples of a row, so each
// stored entry is one broadcast load of (col, val) and one coalesced load of
// M state values; the kernel is bound by HBM (and MALL) bandwidth, which is
// the paper's point about the FOM.
//
// Offline products (Sec. 2.2, eq. (3.3); Sec. 4.4):
//   gemm_tn   C (K1 x K2, column-major) = P^T Q over the N rows of the
//             row-major tall-skinny P (N x K1) and Q (N x K2): the Galerkin
//             reductions Phi^T (A Phi) and Phi^T f, and the Gram matrices
//             X^T X of Cholesky QR.  64 x 64 output tiles, the N range split
//             over workgroups, FP64 partials summed in a fixed order.
//   gemm_nn   Y (N x K2, row-major) = X (N x K1, row-major) B (K1 x K2,
//             column-major): X R^{-1} and Q U of the POD.
// Both stage 16-row slabs of their operands in LDS; each thread owns a 4 x
// 4 block of the output in FP64.
#include <algorithm>

#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

constexpr int kThr = 256;

// MODE 0: Y = A X.  MODE 1: Y += dt (A X + f u(t; mu)^T).  MODE 2: Y += dt A X.
// The entry sum runs in stored order, then f u, then the scaled add, as the
// oracle's loop does (no contraction in this build).
template <int MODE, bool WIDE>
__global__ __launch_bounds__(kThr) void fom_csr_kernel(const int *__restrict__ ptr, const int *__restrict__ col,
                                                       const double *__restrict__ val, const double *__restrict__ X,
                                                       double *__restrict__ Y, int64_t nrows, int M,
                                                       const double *__restrict__ f, const double *__restrict__ mu,
                                                       double t, double dt, int src) {
    const int64_t total = nrows * M;
    for (int64_t e = (int64_t)blockIdx.x * kThr + threadIdx.x; e < total; e += (int64_t)gridDim.x * kThr) {
        int64_t r;
        int m;
        if (WIDE) {
            r = e / M;
            m = (int)(e - r * M);
        } else {
            const unsigned ue = (unsigned)e, uM = (unsigned)M;
            const unsigned ur = ue / uM;
            r = ur;
            m = (int)(ue - ur * uM);
        }
        const int k0 = ptr[r], k1 = ptr[r + 1];
        double inc = 0.0;
        for (int k = k0; k < k1; ++k) inc = inc + val[k] * X[(int64_t)col[k] * M + m];
        if (MODE == 0) {
            Y[e] = inc;
            continue;
        }
        if (MODE == 1) {
            const double fr = f[r];
            if (fr != 0.0) inc = inc + fr * dev::forcing(src, t, mu[m]);
        }
        Y[e] = Y[e] + dt * inc;
    }
}

// The same products from the padded (ELL) copy of the operator: row r's
// entries at [r W, r W + W), unused slots with column -1.  A thread's column
// and value loads then do not wait for the row pointers, which leaves two
// dependent memory trips per element (entries, then the gathered states)
// instead of three.  Entries are summed in stored order, as above.
//
// Work split, two orders.  chunk = 0: grid-stride (all workgroups sweep the
// state together, one contiguous window of memory at a time).  chunk > 0:
// workgroup b takes a contiguous range of chunk elements, dealt out so that
// the workgroups of one XCD (b % 8 under the round-robin dispatch) sweep one
// contiguous eighth of the rows in order, so a stencil neighbour gathered
// again one grid line later is still in that XCD's L2.  The second is faster
// for few samples per row (up to 12 % at M = 4), the first for many (3 - 10 %
// at M >= 16 on the larger grids); the launcher picks by M.
template <int MODE, bool WIDE, int W>
__global__ __launch_bounds__(kThr) void fom_ell_kernel(const int *__restrict__ ecol, const double *__restrict__ eval,
                                                       const double *__restrict__ X, double *__restrict__ Y,
                                                       int64_t nrows, int M, const double *__restrict__ f,
                                                       const double *__restrict__ mu, double t, double dt, int src,
                                                       int64_t chunk) {
    const int64_t total = nrows * M;
    const unsigned b = blockIdx.x, per = gridDim.x / 8;    // chunked launches use a multiple of 8 workgroups
    int64_t e0, e1, step;
    if (chunk > 0) {
        e0 = ((int64_t)(b % 8) * per + b / 8) * chunk;
        e1 = e0 + chunk < total ? e0 + chunk : total;
        step = kThr;
    } else {
        e0 = (int64_t)b * kThr;
        e1 = total;
        step = (int64_t)gridDim.x * kThr;
    }
    for (int64_t e = e0 + threadIdx.x; e < e1; e += step) {
        int64_t r;
        int m;
        if (WIDE) {
            r = e / M;
            m = (int)(e - r * M);
        } else {
            const unsigned ue = (unsigned)e, uM = (unsigned)M;
            const unsigned ur = ue / uM;
            r = ur;
            m = (int)(ue - ur * uM);
        }
        int c[W];
        double v[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            c[k] = ecol[r * W + k];
            v[k] = eval[r * W + k];
        }
        double y = 0.0;
        if (MODE != 0) y = Y[e];
        double x[W];
#pragma unroll
        for (int k = 0; k < W; ++k) x[k] = X[(int64_t)(c[k] < 0 ? 0 : c[k]) * M + m];
        double inc = 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k)
            if (c[k] >= 0) inc = inc + v[k] * x[k];
        if (MODE == 0) {
            Y[e] = inc;
            continue;
        }
        if (MODE == 1) {
            const double fr = f[r];
            if (fr != 0.0) inc = inc + fr * dev::forcing(src, t, mu[m]);
        }
        Y[e] = y + dt * inc;
    }
}

template <int MODE, bool WIDE>
void launch_ell(const FomCsr &A, const double *X, double *Y, int M, const double *f, const double *mu, double t,
                double dt, int src, hipStream_t st) {
    const int64_t n = A.nrows, total = n * M;
    int64_t nb, chunk = 0;
    if (M <= 8) {
        // XCD-contiguous ranges: a multiple of 8 workgroups, each a whole
        // number of 256-element slices
        nb = std::min<int64_t>((total + kThr - 1) / kThr, 32768);
        nb = (nb + 7) / 8 * 8;
        chunk = ((total + nb - 1) / nb + kThr - 1) / kThr * kThr;
    } else {
        nb = std::min<int64_t>((total + kThr - 1) / kThr, 65536);
    }
    const unsigned blocks = (unsigned)nb;
    switch (A.W) {
    case 2:
        hipLaunchKernelGGL((fom_ell_kernel<MODE, WIDE, 2>), dim3(blocks), dim3(kThr), 0, st, A.ecol, A.eval, X, Y, n,
                           M, f, mu, t, dt, src, chunk);
        break;
    case 4:
        hipLaunchKernelGGL((fom_ell_kernel<MODE, WIDE, 4>), dim3(blocks), dim3(kThr), 0, st, A.ecol, A.eval, X, Y, n,
                           M, f, mu, t, dt, src, chunk);
        break;
    default:
        hipLaunchKernelGGL((fom_ell_kernel<MODE, WIDE, 8>), dim3(blocks), dim3(kThr), 0, st, A.ecol, A.eval, X, Y, n,
                           M, f, mu, t, dt, src, chunk);
        break;
    }
}

template <int MODE>
hipError_t launch_csr(const FomCsr &A, const double *X, double *Y, int M, const double *f, const double *mu,
                      double t, double dt, int src, hipStream_t st) {
    const int64_t total = (int64_t)A.nrows * M;
    if (total <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((total + kThr - 1) / kThr, 65536);
    const bool wide = total >= (int64_t)1 << 32;
    if (A.W > 0) {
        if (wide) launch_ell<MODE, true>(A, X, Y, M, f, mu, t, dt, src, st);
        else launch_ell<MODE, false>(A, X, Y, M, f, mu, t, dt, src, st);
    } else if (!wide) {
        hipLaunchKernelGGL((fom_csr_kernel<MODE, false>), dim3((unsigned)blocks), dim3(kThr), 0, st, A.ptr, A.col,
                           A.val, X, Y, (int64_t)A.nrows, M, f, mu, t, dt, src);
    } else {
        hipLaunchKernelGGL((fom_csr_kernel<MODE, true>), dim3((unsigned)blocks), dim3(kThr), 0, st, A.ptr, A.col,
                           A.val, X, Y, (int64_t)A.nrows, M, f, mu, t, dt, src);
    }
    return hipGetLastError();
}

// ---- dense products ------------------------------------------------------

constexpr int kT = 64;     // output tile rows and columns
constexpr int kS = 16;     // reduction slab
constexpr int kLdS = kT + 2;

// part[z] (K1 x K2, column-major) = sum over rows n of slice z of
// P[n, i] Q[n, j].  Thread (tx, ty) = (tid % 16, tid / 16) owns rows
// i0 + 4 tx .. +3 and columns j0 + 4 ty .. +3 of the tile.
__global__ __launch_bounds__(kThr) void gemm_tn_kernel(const double *__restrict__ P, const double *__restrict__ Q,
                                                       int64_t N, int K1, int K2, int64_t nper,
                                                       double *__restrict__ part) {
    __shared__ double ps[kS][kLdS], qs[kS][kLdS];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int i0 = blockIdx.x * kT, j0 = blockIdx.y * kT;
    const int64_t nb = (int64_t)blockIdx.z * nper;
    const int64_t ne = std::min<int64_t>(nb + nper, N);
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int64_t n0 = nb; n0 < ne; n0 += kS) {
        // 16 x 64 slab of each operand: thread loads 4 elements of each
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + q * kThr;          // 0 .. 1023
            const int rr = idx >> 6, cc = idx & 63;
            const int64_t n = n0 + rr;
            const bool nok = n < ne;
            ps[rr][cc] = (nok && i0 + cc < K1) ? P[n * K1 + i0 + cc] : 0.0;
            qs[rr][cc] = (nok && j0 + cc < K2) ? Q[n * K2 + j0 + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int s = 0; s < kS; ++s) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = ps[s][4 * tx + u];
                b[u] = qs[s][4 * ty + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = acc[u][v] + a[u] * b[v];
        }
        __syncthreads();
    }
    double *C = part + (size_t)blockIdx.z * K1 * K2;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + 4 * tx + u, j = j0 + 4 * ty + v;
            if (i < K1 && j < K2) C[(size_t)j * K1 + i] = acc[u][v];
        }
}

// out[i] = sum_{z} part[z][i] in order z = 0, 1, ...
__global__ void sum_parts_kernel(const double *__restrict__ part, int nz, int64_t n, double *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = part[i];
        for (int z = 1; z < nz; ++z) s = s + part[(size_t)z * n + i];
        out[i] = s;
    }
}

// Y (N x K2, row-major) = X (N x K1, row-major) B (K1 x K2, column-major).
// Thread (tx, ty) owns rows n0 + 4 ty .. +3 and columns j0 + 4 tx .. +3.
__global__ __launch_bounds__(kThr) void gemm_nn_kernel(const double *__restrict__ X, const double *__restrict__ B,
                                                       int64_t N, int K1, int K2, double *__restrict__ Y) {
    __shared__ double xs[kS][kLdS], bs[kS][kLdS];     // xs[k][row], bs[k][col]
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * kT;
    const int j0 = blockIdx.y * kT;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int k0 = 0; k0 < K1; k0 += kS) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + q * kThr;
            // X slab: 64 rows x 16 k, k fastest in memory
            const int xr = idx >> 4, xk = idx & 15;
            const int64_t n = r0 + xr;
            xs[xk][xr] = (n < N && k0 + xk < K1) ? X[n * K1 + k0 + xk] : 0.0;
            // B slab: 16 k x 64 columns, k fastest in memory
            const int bc = idx >> 4, bk = idx & 15;
            bs[bk][bc] = (j0 + bc < K2 && k0 + bk < K1) ? B[(size_t)(j0 + bc) * K1 + k0 + bk] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int s = 0; s < kS; ++s) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = xs[s][4 * ty + u];
                b[u] = bs[s][4 * tx + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = acc[u][v] + a[u] * b[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t n = r0 + 4 * ty + u;
        if (n >= N) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + 4 * tx + v;
            if (j < K2) Y[n * K2 + j] = acc[u][v];
        }
    }
}

}  // namespace

hipError_t launch_fom_step(const FomCsr &Av, const FomCsr &As, const double *f, const double *mu, int M, int64_t n,
                           double dt, int source, double *V, double *S, hipStream_t st) {
    const double t = (double)n * dt;
    hipError_t e = launch_csr<1>(Av, S, V, M, f, mu, t, dt, source, st);
    if (e != hipSuccess) return e;
    return launch_csr<2>(As, V, S, M, nullptr, nullptr, t, dt, source, st);
}

hipError_t launch_fom_spmm(const FomCsr &A, const double *X, int M, double *Y, hipStream_t st) {
    return launch_csr<0>(A, X, Y, M, nullptr, nullptr, 0.0, 0.0, 0, st);
}

int gemm_tn_splits(int64_t N, int K1, int K2) {
    const int64_t tiles = (int64_t)((K1 + kT - 1) / kT) * ((K2 + kT - 1) / kT);
    int64_t z = (1024 + tiles - 1) / tiles;
    const int64_t zmax = std::max<int64_t>(1, (N + 4095) / 4096);     // at least 4096 rows a slice
    z = std::min<int64_t>(std::min<int64_t>(z, zmax), 1024);
    return (int)std::max<int64_t>(z, 1);
}

hipError_t launch_gemm_tn(const double *P, const double *Q, int64_t N, int K1, int K2, double *part, double *C,
                          hipStream_t st) {
    if (K1 <= 0 || K2 <= 0) return hipSuccess;
    const int z = gemm_tn_splits(N, K1, K2);
    const int64_t nper = ((N + z - 1) / z + kS - 1) / kS * kS;
    dim3 grid((K1 + kT - 1) / kT, (K2 + kT - 1) / kT, z);
    hipLaunchKernelGGL(gemm_tn_kernel, grid, dim3(kThr), 0, st, P, Q, N, K1, K2, nper, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)K1 * K2;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)blocks), dim3(256), 0, st, part, z, n, C);
    return hipGetLastError();
}

hipError_t launch_gemm_nn(const double *X, const double *B, int64_t N, int K1, int K2, double *Y, hipStream_t st) {
    if (N <= 0 || K2 <= 0) return hipSuccess;
    dim3 grid((unsigned)((N + kT - 1) / kT), (K2 + kT - 1) / kT);
    hipLaunchKernelGGL(gemm_nn_kernel, grid, dim3(kThr), 0, st, X, B, N, K1, K2, Y);
    return hipGetLastError();
}

}  // namespace rom
