// Rank-2 leapfrog stepper for large reduced sizes, FP32 operators and
// states: the panel schedule.
//
// Method: Sec. 2.4 eq. (2.5) for the staggered system of Sec. 3.1 eq. (3.3),
//     V <- V + dt (Avs S + b u(t_n; mu)^T)      then      S <- S + dt Asv V,
// with the probe QoI J_m += dt (c^T V_m)^2 after every velocity half-step.
//
// Why this schedule.  The other FP32 schedules keep something on chip for
// the whole run: the column blocks keep the states of their samples in LDS
// (Kv + Ks <= 4096 padded), the row-split kernels keep a group's state rows
// inside one XCD (K <= 2048), the resident kernel the operator (K <= 256).
// Above those sizes (the paper's scaling study reaches K = 4096) nothing is
// resident across half-steps: each half-step is one launch of a tiled
// matrix product on the FP32 matrix cores, 128 operator rows x 64 samples
// per workgroup, with the compensated state update, the forcing and the
// probe partial sums fused into its epilogue.  Two launches per step; the
// stream orders them, so no workgroup ever waits for another.
//
// Layouts (all zero padded, so the main loop has no bounds checks):
//   operator  A[r * ldA + k], row-major, rows padded to 128, k to 128
//             (velocity: Avs, Kvq x Ksq; stress: Asv, Ksq x Kvq);
//   states    hi and lo words, column-major with ld = rows padded to 128,
//             Mq = M rounded up to 64 columns (the caller's V and S are
//             copied in before the first step and hi + lo written back
//             after the last);
//   probe     per velocity half-step, one FP64 partial of c^T V per
//             (128-row tile, sample), summed by the next stress launch.
//
// Products: v_mfma_f32_16x16x4f32 (A lane l: row l % 16, term l / 16; B lane
// l: term l / 16, column l % 16; D lane l: rows 4 (l / 16) + 0..3 of column
// l % 16).  Within a 32-term chunk the MFMA k-step kk of lane group
// g = l / 16 takes term 8 g + kk, so each lane's 8 terms of a chunk are
// contiguous in LDS (two 16-byte reads per fragment).  FP32 chains of 64
// terms are folded into FP64 sums (the rounding level of the other FP32
// kernels); the update y = (hi + lo) + dt (P + b u) is FP64.
#include <algorithm>

#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

using dev::f4;

constexpr int kPM = 128;           // operator rows per workgroup tile
constexpr int kPN = 64;            // samples per workgroup tile
constexpr int kPK = 32;            // terms per staged chunk
constexpr int kPLd = kPK + 4;      // LDS row stride (floats): 4-bank shift per row
constexpr int kPThreads = 256;

struct PanelArgs {
    const float *A;                // operator, rows x kd row-major (ld kd)
    const float *X;                // hi words of the other field, kd x Mq (ld kd)
    float *Yh, *Yl;                // this field, rows x Mq (ld rows)
    const float *b;                // forcing vector (kv entries) or null
    const float *c;                // probe (kv entries) or null
    const double *mu;              // M
    double *yp;                    // probe partials [rows / 128][Mq]
    const double *yp_in;           // stress launch: partials of the velocity half-step
    double *J, *y;                 // stress launch: J (M, +=) and trace row, or null
    int rows, kd, kreal, M, Mq;    // kreal: unpadded rows of this field (b, c guards)
    int64_t n;                     // step index (forcing at t_n = n dt)
    double dt;
    int source;
};

// Tile of workgroup `bid`: consecutive row tiles with all their column tiles
// on one XCD (workgroups go to XCD bid % 8), so a row tile's operator panel
// is read from that XCD's L2 by all of its column tiles.
__device__ __forceinline__ bool panel_tile(int bid, int ntr, int ntc, int &rt, int &ct) {
    const int T = ntr * ntc, per = (T + 7) / 8;
    const int t = (bid % 8) * per + bid / 8;
    if (t >= T) return false;
    rt = t / ntc;
    ct = t % ntc;
    return true;
}

template <bool FORCED>
__global__ __launch_bounds__(kPThreads) void rank2_panel_kernel(PanelArgs a) {
    __shared__ __align__(16) float As[2][kPM * kPLd];
    __shared__ __align__(16) float Xs[2][kPN * kPLd];
    __shared__ double ysum[4][kPN];

    int rt, ct;
    if (!panel_tile(blockIdx.x, a.rows / kPM, a.Mq / kPN, rt, ct)) return;
    const int tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row0 = rt * kPM, col0 = ct * kPN;

    // stress launch: the probe of the velocity half-step just completed
    if constexpr (!FORCED) {
        if (a.yp_in != nullptr && rt == 0 && tid < kPN) {
            const int m = col0 + tid;
            if (m < a.M) {
                double yv = 0.0;
                for (int t = 0; t < a.kd / kPM; ++t) yv += a.yp_in[(size_t)t * a.Mq + m];
                if (a.J) a.J[m] += a.dt * (yv * yv);
                if (a.y) a.y[m] = yv;
            }
        }
    }

    // staging: chunk k0 of the operator rows (4 float4 per thread) and of
    // the state columns (2 per thread), 8 threads per 32-term row
    const int sr = tid >> 3, sk = (tid & 7) * 4;
    const float *Ag = a.A + (size_t)(row0 + sr) * a.kd + sk;
    const float *Xg = a.X + (size_t)(col0 + sr) * a.kd + sk;
    const size_t astep = (size_t)32 * a.kd;     // 32 rows further
    f4 ra[4], rx[2];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[q] = *reinterpret_cast<const f4 *>(Ag + q * astep + k0);
#pragma unroll
        for (int q = 0; q < 2; ++q) rx[q] = *reinterpret_cast<const f4 *>(Xg + q * astep + k0);
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<f4 *>(&As[buf][(sr + 32 * q) * kPLd + sk]) = ra[q];
#pragma unroll
        for (int q = 0; q < 2; ++q) *reinterpret_cast<f4 *>(&Xs[buf][(sr + 32 * q) * kPLd + sk]) = rx[q];
    };

    f4 acc[2][4];
    double acc64[2][4][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            acc[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[rb][cb][v] = 0.0;
        }
    auto fold = [&]() {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc64[rb][cb][v] += (double)acc[rb][cb][v];
                acc[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
            }
    };

    // fragments: lane l reads terms 8 (l / 16) .. + 7 of row / column l % 16
    const int fr = l & 15, fk = (l >> 4) * 8;
    const int nch = a.kd / kPK;
    fetch(0);
    stage(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) fetch((ch + 1) * kPK);
        f4 fa[2][2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const float *p = &As[buf][(32 * w + 16 * rb + fr) * kPLd + fk];
            fa[rb][0] = *reinterpret_cast<const f4 *>(p);
            fa[rb][1] = *reinterpret_cast<const f4 *>(p + 4);
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const float *p = &Xs[buf][(16 * cb + fr) * kPLd + fk];
            const f4 fb0 = *reinterpret_cast<const f4 *>(p);
            const f4 fb1 = *reinterpret_cast<const f4 *>(p + 4);
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const float xb = kk < 4 ? fb0[kk & 3] : fb1[kk & 3];
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    const float xa = kk < 4 ? fa[rb][0][kk & 3] : fa[rb][1][kk & 3];
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa, xb, acc[rb][cb], 0, 0, 0);
                }
            }
        }
        if (ch + 1 < nch) stage(buf ^ 1);
        if (ch & 1) fold();
        __syncthreads();
    }
    if (nch & 1) fold();

    // ---- epilogue: compensated update of 4 consecutive rows per (rb, cb)
    const double dt = a.dt;
    double ypart[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int m = col0 + 16 * cb + fr;
        double u = 0.0;
        if constexpr (FORCED) u = m < a.M ? dev::forcing(a.source, (double)a.n * dt, a.mu[m]) : 0.0;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int r = row0 + 32 * w + 16 * rb + 4 * (l >> 4);
            const size_t o = (size_t)m * a.rows + r;
            f4 hh = *reinterpret_cast<const f4 *>(a.Yh + o);
            f4 ll = *reinterpret_cast<const f4 *>(a.Yl + o);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double inc = acc64[rb][cb][v];
                if constexpr (FORCED) {
                    const double br = r + v < a.kreal ? (double)a.b[r + v] : 0.0;
                    inc = fma(br, u, inc);
                }
                const double yv = fma(dt, inc, (double)hh[v] + (double)ll[v]);
                const float hv = (float)yv;
                hh[v] = hv;
                ll[v] = (float)(yv - (double)hv);
                if constexpr (FORCED) {
                    if (a.c != nullptr && r + v < a.kreal) ypart[cb] += (double)a.c[r + v] * yv;
                }
            }
            *reinterpret_cast<f4 *>(a.Yh + o) = hh;
            *reinterpret_cast<f4 *>(a.Yl + o) = ll;
        }
    }
    if constexpr (FORCED) {
        if (a.c != nullptr) {
            // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the same column: fold them,
            // then the four waves meet in LDS (the tile's 128 rows)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                ypart[cb] += __shfl_xor(ypart[cb], 16, 64);
                ypart[cb] += __shfl_xor(ypart[cb], 32, 64);
            }
            if (l < 16) {
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) ysum[w][16 * cb + l] = ypart[cb];
            }
            __syncthreads();
            if (tid < kPN) {
                const double s = (ysum[0][tid] + ysum[1][tid]) + (ysum[2][tid] + ysum[3][tid]);
                a.yp[(size_t)rt * a.Mq + col0 + tid] = s;
            }
        }
    }
}

// Pack a column-major FP32 matrix (rows x cols, ld rows) into the row-major
// padded panel operator: dst[r * ldd + k] = src[k * rows + r], zero outside.
__global__ void panel_pack_op_kernel(const float *__restrict__ src, int rows, int cols, int rowsq, int ldd,
                                     float *__restrict__ dst) {
    const int64_t n = (int64_t)rowsq * ldd;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / ldd), k = (int)(i % ldd);
        dst[i] = (r < rows && k < cols) ? src[(size_t)k * rows + r] : 0.f;
    }
}

// Caller state (rows x M, ld rows) -> hi words (rowsq x Mq) and zero lo words.
__global__ void panel_state_in_kernel(const float *__restrict__ src, int rows, int M, int rowsq, int Mq,
                                      float *__restrict__ hi, float *__restrict__ lo) {
    const int64_t n = (int64_t)rowsq * Mq;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(i / rowsq), r = (int)(i % rowsq);
        hi[i] = (r < rows && m < M) ? src[(size_t)m * rows + r] : 0.f;
        lo[i] = 0.f;
    }
}

// hi + lo -> caller state.
__global__ void panel_state_out_kernel(const float *__restrict__ hi, const float *__restrict__ lo, int rows, int M,
                                       int rowsq, float *__restrict__ dst) {
    const int64_t n = (int64_t)rows * M;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(i / rows), r = (int)(i % rows);
        const size_t o = (size_t)m * rowsq + r;
        dst[i] = hi[o] + lo[o];
    }
}

int grid_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 4096); }

}  // namespace

int panel_pad(int k) { return round_up(k, kPM); }

size_t panel_op_bytes(int kv, int ks) { return sizeof(float) * (size_t)panel_pad(kv) * panel_pad(ks); }

size_t panel_ws_bytes(int kv, int ks, int M) {
    const size_t Mq = (size_t)round_up(M, kPN);
    return sizeof(float) * 2 * Mq * ((size_t)panel_pad(kv) + panel_pad(ks))   // hi, lo of V and S
           + sizeof(double) * (size_t)(panel_pad(kv) / kPM) * Mq;             // probe partials
}

hipError_t launch_panel_pack(const float *avs_cm, const float *asv_cm, int kv, int ks, float *avs_rm,
                             float *asv_rm, hipStream_t st) {
    const int kvq = panel_pad(kv), ksq = panel_pad(ks);
    hipLaunchKernelGGL(panel_pack_op_kernel, dim3(grid_for((int64_t)kvq * ksq)), dim3(256), 0, st, avs_cm, kv, ks,
                       kvq, ksq, avs_rm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(panel_pack_op_kernel, dim3(grid_for((int64_t)kvq * ksq)), dim3(256), 0, st, asv_cm, ks, kv,
                       ksq, kvq, asv_rm);
    return hipGetLastError();
}

// The whole run: states in, nsteps x (velocity launch, stress launch),
// states out.  ws holds panel_ws_bytes(kv, ks, M).
hipError_t launch_rank2_panel(const float *avs_rm, const float *asv_rm, const Rank2Args &r2, void *ws,
                              hipStream_t st) {
    const int kvq = panel_pad(r2.kv), ksq = panel_pad(r2.ks), Mq = round_up(r2.M, kPN);
    float *Vh = static_cast<float *>(ws);
    float *Vl = Vh + (size_t)kvq * Mq;
    float *Sh = Vl + (size_t)kvq * Mq;
    float *Sl = Sh + (size_t)ksq * Mq;
    double *yp = reinterpret_cast<double *>(Sl + (size_t)ksq * Mq);
    hipError_t e;
    hipLaunchKernelGGL(panel_state_in_kernel, dim3(grid_for((int64_t)kvq * Mq)), dim3(256), 0, st,
                       static_cast<const float *>(r2.V), r2.kv, r2.M, kvq, Mq, Vh, Vl);
    hipLaunchKernelGGL(panel_state_in_kernel, dim3(grid_for((int64_t)ksq * Mq)), dim3(256), 0, st,
                       static_cast<const float *>(r2.S), r2.ks, r2.M, ksq, Mq, Sh, Sl);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    const bool probe = r2.c != nullptr;
    PanelArgs v{};
    v.A = avs_rm; v.X = Sh; v.Yh = Vh; v.Yl = Vl;
    v.b = static_cast<const float *>(r2.b); v.c = static_cast<const float *>(r2.c); v.mu = r2.mu;
    v.yp = yp; v.rows = kvq; v.kd = ksq; v.kreal = r2.kv; v.M = r2.M; v.Mq = Mq;
    v.dt = r2.dt; v.source = r2.source;
    PanelArgs s{};
    s.A = asv_rm; s.X = Vh; s.Yh = Sh; s.Yl = Sl;
    s.yp_in = probe ? yp : nullptr; s.J = r2.J;
    s.rows = ksq; s.kd = kvq; s.kreal = r2.ks; s.M = r2.M; s.Mq = Mq; s.dt = r2.dt; s.source = r2.source;
    const int gv = 8 * ((kvq / kPM * (Mq / kPN) + 7) / 8), gs = 8 * ((ksq / kPM * (Mq / kPN) + 7) / 8);
    for (int64_t k = 0; k < r2.nsteps; ++k) {
        v.n = r2.n0 + k;
        hipLaunchKernelGGL(rank2_panel_kernel<true>, dim3(gv), dim3(kPThreads), 0, st, v);
        s.n = r2.n0 + k;
        s.y = r2.y ? r2.y + (size_t)k * r2.M : nullptr;
        hipLaunchKernelGGL(rank2_panel_kernel<false>, dim3(gs), dim3(kPThreads), 0, st, s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(panel_state_out_kernel, dim3(grid_for((int64_t)r2.kv * r2.M)), dim3(256), 0, st, Vh, Vl,
                       r2.kv, r2.M, kvq, static_cast<float *>(r2.V));
    hipLaunchKernelGGL(panel_state_out_kernel, dim3(grid_for((int64_t)r2.ks * r2.M)), dim3(256), 0, st, Sh, Sl,
                       r2.ks, r2.M, ksq, static_cast<float *>(r2.S));
    return hipGetLastError();
}

}  // namespace rom
