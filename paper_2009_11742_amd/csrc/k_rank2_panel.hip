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
    double *part;                  // split launches: FP64 partial products [nsplit][Mq][rows]
    int nsplit;                    // k-range splits (1: products and update in one launch)
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

// Stress launches (the update's or the finishing one): the probe of the
// velocity half-step just completed, for the tile's columns: the FP64 sum
// of the row-tile partials in tile order, J += dt y^2 and the trace entry.
__device__ __forceinline__ void probe_reduce(const PanelArgs &a, int col0, int nrt, int tid) {
    if (a.yp_in != nullptr && tid < kPN) {
        const int m = col0 + tid;
        if (m < a.M) {
            double yv = 0.0;
            for (int t = 0; t < nrt; ++t) yv += a.yp_in[(size_t)t * a.Mq + m];
            if (a.J) a.J[m] += a.dt * (yv * yv);
            if (a.y) a.y[m] = yv;
        }
    }
}

// SPLIT: workgroup (tile, s) sums the s-th of nsplit k-ranges and writes
// its FP64 partials; panel_finish_kernel then does the update.
template <bool FORCED, bool SPLIT>
__global__ __launch_bounds__(kPThreads) void rank2_panel_kernel(PanelArgs a) {
    __shared__ __align__(16) float As[2][kPM * kPLd];
    __shared__ __align__(16) float Xs[2][kPN * kPLd];
    __shared__ double ysum[4][kPN];

    int rt, ct, ks = 0;
    if constexpr (SPLIT) {
        // (row tile, split) pairs count as rows of the tile order: the
        // column tiles of one operator segment share an XCD
        int rs;
        if (!panel_tile(blockIdx.x, a.rows / kPM * a.nsplit, a.Mq / kPN, rs, ct)) return;
        rt = rs / a.nsplit;
        ks = rs % a.nsplit;
    } else {
        if (!panel_tile(blockIdx.x, a.rows / kPM, a.Mq / kPN, rt, ct)) return;
    }
    const int tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row0 = rt * kPM, col0 = ct * kPN;

    if constexpr (!FORCED && !SPLIT) {
        if (rt == 0) probe_reduce(a, col0, a.kd / kPM, tid);
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
    // this workgroup's chunks: [c0, c0 + nch) of the kd / 32
    const int nall = a.kd / kPK;
    const int c0 = SPLIT ? ks * nall / a.nsplit : 0;
    const int nch = SPLIT ? (ks + 1) * nall / a.nsplit - c0 : nall;
    Ag += (size_t)c0 * kPK;
    Xg += (size_t)c0 * kPK;
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

    if constexpr (SPLIT) {
        // FP64 partials of 4 consecutive rows per (rb, cb)
        double *pp = a.part + (size_t)ks * a.Mq * a.rows;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const int m = col0 + 16 * cb + fr, r = row0 + 32 * w + 16 * rb + 4 * (l >> 4);
                double2 *d = reinterpret_cast<double2 *>(pp + (size_t)m * a.rows + r);
                d[0] = double2{acc64[rb][cb][0], acc64[rb][cb][1]};
                d[1] = double2{acc64[rb][cb][2], acc64[rb][cb][3]};
            }
        return;
    }

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

// Update of a split half-step: as the one-launch epilogue, with P the sum
// of the nsplit FP64 partials in split order.  Workgroup b takes 8 columns
// (8 (b % 8) .. of tile b / 8) of the tile's 128 rows; thread t rows
// 4 (t % 32) .. + 3 of column t / 32 (each half-wave one column: coalesced
// 16-byte accesses and a half-wave sum for the probe).  Eight workgroups
// per tile, so a launch with few tiles still spreads its partial reads over
// the chip.
template <bool FORCED>
__global__ __launch_bounds__(kPThreads) void panel_finish_kernel(PanelArgs a) {
    const int ntc = a.Mq / kPN, tile = blockIdx.x / 8, jb = blockIdx.x % 8;
    const int rt = tile / ntc, ct = tile % ntc;
    const int tid = threadIdx.x, h = tid & 31;
    const int row0 = rt * kPM, col0 = ct * kPN;
    if constexpr (!FORCED) {
        if (rt == 0 && jb == 0) probe_reduce(a, col0, a.kd / kPM, tid);
    }
    const double dt = a.dt;
    const int r = row0 + 4 * h;
    const size_t plane = (size_t)a.Mq * a.rows;
    {
        const int m = col0 + 8 * jb + (tid >> 5);
        const size_t o = (size_t)m * a.rows + r;
        double P[4] = {0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < a.nsplit; ++q) {
            const double2 *p = reinterpret_cast<const double2 *>(a.part + q * plane + o);
            const double2 p0 = p[0], p1 = p[1];
            P[0] += p0.x; P[1] += p0.y; P[2] += p1.x; P[3] += p1.y;
        }
        double u = 0.0;
        if constexpr (FORCED) u = m < a.M ? dev::forcing(a.source, (double)a.n * dt, a.mu[m]) : 0.0;
        f4 hh = *reinterpret_cast<const f4 *>(a.Yh + o);
        f4 ll = *reinterpret_cast<const f4 *>(a.Yl + o);
        double yp = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double inc = P[v];
            if constexpr (FORCED) {
                const double br = r + v < a.kreal ? (double)a.b[r + v] : 0.0;
                inc = fma(br, u, inc);
            }
            const double yv = fma(dt, inc, (double)hh[v] + (double)ll[v]);
            const float hv = (float)yv;
            hh[v] = hv;
            ll[v] = (float)(yv - (double)hv);
            if constexpr (FORCED) {
                if (a.c != nullptr && r + v < a.kreal) yp += (double)a.c[r + v] * yv;
            }
        }
        *reinterpret_cast<f4 *>(a.Yh + o) = hh;
        *reinterpret_cast<f4 *>(a.Yl + o) = ll;
        if constexpr (FORCED) {
            if (a.c != nullptr) {
#pragma unroll
                for (int off = 1; off < 32; off <<= 1) yp += __shfl_xor(yp, off, 64);
                if (h == 0) a.yp[(size_t)rt * a.Mq + m] = yp;
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

namespace {

// k-range splits of a half-step with `rows` output rows and kd terms: below
// 256 tiles (one workgroup per CU) the product is split until tiles x
// splits reaches 256, with at least 8 chunks (256 terms) per split and at
// most 16 splits; a power of two.  (Measured against splitting up to 512
// work items: 108 against 141 us per step at K = 4096, M = 64, and 194
// against 206 at K = 2048, M = 1024, which 256 tiles fill unsplit.)
int panel_splits(int rows, int kd, int Mq) {
    const int T = rows / kPM * (Mq / kPN);
    int S = 1;
    while (S < 16 && S * T < 256 && kd / kPK >= 8 * 2 * S) S *= 2;
    return S;
}

}  // namespace

size_t panel_op_bytes(int kv, int ks) { return sizeof(float) * (size_t)panel_pad(kv) * panel_pad(ks); }

size_t panel_ws_bytes(int kv, int ks, int M) {
    const int kvq = panel_pad(kv), ksq = panel_pad(ks), Mq = round_up(M, kPN);
    const size_t sv = panel_splits(kvq, ksq, Mq), ss = panel_splits(ksq, kvq, Mq);
    const size_t part = std::max(sv > 1 ? sv * kvq : 0, ss > 1 ? ss * ksq : 0) * (size_t)Mq;
    return sizeof(float) * 2 * (size_t)Mq * ((size_t)kvq + ksq)       // hi, lo of V and S
           + sizeof(double) * (size_t)(kvq / kPM) * Mq                 // probe partials
           + sizeof(double) * part;                                    // split partial products
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
    double *part = yp + (size_t)(kvq / kPM) * Mq;
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
    v.part = s.part = part;
    v.nsplit = panel_splits(kvq, ksq, Mq);
    s.nsplit = panel_splits(ksq, kvq, Mq);
    // launch grids: 8 ceil(items / 8) (panel_tile deals items to XCDs)
    auto grid = [](int items) { return dim3(8 * ((items + 7) / 8)); };
    const int tv = kvq / kPM * (Mq / kPN), ts = ksq / kPM * (Mq / kPN);
    for (int64_t k = 0; k < r2.nsteps; ++k) {
        v.n = r2.n0 + k;
        if (v.nsplit == 1) {
            hipLaunchKernelGGL((rank2_panel_kernel<true, false>), grid(tv), dim3(kPThreads), 0, st, v);
        } else {
            hipLaunchKernelGGL((rank2_panel_kernel<true, true>), grid(tv * v.nsplit), dim3(kPThreads), 0, st, v);
            hipLaunchKernelGGL(panel_finish_kernel<true>, dim3(8 * tv), dim3(kPThreads), 0, st, v);
        }
        s.n = r2.n0 + k;
        s.y = r2.y ? r2.y + (size_t)k * r2.M : nullptr;
        if (s.nsplit == 1) {
            hipLaunchKernelGGL((rank2_panel_kernel<false, false>), grid(ts), dim3(kPThreads), 0, st, s);
        } else {
            hipLaunchKernelGGL((rank2_panel_kernel<false, true>), grid(ts * s.nsplit), dim3(kPThreads), 0, st, s);
            hipLaunchKernelGGL(panel_finish_kernel<false>, dim3(8 * ts), dim3(kPThreads), 0, st, s);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(panel_state_out_kernel, dim3(grid_for((int64_t)r2.kv * r2.M)), dim3(256), 0, st, Vh, Vl,
                       r2.kv, r2.M, kvq, static_cast<float *>(r2.V));
    hipLaunchKernelGGL(panel_state_out_kernel, dim3(grid_for((int64_t)r2.ks * r2.M)), dim3(256), 0, st, Sh, Sl,
                       r2.ks, r2.M, ksq, static_cast<float *>(r2.S));
    return hipGetLastError();
}

}  // namespace rom
