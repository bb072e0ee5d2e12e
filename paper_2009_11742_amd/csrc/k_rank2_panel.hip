// Rank-2 leapfrog stepper for large reduced sizes: the panel schedule, for
// FP32 operators and states and for FP64 states.
//
// Method: Sec. 2.4 eq. (2.5) for the staggered system of Sec. 3.1 eq. (3.3),
//     V <- V + dt (Avs S + b u(t_n; mu)^T)      then      S <- S + dt Asv V,
// with the probe QoI J_m += dt (c^T V_m)^2 after every velocity half-step.
//
// Why this schedule.  The other schedules keep something on chip for the
// whole run: the column blocks keep the states of their samples in LDS
// (FP32: Kv + Ks <= 4096 padded; FP64 on the vector ALUs: about 4800), the
// row-split kernels keep a group's state rows inside one XCD (K <= 2048),
// the resident kernel the operator (K <= 256).  Above those sizes (the
// paper's scaling study reaches K = 4096) nothing is resident across
// half-steps: each half-step is one launch of a tiled matrix product on the
// matrix cores, 128 operator rows x 64 samples per workgroup, with the state
// update, the forcing and the probe partial sums fused into its epilogue.
// Two launches per step; the stream orders them, so no workgroup ever waits
// for another.  With few tiles (small M) the k range is split over more
// workgroups, which write FP64 partial products; a second launch sums them
// and updates.
//
// Layouts (all zero padded, so the main loop has no bounds checks):
//   operator  A[r * ldA + k], row-major, rows padded to 128, k to 128
//             (velocity: Avs, Kvq x Ksq; stress: Asv, Ksq x Kvq);
//   states    column-major with ld = rows padded to 128, Mq = M rounded up
//             to 64 columns; FP32: hi and lo words (the caller's V and S are
//             copied in before the first step and hi + lo written back after
//             the last); FP64: the values;
//   probe     per velocity half-step, one FP64 partial of c^T V per
//             (128-row tile, sample), summed by the next stress launch.
//
// Products: v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64 (A lane l: row
// l % 16, term l / 16; B lane l: term l / 16, column l % 16; D lane l,
// entry v: column l % 16, row 4 (l / 16) + v for FP32, (l / 16) + 4 v for
// FP64).  Chunks of 32 FP32 / 16 FP64 terms
// (128 bytes per row) are staged through LDS; within a chunk the MFMA
// k-step kk of lane group g = l / 16 takes term (chunk / 4) g + kk, so each
// lane's terms of a chunk are contiguous in LDS (two 16-byte reads per
// fragment).  FP32: chains of 64 terms are folded into FP64 sums (the
// rounding level of the other FP32 kernels) and the update
// y = (hi + lo) + dt (P + b u) is FP64; FP64: plain FP64 throughout.
#include <algorithm>
#include <type_traits>

#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

using dev::f4;
typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kPM = 128;           // operator rows per workgroup tile
constexpr int kPN = 64;            // samples per workgroup tile
constexpr int kPThreads = 256;

// Element type traits: 16-byte vector, terms per staged chunk (128 bytes
// per row), MFMA accumulator.
template <typename T> struct Pt;
template <> struct Pt<float> {
    using V = f4;                  // 4 terms per 16 bytes
    using Acc = f4;
    static constexpr int VW = 4, BK = 32;
    static __device__ __forceinline__ Acc mfma(float a, float b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Pt<double> {
    using V = d2;
    using Acc = d4;
    static constexpr int VW = 2, BK = 16;
    static __device__ __forceinline__ Acc mfma(double a, double b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

template <typename T>
struct PanelArgs {
    const T *A;                    // operator, rows x kd row-major (ld kd)
    const T *X;                    // the other field (FP32: hi words), kd x Mq (ld kd)
    T *Yh;                         // this field (FP32: hi words), rows x Mq (ld rows)
    float *Yl;                     // FP32: lo words of this field; FP64: unused
    const T *b;                    // forcing vector (kv entries) or null
    const T *c;                    // probe (kv entries) or null
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
template <typename T>
__device__ __forceinline__ void probe_reduce(const PanelArgs<T> &a, int col0, int nrt, int tid) {
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

// Four consecutive state entries (16-byte aligned) in and out.
template <typename T>
__device__ __forceinline__ void load4(const T *p, T (&h)[4]) {
    if constexpr (std::is_same<T, float>::value) {
        const f4 v = *reinterpret_cast<const f4 *>(p);
        h[0] = v[0]; h[1] = v[1]; h[2] = v[2]; h[3] = v[3];
    } else {
        const d2 v0 = reinterpret_cast<const d2 *>(p)[0], v1 = reinterpret_cast<const d2 *>(p)[1];
        h[0] = v0.x; h[1] = v0.y; h[2] = v1.x; h[3] = v1.y;
    }
}
template <typename T>
__device__ __forceinline__ void store4(T *p, const T (&h)[4]) {
    if constexpr (std::is_same<T, float>::value) {
        *reinterpret_cast<f4 *>(p) = f4{h[0], h[1], h[2], h[3]};
    } else {
        reinterpret_cast<d2 *>(p)[0] = d2{h[0], h[1]};
        reinterpret_cast<d2 *>(p)[1] = d2{h[2], h[3]};
    }
}

// New value of one state entry: y + dt (P + b u) in FP64; FP32 keeps it as
// the (hi, lo) pair.
template <typename T>
__device__ __forceinline__ double update_entry(double P, double br, double u, double dt, T &h, float &l) {
    const double inc = fma(br, u, P);
    if constexpr (std::is_same<T, float>::value) {
        const double yv = fma(dt, inc, (double)h + (double)l);
        h = (float)yv;
        l = (float)(yv - (double)h);
        return yv;
    } else {
        const double yv = fma(dt, inc, h);
        h = yv;
        return yv;
    }
}

// SPLIT: workgroup (tile, s) sums the s-th of nsplit k-ranges and writes
// its FP64 partials; panel_finish_kernel then does the update.
template <typename T, bool FORCED, bool SPLIT>
__global__ __launch_bounds__(kPThreads) void rank2_panel_kernel(PanelArgs<T> a) {
    using V = typename Pt<T>::V;
    using Acc = typename Pt<T>::Acc;
    constexpr int VW = Pt<T>::VW, BK = Pt<T>::BK, LD = BK + VW;   // LDS row: 16-byte shift per row
    constexpr int TPL = BK / 4;                                  // terms per lane per chunk
    constexpr bool F32 = std::is_same<T, float>::value;
    __shared__ __align__(16) T As[2][kPM * LD];
    __shared__ __align__(16) T Xs[2][kPN * LD];
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

    // staging: 16 bytes per thread per 32-row step; 8 threads per row of a
    // chunk (4 steps of the operator rows, 2 of the state columns)
    const int sr = tid >> 3, sk = (tid & 7) * VW;
    const int nall = a.kd / BK;
    const int c0 = SPLIT ? ks * nall / a.nsplit : 0;
    const int nch = SPLIT ? (ks + 1) * nall / a.nsplit - c0 : nall;
    const T *Ag = a.A + (size_t)(row0 + sr) * a.kd + (size_t)c0 * BK + sk;
    const T *Xg = a.X + (size_t)(col0 + sr) * a.kd + (size_t)c0 * BK + sk;
    const size_t astep = (size_t)32 * a.kd;     // 32 rows further
    V ra[4], rx[2];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[q] = *reinterpret_cast<const V *>(Ag + q * astep + k0);
#pragma unroll
        for (int q = 0; q < 2; ++q) rx[q] = *reinterpret_cast<const V *>(Xg + q * astep + k0);
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<V *>(&As[buf][(sr + 32 * q) * LD + sk]) = ra[q];
#pragma unroll
        for (int q = 0; q < 2; ++q) *reinterpret_cast<V *>(&Xs[buf][(sr + 32 * q) * LD + sk]) = rx[q];
    };

    Acc acc[2][4];
    double acc64[2][4][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            acc[rb][cb] = Acc{0, 0, 0, 0};
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[rb][cb][v] = 0.0;
        }
    // FP32: FP32 chains of 64 terms folded into FP64 sums
    auto fold = [&]() {
        if constexpr (F32) {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc64[rb][cb][v] += (double)acc[rb][cb][v];
                    acc[rb][cb] = Acc{0, 0, 0, 0};
                }
        }
    };

    // fragments: lane l reads terms TPL (l / 16) .. + TPL - 1 of row / column l % 16
    const int fr = l & 15, fk = (l >> 4) * TPL;
    fetch(0);
    stage(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) fetch((ch + 1) * BK);
        V fa[2][2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const T *p = &As[buf][(32 * w + 16 * rb + fr) * LD + fk];
            fa[rb][0] = *reinterpret_cast<const V *>(p);
            fa[rb][1] = *reinterpret_cast<const V *>(p + VW);
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const T *p = &Xs[buf][(16 * cb + fr) * LD + fk];
            const V fb0 = *reinterpret_cast<const V *>(p);
            const V fb1 = *reinterpret_cast<const V *>(p + VW);
#pragma unroll
            for (int kk = 0; kk < TPL; ++kk) {
                const T xb = kk < VW ? fb0[kk % VW] : fb1[kk % VW];
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    const T xa = kk < VW ? fa[rb][0][kk % VW] : fa[rb][1][kk % VW];
                    acc[rb][cb] = Pt<T>::mfma(xa, xb, acc[rb][cb]);
                }
            }
        }
        if (ch + 1 < nch) stage(buf ^ 1);
        if (ch & 1) fold();
        __syncthreads();
    }
    if constexpr (F32) {
        if (nch & 1) fold();
    } else {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc64[rb][cb][v] = acc[rb][cb][v];
    }

    // Output rows of a lane's 4 accumulator entries v within a 16 x 16
    // block: FP32 4 (l / 16) + v (consecutive), FP64 (l / 16) + 4 v (the
    // FP64 instruction's layout, checked on the device).
    constexpr int RS = F32 ? 1 : 4;
    const int rl = F32 ? 4 * (l >> 4) : (l >> 4);

    if constexpr (SPLIT) {
        // FP64 partials of the lane's 4 rows per (rb, cb)
        double *pp = a.part + (size_t)ks * a.Mq * a.rows;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const int m = col0 + 16 * cb + fr, r = row0 + 32 * w + 16 * rb + rl;
                double *d = pp + (size_t)m * a.rows + r;
                if constexpr (F32) {
                    reinterpret_cast<d2 *>(d)[0] = d2{acc64[rb][cb][0], acc64[rb][cb][1]};
                    reinterpret_cast<d2 *>(d)[1] = d2{acc64[rb][cb][2], acc64[rb][cb][3]};
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) d[RS * v] = acc64[rb][cb][v];
                }
            }
        return;
    }

    // ---- epilogue: update of the lane's 4 rows per (rb, cb)
    const double dt = a.dt;
    double ypart[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int m = col0 + 16 * cb + fr;
        double u = 0.0;
        if constexpr (FORCED) u = m < a.M ? dev::forcing(a.source, (double)a.n * dt, a.mu[m]) : 0.0;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int r = row0 + 32 * w + 16 * rb + rl;
            const size_t o = (size_t)m * a.rows + r;
            T hh[4];
            float ll[4] = {0.f, 0.f, 0.f, 0.f};
            if constexpr (F32) {
                load4(a.Yh + o, hh);
                load4(a.Yl + o, ll);
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) hh[v] = a.Yh[o + RS * v];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rv = r + RS * v;
                const double br = (FORCED && rv < a.kreal) ? (double)a.b[rv] : 0.0;
                const double yv = update_entry<T>(acc64[rb][cb][v], br, u, dt, hh[v], ll[v]);
                if constexpr (FORCED) {
                    if (a.c != nullptr && rv < a.kreal) ypart[cb] += (double)a.c[rv] * yv;
                }
            }
            if constexpr (F32) {
                store4(a.Yh + o, hh);
                store4(a.Yl + o, ll);
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) a.Yh[o + RS * v] = hh[v];
            }
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
// accesses and a half-wave sum for the probe).  Eight workgroups per tile,
// so a launch with few tiles still spreads its partial reads over the chip.
template <typename T, bool FORCED>
__global__ __launch_bounds__(kPThreads) void panel_finish_kernel(PanelArgs<T> a) {
    constexpr bool F32 = std::is_same<T, float>::value;
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
    const int m = col0 + 8 * jb + (tid >> 5);
    const size_t o = (size_t)m * a.rows + r;
    double P[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = 0; q < a.nsplit; ++q) {
        const d2 *p = reinterpret_cast<const d2 *>(a.part + q * plane + o);
        const d2 p0 = p[0], p1 = p[1];
        P[0] += p0.x; P[1] += p0.y; P[2] += p1.x; P[3] += p1.y;
    }
    double u = 0.0;
    if constexpr (FORCED) u = m < a.M ? dev::forcing(a.source, (double)a.n * dt, a.mu[m]) : 0.0;
    T hh[4];
    float ll[4] = {0.f, 0.f, 0.f, 0.f};
    load4(a.Yh + o, hh);
    if constexpr (F32) load4(a.Yl + o, ll);
    double yp = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double br = (FORCED && r + v < a.kreal) ? (double)a.b[r + v] : 0.0;
        const double yv = update_entry<T>(P[v], br, u, dt, hh[v], ll[v]);
        if constexpr (FORCED) {
            if (a.c != nullptr && r + v < a.kreal) yp += (double)a.c[r + v] * yv;
        }
    }
    store4(a.Yh + o, hh);
    if constexpr (F32) store4(a.Yl + o, ll);
    if constexpr (FORCED) {
        if (a.c != nullptr) {
#pragma unroll
            for (int off = 1; off < 32; off <<= 1) yp += __shfl_xor(yp, off, 64);
            if (h == 0) a.yp[(size_t)rt * a.Mq + m] = yp;
        }
    }
}

// Pack a column-major matrix (rows x cols, ld rows) into the row-major
// padded panel operator: dst[r * ldd + k] = src[k * rows + r], zero outside.
template <typename T>
__global__ void panel_pack_op_kernel(const T *__restrict__ src, int rows, int cols, int rowsq, int ldd,
                                     T *__restrict__ dst) {
    const int64_t n = (int64_t)rowsq * ldd;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / ldd), k = (int)(i % ldd);
        dst[i] = (r < rows && k < cols) ? src[(size_t)k * rows + r] : T(0);
    }
}

// Caller state (rows x M, ld rows) -> padded state (rowsq x Mq), FP32 with
// zero lo words.
template <typename T>
__global__ void panel_state_in_kernel(const T *__restrict__ src, int rows, int M, int rowsq, int Mq,
                                      T *__restrict__ hi, float *__restrict__ lo) {
    const int64_t n = (int64_t)rowsq * Mq;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(i / rowsq), r = (int)(i % rowsq);
        hi[i] = (r < rows && m < M) ? src[(size_t)m * rows + r] : T(0);
        if (lo) lo[i] = 0.f;
    }
}

// Padded state (FP32: hi + lo) -> caller state.
template <typename T>
__global__ void panel_state_out_kernel(const T *__restrict__ hi, const float *__restrict__ lo, int rows, int M,
                                       int rowsq, T *__restrict__ dst) {
    const int64_t n = (int64_t)rows * M;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(i / rows), r = (int)(i % rows);
        const size_t o = (size_t)m * rowsq + r;
        dst[i] = lo ? T(hi[o] + lo[o]) : hi[o];
    }
}

int grid_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 4096); }

// k-range splits of a half-step with `rows` output rows and kd terms, a
// power of two with at least 256 terms per split.  Below 256 tiles (one
// workgroup per CU) the product is split until tiles x splits reaches 256,
// at most 16 ways (measured against splitting up to 512 work items: 108
// against 141 us per step at K = 4096, M = 64).  From 256 tiles on, S in
// {1, 2, 4} minimising ceil(T S / 256) / S, the time of the busiest CU
// when each takes its share of items of 1 / S the work (smaller S on ties):
// 288 tiles (K = 2304, M = 1024) split 4 ways, 364 -> 283 us per step; 384
// (K = 3072, M = 1024) 2 ways, 481 -> 410; 256 and 512 stay whole.
int panel_splits(int rows, int kd, int Mq) {
    const int T = rows / kPM * (Mq / kPN);
    int S = 1;
    if (T < 256) {
        while (S < 16 && S * T < 256 && kd >= 256 * 2 * S) S *= 2;
        return S;
    }
    double best = 1e30;
    for (int s = 1; s <= 4 && kd >= 256 * s; s *= 2) {
        const double c = (double)((T * s + 255) / 256) / s;
        if (c < best - 1e-9) { best = c; S = s; }
    }
    return S;
}

template <typename T>
hipError_t run_panel_typed(const T *avs_rm, const T *asv_rm, const Rank2Args &r2, void *ws, hipStream_t st) {
    constexpr bool F32 = std::is_same<T, float>::value;
    const int kvq = panel_pad(r2.kv), ksq = panel_pad(r2.ks), Mq = round_up(r2.M, kPN);
    T *Vh = static_cast<T *>(ws);
    T *Sh = Vh + (size_t)kvq * Mq;
    float *Vl = reinterpret_cast<float *>(Sh + (size_t)ksq * Mq);
    float *Sl = Vl + (F32 ? (size_t)kvq * Mq : 0);
    double *yp = reinterpret_cast<double *>(Sl + (F32 ? (size_t)ksq * Mq : 0));
    double *part = yp + (size_t)(kvq / kPM) * Mq;
    hipError_t e;
    hipLaunchKernelGGL(panel_state_in_kernel<T>, dim3(grid_for((int64_t)kvq * Mq)), dim3(256), 0, st,
                       static_cast<const T *>(r2.V), r2.kv, r2.M, kvq, Mq, Vh, F32 ? Vl : nullptr);
    hipLaunchKernelGGL(panel_state_in_kernel<T>, dim3(grid_for((int64_t)ksq * Mq)), dim3(256), 0, st,
                       static_cast<const T *>(r2.S), r2.ks, r2.M, ksq, Mq, Sh, F32 ? Sl : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    const bool probe = r2.c != nullptr;
    PanelArgs<T> v{};
    v.A = avs_rm; v.X = Sh; v.Yh = Vh; v.Yl = Vl;
    v.b = static_cast<const T *>(r2.b); v.c = static_cast<const T *>(r2.c); v.mu = r2.mu;
    v.yp = yp; v.rows = kvq; v.kd = ksq; v.kreal = r2.kv; v.M = r2.M; v.Mq = Mq;
    v.dt = r2.dt; v.source = r2.source;
    PanelArgs<T> s{};
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
            hipLaunchKernelGGL((rank2_panel_kernel<T, true, false>), grid(tv), dim3(kPThreads), 0, st, v);
        } else {
            hipLaunchKernelGGL((rank2_panel_kernel<T, true, true>), grid(tv * v.nsplit), dim3(kPThreads), 0, st, v);
            hipLaunchKernelGGL((panel_finish_kernel<T, true>), dim3(8 * tv), dim3(kPThreads), 0, st, v);
        }
        s.n = r2.n0 + k;
        s.y = r2.y ? r2.y + (size_t)k * r2.M : nullptr;
        if (s.nsplit == 1) {
            hipLaunchKernelGGL((rank2_panel_kernel<T, false, false>), grid(ts), dim3(kPThreads), 0, st, s);
        } else {
            hipLaunchKernelGGL((rank2_panel_kernel<T, false, true>), grid(ts * s.nsplit), dim3(kPThreads), 0, st, s);
            hipLaunchKernelGGL((panel_finish_kernel<T, false>), dim3(8 * ts), dim3(kPThreads), 0, st, s);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(panel_state_out_kernel<T>, dim3(grid_for((int64_t)r2.kv * r2.M)), dim3(256), 0, st, Vh,
                       F32 ? Vl : nullptr, r2.kv, r2.M, kvq, static_cast<T *>(r2.V));
    hipLaunchKernelGGL(panel_state_out_kernel<T>, dim3(grid_for((int64_t)r2.ks * r2.M)), dim3(256), 0, st, Sh,
                       F32 ? Sl : nullptr, r2.ks, r2.M, ksq, static_cast<T *>(r2.S));
    return hipGetLastError();
}

}  // namespace

int panel_pad(int k) { return round_up(k, kPM); }

size_t panel_op_bytes(int kv, int ks, bool f64) {
    return (f64 ? sizeof(double) : sizeof(float)) * (size_t)panel_pad(kv) * panel_pad(ks);
}

size_t panel_ws_bytes(int kv, int ks, int M, bool f64) {
    const int kvq = panel_pad(kv), ksq = panel_pad(ks), Mq = round_up(M, kPN);
    const size_t sv = panel_splits(kvq, ksq, Mq), ss = panel_splits(ksq, kvq, Mq);
    const size_t part = std::max(sv > 1 ? sv * kvq : 0, ss > 1 ? ss * ksq : 0) * (size_t)Mq;
    const size_t states = (size_t)Mq * ((size_t)kvq + ksq);
    return (f64 ? sizeof(double) * states : 2 * sizeof(float) * states)   // values (FP32: hi, lo)
           + sizeof(double) * (size_t)(kvq / kPM) * Mq                   // probe partials
           + sizeof(double) * part;                                      // split partial products
}

hipError_t launch_panel_pack(const void *avs_cm, const void *asv_cm, int kv, int ks, bool f64, void *avs_rm,
                             void *asv_rm, hipStream_t st) {
    const int kvq = panel_pad(kv), ksq = panel_pad(ks);
    const dim3 g(grid_for((int64_t)kvq * ksq));
    if (f64) {
        hipLaunchKernelGGL(panel_pack_op_kernel<double>, g, dim3(256), 0, st, static_cast<const double *>(avs_cm), kv,
                           ks, kvq, ksq, static_cast<double *>(avs_rm));
        hipLaunchKernelGGL(panel_pack_op_kernel<double>, g, dim3(256), 0, st, static_cast<const double *>(asv_cm), ks,
                           kv, ksq, kvq, static_cast<double *>(asv_rm));
    } else {
        hipLaunchKernelGGL(panel_pack_op_kernel<float>, g, dim3(256), 0, st, static_cast<const float *>(avs_cm), kv,
                           ks, kvq, ksq, static_cast<float *>(avs_rm));
        hipLaunchKernelGGL(panel_pack_op_kernel<float>, g, dim3(256), 0, st, static_cast<const float *>(asv_cm), ks,
                           kv, ksq, kvq, static_cast<float *>(asv_rm));
    }
    return hipGetLastError();
}

// The whole run: states in, nsteps x (velocity launch(es), stress
// launch(es)), states out.  ws holds panel_ws_bytes(kv, ks, M, f64).
hipError_t launch_rank2_panel(const void *avs_rm, const void *asv_rm, const Rank2Args &r2, bool f64, void *ws,
                              hipStream_t st) {
    if (f64)
        return run_panel_typed<double>(static_cast<const double *>(avs_rm), static_cast<const double *>(asv_rm), r2,
                                       ws, st);
    return run_panel_typed<float>(static_cast<const float *>(avs_rm), static_cast<const float *>(asv_rm), r2, ws, st);
}

}  // namespace rom
