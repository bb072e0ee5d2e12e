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
#include <type_traits>

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
// with the whole chip busy and no launch per step.
//
// Per half-step the rows go in passes of four 64-row blocks; in a pass lane
// l of every wave holds row l of each of the four blocks, and wave w sums
// the reduction quarter w for all four, so each k step issues four
// independent 256-byte loads (one per block); the loads of two batches of
// kBatch terms are in flight at once.  The four quarter sums of block j meet in LDS and wave j
// finishes them.  Per row this is exactly the single-sample kernel's
// arithmetic (the same quarters, chunks of kChunk terms, two-sums, combine
// order, forcing and double-float update, rounded once per half-step), so a
// sample's trajectory equals rom_step_rank1's bit for bit.  The state hi
// words pass through LDS to the other half-step.
constexpr int kRank1Rows = 4;          // rows per lane and field (K <= 1024)
typedef const __attribute__((address_space(1))) unsigned char gbyte;
typedef const __attribute__((address_space(1))) dev::f4 gf4;
typedef const __attribute__((address_space(1))) float gfloat;
constexpr int kBatch = 16;             // terms per batch of loads (two batches in flight)

// Operator loads of one batch: kBatch columns k0 + kBatch bi + t of the
// lane's rows of pass `pass` of A (rows x cols), into a[t][0..3].  Columns
// past the end load column cols - 1 (in bounds; their multiplier is 0).
// Column k's address is wave-uniform (scalar base), the lane's rows a 32-bit
// byte offset: no 64-bit address registers per load.  VEC: rows a multiple
// of 4, so a lane's four rows of a pass are 4 consecutive ones, one 16-byte
// load per term (1 KB per wave instruction); else one row from each of four
// 64-row blocks, 4-byte loads.
template <bool VEC>
__device__ __forceinline__ void issue_ops(const float *__restrict__ A, int rows, int cols, int pass, int k0, int bi,
                                          float (&a)[kBatch][4]) {
    const int lane = threadIdx.x & 63;
    unsigned ro[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)   // rows past the end read the last row(s) and are never finished
        ro[j] = 4u * (unsigned)(VEC ? min(256 * pass + 4 * lane, rows - 4) + j
                                    : min((4 * pass + j) * 64 + lane, rows - 1));
    const int kb = k0 + bi * kBatch;
#pragma unroll
    for (int t = 0; t < kBatch; ++t) {
        const int k = min(kb + t, cols - 1);
        gbyte *col = reinterpret_cast<gbyte *>(reinterpret_cast<uint64_t>(A + (size_t)k * rows));
        if constexpr (VEC) {
            const dev::f4 v = *reinterpret_cast<gf4 *>(col + ro[0]);
#pragma unroll
            for (int j = 0; j < 4; ++j) a[t][j] = v[j];
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) a[t][j] = *reinterpret_cast<gfloat *>(col + ro[j]);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

// The operand a pass reads: operator A (rows x cols), layout VEC.
struct R1Half {
    const float *A;
    int rows, cols;
};

// One half-step of the field with operator H.A: x (LDS, cols) is the other
// field, xo (LDS, rows) receives this field's new hi words; h are this
// lane's rows (one per pass).  FORCED adds b u.  ONE (both fields at most
// 256 rows, one pass): the register ring av holds the first two batches on
// entry (issued by the caller or the previous half-step), and while the last
// chunk is multiplied the first two batches of the next half-step (operator
// N.A, layout NVEC) are issued, so those loads are in flight across the
// reduction and the update.  Otherwise each pass issues its own first two
// batches.
template <bool FORCED, bool VEC, bool NVEC, bool ONE>
__device__ __forceinline__ void rank1_batch_half(const R1Half &H, const R1Half &N, const float *__restrict__ x,
                                                 float *__restrict__ xo, const float (&bq)[kRank1Rows], float uh,
                                                 float ul, float dt, float (&h)[kRank1Rows], float (&pH)[4][4][64],
                                                 float (&pL)[4][4][64], float (&av)[2][kBatch][4]) {
    static_assert(kChunk == 2 * kBatch, "a chunk is two batches");
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rows = H.rows, cols = H.cols;
    const int kq = (cols + 3) / 4;
    const int k0 = w * kq, k1 = min(cols, k0 + kq);
    const int nblk = (rows + 63) / 64;
    const int npass = ONE ? 1 : (nblk + 3) / 4;
    // chunks of this wave's terms k0 .. k1-1 (none if the range is empty)
    const int nch = k1 > k0 ? (k1 - k0 + kChunk - 1) / kChunk : 0;
    const int nk0 = w * ((N.cols + 3) / 4);   // the next half-step's first term of this wave
    for (int pass = 0; pass < npass; ++pass) {
        float hi[4], lo[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) hi[j] = lo[j] = 0.f;
        // Straight-line code, two batches of kBatch terms (one chunk) in
        // flight: batch i + 1's loads are issued before batch i's
        // multiply-adds.  A term past k1 has multiplier 0, which adds an
        // exact zero, so every batch takes the same instructions.
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        auto consume = [&](int bi, const float (&a)[kBatch][4]) {
            const int kb = k0 + bi * kBatch;
            float xx[kBatch];
#pragma unroll
            for (int t = 0; t < kBatch; ++t)   // a product, not a branch around the load
                xx[t] = x[min(kb + t, cols - 1)] * (kb + t < k1 ? 1.f : 0.f);
#pragma unroll
            for (int t = 0; t < kBatch; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[j] = fmaf(a[t][j], xx[t], acc[j]);
            __builtin_amdgcn_sched_barrier(0);
        };
        // end of a chunk: fold its FP32 sum into (hi, lo)
        auto fold = [&]() {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float s, e;
                dev::two_sum(hi[j], acc[j], s, e);
                hi[j] = s;
                lo[j] += e;
                acc[j] = 0.f;
            }
        };
        // the first two batches of the next half-step
        auto prefetch = [&](int bi) {
            if constexpr (ONE) issue_ops<NVEC>(N.A, N.rows, N.cols, 0, nk0, bi, av[bi]);
        };
        if constexpr (!ONE) {
            if (nch > 0) {
                issue_ops<VEC>(H.A, rows, cols, pass, k0, 0, av[0]);
                issue_ops<VEC>(H.A, rows, cols, pass, k0, 1, av[1]);
            }
        }
        for (int c = 0; c < nch - 1; ++c) {
            consume(2 * c, av[0]);
            issue_ops<VEC>(H.A, rows, cols, pass, k0, 2 * c + 2, av[0]);
            consume(2 * c + 1, av[1]);
            fold();
            issue_ops<VEC>(H.A, rows, cols, pass, k0, 2 * c + 3, av[1]);
        }
        if (nch > 0) {
            consume(2 * nch - 2, av[0]);
            prefetch(0);
            consume(2 * nch - 1, av[1]);
            fold();
            prefetch(1);
        } else {
            prefetch(0);
            prefetch(1);
        }
        // partial of pass row q (0..255) at pH[w][q / 64][q % 64]
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = VEC ? 4 * lane + j : 64 * j + lane;
            pH[w][q >> 6][q & 63] = hi[j];
            pL[w][q >> 6][q & 63] = lo[j];
        }
        __syncthreads();
        const int i = (4 * pass + w) * 64 + lane;       // wave w finishes block 4 pass + w
        if (i < rows) {
            float Hs = pH[0][w][lane], L = pL[0][w][lane];
            for (int q = 1; q < 4; ++q) {
                float s, e;
                dev::two_sum(Hs, pH[q][w][lane], s, e);
                Hs = s;
                L += e + pL[q][w][lane];
            }
            float F = 0.f, Fe = 0.f;
            if (FORCED) {
                const float bi = bq[pass];
                F = bi * uh;
                Fe = fmaf(bi, uh, -F) + bi * ul;
            }
            float hh = h[pass], ll = 0.f;
            dev::comp_update(hh, ll, Hs, L, F, Fe, dt);
            h[pass] = hh + ll;                  // rounded once per half-step
            xo[i] = h[pass];
        }
        __syncthreads();                        // partials read before the next pass writes them
    }
}

// VV / VS: Kv / Ks a multiple of 4 (16-byte operator loads for that
// half-step); ONE: Kv, Ks <= 256 (one pass per half-step).
template <bool VV, bool VS, bool ONE>
__global__ __launch_bounds__(256) void rank1_batch_f32(const float *__restrict__ Avs, const float *__restrict__ Asv,
                                                       const float *__restrict__ b, const double *__restrict__ mu,
                                                       int kv, int ks, double dt, int64_t n0, int64_t nsteps,
                                                       int src, float *__restrict__ V, float *__restrict__ S) {
    extern __shared__ float xsh[];
    __shared__ float pH[4][4][64], pL[4][4][64];
    float *xs = xsh, *xv = xsh + ks;           // S and V hi words
    const int m = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // lane's rows: (4 pass + w) * 64 + lane, pass = 0 .. kRank1Rows - 1
    float vh[kRank1Rows], sh[kRank1Rows], bq[kRank1Rows];
#pragma unroll
    for (int q = 0; q < kRank1Rows; ++q) {
        const int i = (4 * q + w) * 64 + lane;
        bq[q] = i < kv ? b[i] : 0.f;             // this lane's source rows, held for the run
        vh[q] = i < kv ? V[(size_t)m * kv + i] : 0.f;
        sh[q] = i < ks ? S[(size_t)m * ks + i] : 0.f;
        if (i < ks) xs[i] = sh[q];
    }
    const R1Half hv = {Avs, kv, ks}, hs = {Asv, ks, kv};
    // the ring: (one pass) the first two batches of the first velocity half-step
    float av[2][kBatch][4];
    if constexpr (ONE) {
        const int wq = __builtin_amdgcn_readfirstlane(w) * ((ks + 3) / 4);
        issue_ops<VV>(Avs, kv, ks, 0, wq, 0, av[0]);
        issue_ops<VV>(Avs, kv, ks, 0, wq, 1, av[1]);
    }
    const double mum = mu[m];
    __syncthreads();
    for (int64_t k = 0; k < nsteps; ++k) {
        const double u = dev::forcing(src, (double)(n0 + k) * dt, mum);
        const float uh = (float)u, ul = (float)(u - (double)uh);
        rank1_batch_half<true, VV, VS, ONE>(hv, hs, xs, xv, bq, uh, ul, (float)dt, vh, pH, pL, av);
        rank1_batch_half<false, VS, VV, ONE>(hs, hv, xv, xs, bq, 0.f, 0.f, (float)dt, sh, pH, pL, av);
    }
    __builtin_amdgcn_s_waitcnt(0);   // the last prefetch (never used) has landed
#pragma unroll
    for (int q = 0; q < kRank1Rows; ++q) {
        const int i = (4 * q + w) * 64 + lane;
        if (i < kv) V[(size_t)m * kv + i] = vh[q];
        if (i < ks) S[(size_t)m * ks + i] = sh[q];
    }
}

}  // namespace

hipError_t launch_rank1_batch(const Rank2Args &a, hipStream_t st) {
    if (a.kv > 256 * kRank1Rows || a.ks > 256 * kRank1Rows) return hipErrorInvalidValue;
    const size_t lds = sizeof(float) * (size_t)(a.kv + a.ks);
    const bool one = a.kv <= 256 && a.ks <= 256;
    auto pick = [&](auto vv, auto vs) {
        constexpr bool VV = decltype(vv)::value, VS = decltype(vs)::value;
        return one ? rank1_batch_f32<VV, VS, true> : rank1_batch_f32<VV, VS, false>;
    };
    using T = std::true_type;
    using F = std::false_type;
    auto f = (a.kv % 4 == 0) ? ((a.ks % 4 == 0) ? pick(T{}, T{}) : pick(T{}, F{}))
                             : ((a.ks % 4 == 0) ? pick(F{}, T{}) : pick(F{}, F{}));
    hipLaunchKernelGGL(f, dim3(a.M), dim3(256), lds, st, static_cast<const float *>(a.avs),
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
