// Rank-2 leapfrog stepper, row-split schedule: low-precision (BF16 /
// FP8-E4M3) operators, FP32 states.
//
// Method: Sec. 2.4 eq. (2.5) for the staggered system of Sec. 3.1 eq. (3.3),
// one step being  V <- V + dt (Avs S + b u(t_n; mu)^T),  S <- S + dt Asv V.
//
// Why a second schedule.  The column-block kernels give every workgroup a
// few sample columns and the whole operator, so each CU streams the full
// operator every step; with BF16 / FP8 operators at K = 1024 that stream
// (4 MB / 2 MB per step per CU) bounds the step far above the MFMA time.
// Here the operator rows are split instead: the workgroups of a column
// group (kRows = 64 rows each, R = K / 64 of them) cover K rows of both
// fields for a group of samples: 16, 32 or 64 columns (the narrowest whose
// workgroups all fit on the chip; kCols = 64 sizes the buffers).  Each keeps
// its operator rows in
// registers for the whole run (every wave holds a quarter of the reduction
// of both fields as BF16 MFMA fragments: 256 registers per lane at K =
// 1024), so no operator bytes move after the start.  The price is one
// exchange per half-step: a workgroup publishes its updated rows, as the
// BF16 (hi, lo) pair the products consume, and the group meets at a
// barrier before the other half-step reads them.
//
// The exchange stays inside one XCD: a workgroup reads the XCD it runs on
// (HW_REG_XCC_ID) and takes a group slot on that XCD with an atomic, so a
// group's members share an L2 and the exchange needs no L2 write-back or
// invalidate, only each wave's L1 invalidated after the barrier.  The
// launch is cooperative (all workgroups resident; one per CU); every wait
// is bounded, and a wait that runs out sets ROM_E_TIMEOUT in the status
// word and makes every later wait return at once, so the kernel always ends.
//
// Products: v_mfma_f32_16x16x32_bf16 (A lane l: row l % 16, terms
// 8 (l / 16) .. +7; B lane l: terms 8 (l / 16) .. +7, column l % 16;
// D register r of lane l: row 4 (l / 16) + r, column l % 16).  Wave w of a
// workgroup sums reduction terms [w kp/4, (w+1) kp/4) for all 64 x 64
// outputs, with the state operand fed as x_hi + x_lo (two MFMAs; x_hi alone,
// one MFMA, in the single-pass variant, which also publishes x_hi only); the four
// FP32 partials meet in LDS, where each thread finishes 16 outputs: their
// FP32 sum, then in FP64 the scale (FP8), forcing and the update of the
// FP32 (hi, lo) state.
#include <mutex>
#include <type_traits>
#include <string>

#include "k_common.h"
#include "rom_internal.h"

namespace rom {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
using dev::f4;

constexpr int kRows = 64;          // rows per workgroup tile
constexpr int kCols = 64;          // sample columns per group
constexpr int kWaves = 4;
constexpr int kThreads = 256;
constexpr int kLd = kRows + 4;     // LDS column stride (floats)
constexpr long kSpinMax = 1L << 20;     // polls of one bounded wait
constexpr int kCntStride = 64;     // counters 256 bytes apart
constexpr int kXcds = 8, kCusPerXcd = 32;

__device__ __forceinline__ bf8 as_bf8(u4 v) { return __builtin_bit_cast(bf8, v); }

// A 64-bit value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

struct SplitArgs {
    const u4 *opv, *ops;        // packed BF16 fragments of Avs and Asv
    const float *b, *c;         // source (kv), probe (kv) or null
    const double *mu;
    float *V, *S;               // caller states, ld kv / ks
    double *J, *y;
    unsigned short *xv, *xs;    // exchange, BF16 in MFMA B-fragment order (see frag_offset)
    double *yp;                 // probe partials [group][row tile][col]
    unsigned *cnt;              // group counters, kCntStride apart
    unsigned *slots;            // per-XCD slot counters (8)
    int *status;                // status[1] <- ROM_E_TIMEOUT
    float *vtr, *str;           // FP32 traced runs: state traces (entry e, sample m, row: [e][m][row])
    const double *ytr;          // adjoint runs: forward probe trace [step][m]
    float *wtr, *qtr;           // adjoint runs: P after / Q before each step's P update
    double *dmu;                // adjoint runs: += dt (b^T P) du/dmu
    const SplitGroup *grp;      // grouped FP32 runs: per-group instance data, from grp[g0]
    const int *smap;            // grouped FP32 runs: slot map (see rank2_split_f32_kernel)
    int g0;
    int source;                 // source signal (dev::Source)
    // bounded waits: poll budget (kSpinMax), and a bias added to every
    // barrier target (0; 1 makes every first wait run out, the host-forced
    // time-out of the failure-handling tests)
    long spin_max;
    unsigned wait_bias;
    int kv, kp, M, G, R;
    int64_t n0, nsteps;
    double dt;
    float scale;
};

// Group barrier number `phase` (1, 2, ...): publish-side stores of this
// workgroup are complete when every thread has passed s_waitcnt; thread 0
// counts the workgroup in and waits for the whole group.
__device__ __forceinline__ void group_barrier(const SplitArgs &a, unsigned *cnt, unsigned target) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        long spins = 0;
        target += a.wait_bias;
        while (__hip_atomic_load(&a.status[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
               __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > a.spin_max) {
                __hip_atomic_store(&a.status[1], (int)ROM_E_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&a.status[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __syncthreads();
    // The group's rows were written through other CUs' L1s into the shared
    // L2.  This CU's L1 may still hold the lines of its previous read of the
    // same addresses, so every read of data other workgroups wrote (exchange
    // fragments, probe partials) is a device-scope load (XBuf, ld_shared),
    // which the L1 does not serve.  An L1 invalidate here would do too, but only in
    // its agent-scope form (the workgroup-scope one does not reach the L1
    // outside threadgroup-split mode), and that one costs several us per
    // barrier.
}

// Probe partials of one column: the R row tiles' values at p[q * stride],
// read with device-scope loads (other workgroups wrote them), kProbeBatch at
// a time per thread, all in flight before the first is used (entries past R
// re-read entry R - 1 and are not added; four keep the register pressure of
// the kernels' time loop where it was).
constexpr int kProbeBatch = 4;

// Their sum, spread over the TPC consecutive threads of the column: thread
// fs reads the partials q = fs, fs + TPC, .. (four at a time, all in flight
// together: one round trip to L2 for R <= 4 TPC instead of R / 4), sums
// them in increasing q, and the TPC threads meet in a butterfly; every one
// of them returns the column's total.  All TPC threads must call it.
template <int TPC>
__device__ __forceinline__ double sum_partials_spread(const double *p, int stride, int R, int fs) {
    double y = 0.0;
    for (int q0 = fs; q0 < R; q0 += kProbeBatch * TPC) {
        double v[kProbeBatch];
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q)
            v[q] = __hip_atomic_load(p + (size_t)min(q0 + q * TPC, R - 1) * stride, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q)
            if (q0 + q * TPC < R) y += v[q];
    }
#pragma unroll
    for (int off = 1; off < TPC; off <<= 1) y += __shfl_xor(y, off, 64);
    return y;
}

// Forcing of a window of kUWin steps for the group's NC columns, in LDS:
// u[s][j] = u(t_{n + s}; mu of column col0 + j) (zero past M), evaluated by
// all threads together once per window, so each step reads its column's
// value instead of evaluating the source (whose exp constants would
// otherwise be held, and spilled, across the time loop).
constexpr int kUWin = 16;
template <int NC>
__device__ __forceinline__ void forcing_window(double *u, int src, int64_t n, double dt, const double *mu, int col0,
                                               int M) {
    for (int idx = threadIdx.x; idx < kUWin * NC; idx += kThreads) {
        const int s = idx / NC, j = idx - s * NC, m = col0 + j;
        u[idx] = m < M ? dev::forcing(src, (double)(n + s) * dt, mu[m]) : 0.0;
    }
}

// Adjoint amplitude window: u[s][j] = 2 y(step r0 - s, column col0 + j)
// for the kUWin iterations from r0 down (zero before the segment or past M):
// the reverse sweep's source amplitude, from the forward probe trace.
template <int NC>
__device__ __forceinline__ void adjoint_window(double *u, const double *ytr, int64_t r0, int col0, int M) {
    for (int idx = threadIdx.x; idx < kUWin * NC; idx += kThreads) {
        const int s = idx / NC, j = idx - s * NC, m = col0 + j;
        const int64_t r = r0 - s;
        u[idx] = (m < M && r >= 0) ? 2.0 * ytr[(size_t)r * M + m] : 0.0;
    }
}

// Products of one half-step for wave w: acc[rb][cb] (rows 16 rb.., columns
// 16 cb..) = sum over this wave's KB k-blocks of op fragments x (x_hi + x_lo).
// x points at the group's exchange block of the other field.  The B
// fragments of k-block kb are loaded kDepth k-blocks ahead into a register
// ring; the loop is fully unrolled (static fragment indices) and
// sched_barriers keep every load batch ahead of the MFMAs it must precede,
// which the scheduler would otherwise sink next to their use under this
// kernel's register pressure.
constexpr int kDepth = 2;

// Exchange layout: per group of NCB 16-column blocks, [k-block (kp/32)]
// [column block (NCB)][hi | lo][lane (64)][8 terms], lane = 16 ((k % 32) / 8)
// + column % 16 -- exactly the B fragments, so one wave load reads 1 KB
// contiguous.  Offset (in BF16 elements) of fragment (kb, cb, hl) within a
// group's block:
template <int NCB>
__device__ __forceinline__ size_t frag_offset(int kb, int cb, int hl) {
    return ((size_t)(kb * NCB + cb) * 2 + hl) * 512;
}

// Global memory bytes: with a wave-uniform base and an unsigned 32-bit lane
// offset, loads take the scalar-base + vector-offset form and need no 64-bit
// address registers (the FP32 operator stream).
typedef const __attribute__((address_space(1))) unsigned char gbyte;

// A group's exchange block, read with 16-byte buffer loads under the
// device-scope cache policy (sc1): the vector L1 does not serve them from
// lines it kept from an earlier read of the same addresses, which other
// workgroups have rewritten since.  The base is wave-uniform; offsets are in
// bytes, and one past the block reads zeros (the buffer's bound) instead of
// faulting.
constexpr int kDeviceScope = 16;             // cache-policy bit SC1
constexpr int kRawBufferWord3 = 0x00020000;  // untyped 32-bit data format
struct XBuf {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ XBuf(uint64_t base, unsigned bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(base), (short)0, (int)bytes, kRawBufferWord3)) {}
    __device__ __forceinline__ u4 ld(unsigned off) const {
        return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kDeviceScope);
    }
};

// The same guarantee as two relaxed device-scope 8-byte loads
// (global_load_dwordx2 ... sc1), which the FP32 kernel's long unrolled
// k-group loop schedules better (measured: 41 against 48 us per step at K =
// M = 1024; the BF16 kernel is faster with XBuf).
typedef const __attribute__((address_space(1))) unsigned long long gu64;
__device__ __forceinline__ u4 ld_shared(gbyte *p) {
    const gu64 *q = reinterpret_cast<const gu64 *>(p);
    const unsigned long long lo = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long hi = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return u4{(unsigned)lo, (unsigned)(lo >> 32), (unsigned)hi, (unsigned)(hi >> 32)};
}

template <bool SINGLE, int NCB>
__device__ __forceinline__ void load_b(const XBuf &xg, int kb, unsigned loff, u4 (&bh)[NCB], u4 (&bl)[NCB]) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        bh[cb] = xg.ld(2u * (unsigned)frag_offset<NCB>(kb, cb, 0) + loff);
        if constexpr (!SINGLE) bl[cb] = xg.ld(2u * (unsigned)frag_offset<NCB>(kb, cb, 1) + loff);
    }
}

// Ring depth in k-blocks (measured at K = 1024: the single-operand kernel
// with 64-column groups takes 7.2 us per step at depth 2, 7.5 at 3 and 7.7
// at 4; the pair 10.6 at 2 and 10.7 at 3 or 4), deeper only for the
// narrower pair groups.
template <int KB, bool SINGLE, int NCB>
constexpr int ring_depth() {
    constexpr int d = (SINGLE || NCB == 4) ? kDepth : 3;
    return KB < d ? KB : d;
}

template <int KB, bool SINGLE, int NCB>
__device__ __forceinline__ void products(const u4 (&op)[4][KB], const unsigned short *x, unsigned xbytes, int w,
                                         int lane, f4 (&acc)[4][NCB]) {
    constexpr int D = ring_depth<KB, SINGLE, NCB>();
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
    // The fragment addresses are the same every step; without this opaque
    // redefinition of the base the compiler hoists all of them out of the
    // time loop and spills them.
    uint64_t bits = reinterpret_cast<uint64_t>(x);
    asm volatile("" : "+s"(bits));
    const XBuf xg(bits, xbytes);
    // this wave's k-blocks are w KB .. w KB + KB - 1 of the group's block
    const int kb0 = w * KB;
    const unsigned loff = 16u * (unsigned)lane;
    u4 rh[D][NCB], rl[D][NCB];
#pragma unroll
    for (int d = 0; d < D; ++d) load_b<SINGLE, NCB>(xg, kb0 + d, loff, rh[d], rl[d]);
    __builtin_amdgcn_sched_barrier(0);
    // Column block by column block: the MFMAs of k-block kb that read a ring
    // slot's column-block fragments are issued, then that column block's
    // fragments of k-block kb + D are loaded into the same registers.  The
    // ring needs no copies of the fragments in use, and each load still has
    // the rest of this k-block and all of the next ahead of its use.
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int slot = kb % D;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const bf8 A = as_bf8(op[rb][kb]);
                acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, as_bf8(rh[slot][cb]), acc[rb][cb], 0, 0, 0);
                if constexpr (!SINGLE)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, as_bf8(rl[slot][cb]), acc[rb][cb], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            if (kb + D < KB) {
                rh[slot][cb] = xg.ld(2u * (unsigned)frag_offset<NCB>(kb0 + kb + D, cb, 0) + loff);
                if constexpr (!SINGLE) rl[slot][cb] = xg.ld(2u * (unsigned)frag_offset<NCB>(kb0 + kb + D, cb, 1) + loff);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// NCB: 16-column blocks per group (NC = 16 NCB samples).  Finishing
// threads: TPC = 256 / NC per column, each owning RPT = 4 NCB consecutive rows
// of the tile, published in runs of 8 rows (one lane's B fragment) or 4 (half
// of one).
template <int KB, bool SINGLE, int NCB>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void rank2_split_kernel(SplitArgs a) {
    static_assert(NCB == 1 || NCB == 2 || NCB == 4, "16, 32 or 64 columns per group");
    constexpr int NC = 16 * NCB, TPC = kThreads / NC, RPT = 4 * NCB;
    extern __shared__ __align__(16) unsigned char smem[];
    float *sth = reinterpret_cast<float *>(smem);          // [field][col][kLd] hi
    float *stl = sth + 2 * NC * kLd;                     // lo
    float *part = stl + 2 * NC * kLd;                    // [wave][col][kLd]
    float *bl = part + kWaves * NC * kLd;                // own rows of b
    float *cl = bl + kRows;                                 // own rows of c
    __shared__ int sh_slot;
    __shared__ double uwin[kUWin * NC];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kp = a.kp, R = a.R;

    // ---- group slot on this workgroup's XCD
    if (tid == 0) {
        const unsigned xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u;   // HW_REG_XCC_ID
        const unsigned s = __hip_atomic_fetch_add(&a.slots[xcc], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sh_slot = (int)(xcc + 8u * s);
    }
    __syncthreads();
    const int code = __builtin_amdgcn_readfirstlane(sh_slot);
    const int xcc = code & 7, s = code >> 3;
    const int r = s % R;                       // row tile
    const int g = (s / R) * 8 + xcc;           // group, interleaved over the XCDs
    if (g >= a.G) return;                      // idle workgroup (never counted)
    const int col0 = g * NC;
    unsigned *cnt = a.cnt + (size_t)g * kCntStride;
    unsigned phase = 0;

    // ---- operator fragments (registers for the whole run)
    u4 opv[4][KB], ops[4][KB];
    {
        const u4 *pv = a.opv + ((size_t)(r * kWaves + w) * 4 * KB) * 64 + lane;
        const u4 *ps = a.ops + ((size_t)(r * kWaves + w) * 4 * KB) * 64 + lane;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                opv[rb][kb] = pv[(rb * KB + kb) * 64];
                ops[rb][kb] = ps[(rb * KB + kb) * 64];
            }
    }

    // ---- own tiles of V and S, b, c
    const int row0 = r * kRows;
    for (int idx = tid; idx < 2 * NC * kRows; idx += kThreads) {
        const int f = idx / (NC * kRows), rem = idx - f * NC * kRows;
        const int j = rem / kRows, i = rem - j * kRows;
        const int m = col0 + j, row = row0 + i;
        const float *src = f == 0 ? a.V : a.S;
        float v = 0.f;
        if (m < a.M && row < a.kv) v = src[(size_t)m * a.kv + row];
        sth[(f * NC + j) * kLd + i] = v;
        stl[(f * NC + j) * kLd + i] = 0.f;
    }
    for (int i = tid; i < kRows; i += kThreads) {
        const int row = row0 + i;
        bl[i] = row < a.kv ? a.b[row] : 0.f;
        cl[i] = (a.c != nullptr && row < a.kv) ? a.c[row] : 0.f;
    }
    __syncthreads();

    // finishing thread: column fj, rows RPT fs .. RPT fs + RPT - 1
    const int fj = tid / TPC, fs = tid % TPC;
    const int fm = col0 + fj;
    const bool fok = fm < a.M;

    // publish rows of field f (hi words) as BF16 (hi, lo) into x, in the
    // B-fragment order: tile row o of column fj is term o % 8 of lane
    // 16 ((o % 32) / 8) + fj % 16 of k-block (row0 + o) / 32, column block
    // fj / 16 (row0 is a multiple of 32)
    // (value i of the thread's RPT rows from `hv`: the LDS tile, or the
    // finishing loop's registers)
    auto publish = [&](int f, unsigned short *x, auto hv) {
        constexpr int CH = RPT < 8 ? RPT : 8;      // rows per store
        (void)f;
        unsigned short *xg = x + (size_t)g * NC * 2 * kp;
        const int cb = fj / 16;
#pragma unroll
        for (int c = 0; c < RPT / CH; ++c) {
            unsigned ph[CH / 2], pl[CH / 2];
#pragma unroll
            for (int q = 0; q < CH / 2; ++q) {
                // hardware round-to-nearest-even, two values per instruction
                const f2 v = {hv(CH * c + 2 * q), hv(CH * c + 2 * q + 1)};
                const bf2 hi = __builtin_convertvector(v, bf2);
                const f2 r = v - __builtin_convertvector(hi, f2);
                const bf2 lo = __builtin_convertvector(r, bf2);
                ph[q] = __builtin_bit_cast(unsigned, hi);
                pl[q] = __builtin_bit_cast(unsigned, lo);
            }
            const int o = RPT * fs + CH * c;
            const int kb = (row0 + o) / 32, ln = 16 * ((o % 32) / 8) + (fj & 15);
            unsigned short *dh = xg + frag_offset<NCB>(kb, cb, 0) + 8 * ln + o % 8;
            unsigned short *dl = xg + frag_offset<NCB>(kb, cb, 1) + 8 * ln + o % 8;
            if constexpr (CH == 8) {
                *reinterpret_cast<u4 *>(dh) = u4{ph[0], ph[1], ph[2], ph[3]};
                if constexpr (!SINGLE) *reinterpret_cast<u4 *>(dl) = u4{pl[0], pl[1], pl[2], pl[3]};
            } else {
                typedef unsigned int u2 __attribute__((ext_vector_type(2)));
                *reinterpret_cast<u2 *>(dh) = u2{ph[0], ph[1]};
                if constexpr (!SINGLE) *reinterpret_cast<u2 *>(dl) = u2{pl[0], pl[1]};
            }
        }
    };

    // products -> LDS partials -> finished rows (FP64 update) -> published
    auto half_step = [&](int f, const u4 (&op)[4][KB], const unsigned short *xother, unsigned short *xmine,
                         const double *up, bool forced) -> double {
        f4 acc[4][NCB];
        products<KB, SINGLE, NCB>(op, xother + (size_t)g * NC * 2 * kp, 2u * NC * 2 * kp, w, lane, acc);
        float *pw = part + w * NC * kLd;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
                *reinterpret_cast<f4 *>(pw + (16 * cb + (lane & 15)) * kLd + 16 * rb + 4 * (lane >> 4)) = acc[rb][cb];
        __syncthreads();
        const double u = forced ? *up : 0.0;
        double ypart = 0.0;
        float *h = sth + (f * NC + fj) * kLd + RPT * fs;
        float *l = stl + (f * NC + fj) * kLd + RPT * fs;
        float hn[RPT];                             // the new hi words, published below
#pragma unroll
        for (int q = 0; q < RPT / 4; ++q) {
            f4 p0 = *reinterpret_cast<const f4 *>(part + (0 * NC + fj) * kLd + RPT * fs + 4 * q);
            f4 p1 = *reinterpret_cast<const f4 *>(part + (1 * NC + fj) * kLd + RPT * fs + 4 * q);
            f4 p2 = *reinterpret_cast<const f4 *>(part + (2 * NC + fj) * kLd + RPT * fs + 4 * q);
            f4 p3 = *reinterpret_cast<const f4 *>(part + (3 * NC + fj) * kLd + RPT * fs + 4 * q);
            f4 hh = *reinterpret_cast<const f4 *>(h + 4 * q);
            f4 ll = *reinterpret_cast<const f4 *>(l + 4 * q);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = RPT * fs + 4 * q + e;
                // the wave partials are FP32 chain sums; one more FP32 rounding is
                // far below the BF16 state operand's
                double inc = (double)((p0[e] + p1[e]) + (p2[e] + p3[e])) * (double)a.scale;
                if (forced) inc = fma((double)bl[i], u, inc);
                const double yv = fma(a.dt, inc, (double)hh[e] + (double)ll[e]);
                const float hv = (float)yv;
                hh[e] = hv;
                ll[e] = (float)(yv - (double)hv);
                if (forced) ypart += (double)cl[i] * yv;
            }
            *reinterpret_cast<f4 *>(h + 4 * q) = hh;
            *reinterpret_cast<f4 *>(l + 4 * q) = ll;
#pragma unroll
            for (int e = 0; e < 4; ++e) hn[4 * q + e] = hh[e];
        }
        publish(f, xmine, [&](int i) { return hn[i]; });
        return ypart;
    };

    // ---- initial exchange: S rows (the first half-step reads S)
    {
        const float *h0 = sth + (1 * NC + fj) * kLd + RPT * fs;
        publish(1, a.xs, [&](int i) { return h0[i]; });
    }
    group_barrier(a, cnt, (unsigned)R * ++phase);

    double Jacc = 0.0;
    const bool probe = a.c != nullptr;
    for (int64_t k = 0; k < a.nsteps; ++k) {
        if (k % kUWin == 0) forcing_window<NC>(uwin, a.source, a.n0 + k, a.dt, a.mu, col0, a.M);
        // (read after the products' barrier inside half_step)
        double yp = half_step(0, opv, a.xs, a.xv, uwin + (k % kUWin) * NC + fj, true);
        if (probe) {
            // sum the TPC strips of column fj, then publish this tile's partial
#pragma unroll
            for (int off = 1; off < TPC; off <<= 1) yp += __shfl_xor(yp, off, 64);
            if (fs == 0) a.yp[((size_t)g * R + r) * NC + fj] = yp;
        }
        group_barrier(a, cnt, (unsigned)R * ++phase);
        if (probe && r == 0 && fok) {
            // the R row-tile partials, spread over the column's threads
            const double yv = sum_partials_spread<TPC>(a.yp + (size_t)g * R * NC + fj, NC, R, fs);
            if (fs == 0) {
                Jacc += a.dt * (yv * yv);
                if (a.y) a.y[(size_t)k * a.M + fm] = yv;
            }
        }
        half_step(1, ops, a.xv, a.xs, nullptr, false);
        group_barrier(a, cnt, (unsigned)R * ++phase);
    }

    // ---- write back (hi + lo), J
    for (int idx = tid; idx < 2 * NC * kRows; idx += kThreads) {
        const int f = idx / (NC * kRows), rem = idx - f * NC * kRows;
        const int j = rem / kRows, i = rem - j * kRows;
        const int m = col0 + j, row = row0 + i;
        if (m < a.M && row < a.kv) {
            float *dst = f == 0 ? a.V : a.S;
            dst[(size_t)m * a.kv + row] = sth[(f * NC + j) * kLd + i] + stl[(f * NC + j) * kLd + i];
        }
    }
    if (probe && a.J && r == 0 && fs == 0 && fok) a.J[fm] += Jacc;
}

// ---------------------------------------------------------------------------
// FP32 operators, FP32 states, same row-split schedule.  The FP32 operator
// rows of a workgroup (512 KB at K = 1024) do not fit in registers, so each
// wave streams its quarter of the reduction of the current field from L2
// every half-step; products on v_mfma_f32_16x16x4f32 (A lane l: row l % 16,
// term l / 16; B lane l: term l / 16, column l % 16; D as above).  Operands
// come in k-groups of 16 terms (4 MFMA k-steps): lane l holds terms
// 4 j + l / 16 (j = 0..3) as one float4, for the operator
//   opf[t][w][kg][rb][lane] = op[64 t + 16 rb + l % 16][w kp/4 + 16 kg + 4 j + l / 16]
// and for the exchanged state, per group of NC = 16 NCB columns,
//   xf[kgg][cb][lane] = x[16 kgg + 4 j + l / 16][16 cb + l % 16]   (cb < NCB)
// (kgg = the global k-group), so every wave load is 1 KB contiguous.  FP32
// chains of 64 terms are folded into FP64 sums (the products' FP32 rounding
// then stays at the column-block kernel's level); the four wave partials
// meet in LDS in FP64, and the state (hi, lo) of a finishing thread's 4 NCB
// entries per field lives in its registers.
//
// Group width: each workgroup streams its 64 operator rows whatever the
// width, while its products and exchanged reads scale with NC, so the host
// takes the narrowest group (16, 32 or 64 columns) that still fits all
// workgroups on the chip: at M = 256 and K = 512 that is 16 columns on 128
// CUs instead of 64 columns on 32.  A column's state arithmetic (the
// k-quarter per wave, the 64-term chains, the fold and the partial-sum
// order) does not depend on NC, so every width gives bitwise the same
// states; only the probe's FP64 row sum (4 NCB rows per thread, then a
// shuffle tree) is associated differently.
constexpr int kChainGroups = 4;    // k-groups per FP32 chain (64 terms)
constexpr int kLdD = kRows + 2;    // LDS column stride of the FP64 partials (doubles)

typedef const __attribute__((address_space(1))) f4 gf4;

// KGT: k-groups per wave (K / 64) when fixed at compile time (fully
// unrolled; K = 256, 512, 1024), 0 for any K that is a multiple of 64 (KG
// taken at run time).  Both forms issue the same MFMAs in the same order
// (FP32 chains of 4 k-groups, the last one shorter when KG % 4 != 0, each
// folded into FP64 at its end), so they give the same sums.
template <int KGT, int NCB>
__device__ __forceinline__ void products_f32(const f4 *opw, const float *xgrp, int KG, int w, int lane,
                                             double (&acc)[4][NCB][4]) {
    constexpr int D = 2;     // ring depth in k-groups (K >= 128: KG >= 2)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[rb][cb][r] = 0.0;
    // opaque per-step bases (see products): no hoisted, spilled addresses
    uint64_t ob = reinterpret_cast<uint64_t>(opw), xb = reinterpret_cast<uint64_t>(xgrp);
    asm volatile("" : "+s"(ob), "+s"(xb));
    const unsigned loff = 16u * (unsigned)lane;
    f4 ra[D][4], rbx[D][NCB];
    // one FP32 chain of NQ k-groups from kg0, folded into the FP64 sums at
    // its end; `load` refills ring slot kg % D with k-group kg + D
    auto chain = [&](auto nq, int kg0, auto &&load) {
        constexpr int NQ = decltype(nq)::value;
        f4 c[4][NCB];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) c[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int kg = kg0 + q;
            const int slot = q % D;   // kg0 is a multiple of kChainGroups, itself one of D
            f4 a[4], b[NCB];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = ra[slot][i];
#pragma unroll
            for (int i = 0; i < NCB; ++i) b[i] = rbx[slot][i];
            load(kg + D, ra[slot], rbx[slot]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb)
                        c[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][j], b[cb][j], c[rb][cb], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[rb][cb][r] += (double)c[rb][cb][r];
        __builtin_amdgcn_sched_barrier(0);
    };
    using Q4 = std::integral_constant<int, kChainGroups>;
    if constexpr (KGT > 0) {
        gbyte *opb = reinterpret_cast<gbyte *>(ob);
        gbyte *xbb = reinterpret_cast<gbyte *>(xb) + (size_t)w * KGT * NCB * 1024;   // this wave's k-groups
        auto load = [&](int kg, f4 (&a)[4], f4 (&b)[NCB]) {
            if (kg >= KGT) return;
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = *reinterpret_cast<gf4 *>(opb + (size_t)(kg * 4 + q) * 1024 + loff);
#pragma unroll
            for (int q = 0; q < NCB; ++q)
                b[q] = __builtin_bit_cast(f4, ld_shared(xbb + (size_t)(kg * NCB + q) * 1024 + loff));
        };
#pragma unroll
        for (int d = 0; d < D; ++d) load(d, ra[d], rbx[d]);
        __builtin_amdgcn_sched_barrier(0);
        static_assert(KGT % kChainGroups == 0, "whole chains");
#pragma unroll
        for (int kg0 = 0; kg0 < KGT; kg0 += kChainGroups) chain(Q4{}, kg0, load);
    } else {
        // Run-time KG: buffer loads whose k-group offset is a scalar
        // (soffset), so no per-load address arithmetic; a ring refill past
        // the wave's last k-group re-reads that k-group (straight-line code:
        // a branch around the refill would make the compiler wait for every
        // load in flight).  Exchange loads take the device-scope policy.
        const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
            reinterpret_cast<void *>(ob), (short)0, KG * 4 * 1024, kRawBufferWord3);
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
            reinterpret_cast<void *>(xb), (short)0, 4 * KG * NCB * 1024, kRawBufferWord3);
        const int xw = w * KG * NCB * 1024;
        auto load = [&](int kg, f4 (&a)[4], f4 (&b)[NCB]) {
            kg = min(kg, KG - 1);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                a[q] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(ro, loff, (kg * 4 + q) * 1024, 0));
#pragma unroll
            for (int q = 0; q < NCB; ++q)
                b[q] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(
                                                  rx, loff, xw + (kg * NCB + q) * 1024, kDeviceScope));
        };
#pragma unroll
        for (int d = 0; d < D; ++d) load(d, ra[d], rbx[d]);
        __builtin_amdgcn_sched_barrier(0);
        const int full = KG - KG % kChainGroups;
        for (int kg0 = 0; kg0 < full; kg0 += kChainGroups) chain(Q4{}, kg0, load);
        switch (KG % kChainGroups) {
        case 1: chain(std::integral_constant<int, 1>{}, full, load); break;
        case 2: chain(std::integral_constant<int, 2>{}, full, load); break;
        case 3: chain(std::integral_constant<int, 3>{}, full, load); break;
        default: break;
        }
    }
}

// GR: grouped run of many instances (64-column groups, each with its own
// padded K).  A workgroup finds its group and row tile in the launch's slot
// map (a.smap[32 xcc + slot]: 32 lg + r, or -1 for an idle slot); group lg
// then takes its operators, source, mu, states, sizes, padded K, exchange
// offset, first sample column and dt from a.grp[a.g0 + lg] (the probe is
// off).  Otherwise they come from the arguments, the R = K / 64 row tiles of
// group g are R consecutive slots of one XCD, and group g owns columns NC g
// .. NC g + NC - 1.  The arithmetic of a column is the same either way.
//
// Finishing threads: TPC = 256 / NC threads per column; thread fs of column
// fj owns the rows 16 kgl + 4 j + q0 + qq (j = 0..3, qq < NCB) of the row
// tile, kgl = fs / (4 / NCB), q0 = NCB (fs % (4 / NCB)), as entry e = NCB j +
// qq of its registers: with the exchange layout above, the entries of one qq
// are the 4 terms of one lane's fragment, published as one float4.
// MODE: kSplitPlain, kSplitTraced (also writes the state after every step to
// a.vtr / a.str, entry 0 the state given, and the probe trace to a.y), or
// kSplitAdjoint: the discrete adjoint of the step run backwards, with the
// fields (V, S) holding (P, Q), the operators packed as (Asv^T, Avs^T), the
// host passing c as the source vector and b as the probe, the amplitude 2 y
// read from a.ytr, iteration k taking step n = n0 + nsteps - 1 - k; it
// writes a.qtr[n - n0] = Q before and a.wtr[n - n0] = P after the P update
// and adds dt (b^T P) du/dmu(t_n) to a.dmu.
enum SplitMode { kSplitPlain = 0, kSplitTraced = 1, kSplitAdjoint = 2 };

// This workgroup's slot code (xcd + 8 * slot on that XCD), from the launch's
// per-XCD slot counters.
__device__ __forceinline__ int take_slot(unsigned *slots) {
    __shared__ int sh_slot;
    if (threadIdx.x == 0) {
        const unsigned xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u;   // HW_REG_XCC_ID
        const unsigned s = __hip_atomic_fetch_add(&slots[xcc], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sh_slot = (int)(xcc + 8u * s);
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(sh_slot);
}

// The run of row tile r of group g (see the kernels below).
template <int KGT, bool GR, int NCB, int MODE>
__device__ __forceinline__ void split_f32_run(const SplitArgs &a, int g, int r, double *uwin) {
    static_assert(NCB == 1 || NCB == 2 || NCB == 4, "16, 32 or 64 columns per group");
    static_assert(!GR || NCB == 4, "grouped runs use 64-column groups");
    static_assert(MODE == kSplitPlain || (!GR && KGT == 0), "traced and adjoint runs: single, run-time K");
    constexpr int NC = 16 * NCB;               // columns per group
    constexpr int TPC = kThreads / NC;         // finishing threads per column
    constexpr int RPT = 4 * NCB;               // rows per finishing thread and field
    extern __shared__ __align__(16) unsigned char smem[];
    double *part = reinterpret_cast<double *>(smem);        // [wave][col][kLdD]
    float *bl = reinterpret_cast<float *>(part + kWaves * NC * kLdD);
    float *cl = bl + kRows;

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    int kp = a.kp, R = a.R;
    int kv = a.kv, M = a.M, col0 = g * NC, src = a.source;
    size_t xoff = (size_t)g * NC * kp;         // the group's exchange block (floats)
    double dt = a.dt;
    const float *bsrc = a.b, *csrc = a.c;
    const double *mup = a.mu;
    float *Vp = a.V, *Sp = a.S;
    const void *opv = a.opv, *ops = a.ops;
    if constexpr (GR) {
        // the descriptor is the same for the whole workgroup: keep its
        // fields in scalar registers (the operator bases must be scalar)
        const SplitGroup &q = a.grp[a.g0 + g];
        kv = __builtin_amdgcn_readfirstlane(q.kv);
        kp = __builtin_amdgcn_readfirstlane(q.kp);
        R = kp / kRows;
        xoff = (size_t)uniform64((uint64_t)q.xoff);
        M = __builtin_amdgcn_readfirstlane(q.M);
        col0 = __builtin_amdgcn_readfirstlane(q.col0);
        src = __builtin_amdgcn_readfirstlane(q.source);
        dt = __builtin_bit_cast(double, uniform64(__builtin_bit_cast(uint64_t, q.dt)));
        bsrc = reinterpret_cast<const float *>(uniform64(reinterpret_cast<uint64_t>(q.b)));
        csrc = nullptr;
        mup = reinterpret_cast<const double *>(uniform64(reinterpret_cast<uint64_t>(q.mu)));
        Vp = reinterpret_cast<float *>(uniform64(reinterpret_cast<uint64_t>(q.V)));
        Sp = reinterpret_cast<float *>(uniform64(reinterpret_cast<uint64_t>(q.S)));
        opv = reinterpret_cast<const void *>(uniform64(reinterpret_cast<uint64_t>(q.opv)));
        ops = reinterpret_cast<const void *>(uniform64(reinterpret_cast<uint64_t>(q.ops)));
    }
    unsigned *cnt = a.cnt + (size_t)g * kCntStride;
    unsigned phase = 0;
    const int row0 = r * kRows;

    for (int i = tid; i < kRows; i += kThreads) {
        const int row = row0 + i;
        bl[i] = row < kv ? bsrc[row] : 0.f;
        cl[i] = (csrc != nullptr && row < kv) ? csrc[row] : 0.f;
    }
    // finishing thread: column fj, RPT rows (see above); its state entries of
    // both fields stay in registers
    const int fj = tid / TPC, fs = tid % TPC;
    const int kgl = fs / (4 / NCB), q0 = NCB * (fs % (4 / NCB));
    auto frow = [&](int e) { return 16 * kgl + 4 * (e / NCB) + q0 + e % NCB; };   // row within the tile
    const int fm = col0 + fj;
    const bool fok = fm < M;
    float sh[2][RPT], sl[2][RPT];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
            const int row = row0 + frow(e);
            const float *src = f == 0 ? Vp : Sp;
            sh[f][e] = (fok && row < kv) ? src[(size_t)fm * kv + row] : 0.f;
            sl[f][e] = 0.f;
        }
    __syncthreads();

    // this wave's operator panel (k-groups w KG .. of row tile r)
    const int KG = KGT > 0 ? KGT : kp / 64;
    const f4 *opvw = reinterpret_cast<const f4 *>(opv) + (size_t)(r * kWaves + w) * KG * 4 * 64;
    const f4 *opsw = reinterpret_cast<const f4 *>(ops) + (size_t)(r * kWaves + w) * KG * 4 * 64;
    float *xv = reinterpret_cast<float *>(a.xv), *xs = reinterpret_cast<float *>(a.xs);

    // publish this thread's rows (hi words) of field f in fragment order:
    // row row0 + 16 kgl + 4 j + q of column fj is term j of lane 16 q + fj % 16
    // in k-group (row0 + 16 kgl) / 16, column block fj / 16
    auto publish = [&](int f, float *x) {
        float *xg = x + xoff;
        const int kgg = (row0 + 16 * kgl) / 16, cb = fj / 16;
#pragma unroll
        for (int qq = 0; qq < NCB; ++qq) {
            const f4 v = {sh[f][qq], sh[f][NCB + qq], sh[f][2 * NCB + qq], sh[f][3 * NCB + qq]};
            *reinterpret_cast<f4 *>(xg + ((size_t)(kgg * NCB + cb) * 64 + 16 * (q0 + qq) + (fj & 15)) * 4) = v;
        }
    };

    auto half_step = [&](int f, const f4 *opw, const float *xother, float *xmine, const double *up,
                         bool forced) -> double {
        double acc[4][NCB][4];
        products_f32<KGT, NCB>(opw, xother + xoff, KG, w, lane, acc);
        double *pw = part + w * NC * kLdD;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                double *d = pw + (16 * cb + (lane & 15)) * kLdD + 16 * rb + 4 * (lane >> 4);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) d[rr] = acc[rb][cb][rr];
            }
        __syncthreads();
        const double u = forced ? *up : 0.0;
        double ypart = 0.0;
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
            const int i = frow(e);
            double inc = (part[(0 * NC + fj) * kLdD + i] + part[(1 * NC + fj) * kLdD + i]) +
                         (part[(2 * NC + fj) * kLdD + i] + part[(3 * NC + fj) * kLdD + i]);
            if (forced) inc = fma((double)bl[i], u, inc);
            const double yv = fma(dt, inc, (double)sh[f][e] + (double)sl[f][e]);
            const float hv = (float)yv;
            sh[f][e] = hv;
            sl[f][e] = (float)(yv - (double)hv);
            if (forced) ypart += (double)cl[i] * yv;
        }
        publish(f, xmine);
        __syncthreads();   // partials read before the next half-step writes them
        return ypart;
    };

    // this thread's rows of field f (hi + lo) into trace matrix tr (M x kv
    // per entry), entry e
    auto trace = [&](float *tr, int f, int64_t e) {
        float *d = tr + (size_t)e * M * kv + (size_t)fm * kv;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int row = row0 + frow(i);
            if (fok && row < kv) d[row] = sh[f][i] + sl[f][i];
        }
    };

    publish(1, xs);
    group_barrier(a, cnt, (unsigned)R * ++phase);
    if constexpr (MODE == kSplitTraced) {
        trace(a.vtr, 0, 0);
        trace(a.str, 1, 0);
    }

    double Jacc = 0.0;
    const bool probe = csrc != nullptr;
    const double muf = fok ? mup[fm] : 1.0;
    for (int64_t k = 0; k < a.nsteps; ++k) {
        // step n of this iteration, its trace row
        const int64_t n = MODE == kSplitAdjoint ? a.n0 + a.nsteps - 1 - k : a.n0 + k;
        if (k % kUWin == 0) {
            if constexpr (MODE == kSplitAdjoint)
                adjoint_window<NC>(uwin, a.ytr, a.nsteps - 1 - k, col0, M);
            else
                forcing_window<NC>(uwin, src, a.n0 + k, dt, mup, col0, M);
        }
        if constexpr (MODE == kSplitAdjoint) trace(a.qtr, 1, n - a.n0);   // Q^{n+1}
        // (read after the products' barrier inside half_step)
        double yp = half_step(0, opvw, xs, xv, uwin + (k % kUWin) * NC + fj, true);
        if constexpr (MODE == kSplitAdjoint) trace(a.wtr, 0, n - a.n0);   // w^n
        if constexpr (MODE == kSplitTraced) trace(a.vtr, 0, k + 1);
        if (probe) {
            // sum over the TPC consecutive threads of column fj
#pragma unroll
            for (int off = 1; off < TPC; off <<= 1) yp += __shfl_xor(yp, off, 64);
            if (fs == 0) a.yp[((size_t)g * R + r) * NC + fj] = yp;
        }
        group_barrier(a, cnt, (unsigned)R * ++phase);
        if (probe && r == 0 && fok) {
            const double yv = sum_partials_spread<TPC>(a.yp + (size_t)g * R * NC + fj, NC, R, fs);
            if (fs == 0) {
                if constexpr (MODE == kSplitAdjoint) {
                    Jacc += dt * yv * dev::forcing_dmu(src, (double)n * dt, muf);
                } else {
                    Jacc += dt * (yv * yv);
                    if (a.y) a.y[(size_t)k * M + fm] = yv;
                }
            }
        }
        half_step(1, opsw, xv, xs, nullptr, false);
        if constexpr (MODE == kSplitTraced) trace(a.str, 1, k + 1);
        group_barrier(a, cnt, (unsigned)R * ++phase);
    }

#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
            const int row = row0 + frow(e);
            float *dst = f == 0 ? Vp : Sp;
            if (fok && row < kv) dst[(size_t)fm * kv + row] = sh[f][e] + sl[f][e];
        }
    if constexpr (MODE == kSplitAdjoint) {
        if (probe && a.dmu && r == 0 && fs == 0 && fok) a.dmu[fm] += Jacc;
    } else {
        if (probe && a.J && r == 0 && fs == 0 && fok) a.J[fm] += Jacc;
    }
}

template <int KGT, bool GR, int NCB, int MODE = kSplitPlain>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void rank2_split_f32_kernel(SplitArgs a) {
    __shared__ double uwin[kUWin * 16 * NCB];
    const int code = take_slot(a.slots);
    const int xcc = code & 7, s = code >> 3;
    int r, g;
    if constexpr (GR) {
        const int e = s < 32 ? a.smap[32 * xcc + s] : -1;
        if (e < 0) return;                     // idle workgroup (never counted)
        g = __builtin_amdgcn_readfirstlane(e >> 5);
        r = __builtin_amdgcn_readfirstlane(e & 31);
    } else {
        r = s % a.R;
        g = (s / a.R) * 8 + xcc;
        if (g >= a.G) return;
    }
    split_f32_run<KGT, GR, NCB, MODE>(a, g, r, uwin);
}

// Two runs of one shape side by side in one launch, on disjoint workgroups:
// groups 0 .. G-1 run a0 traced (the adjoint's recompute of a segment),
// groups G .. 2G-1 run a1 in adjoint mode (the reverse sweep of the next
// segment).  Each run has its own workspace (exchange, counters); the slot
// counters are a0's.
template <int NCB>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void rank2_split_f32_dual_kernel(SplitArgs a0, SplitArgs a1) {
    __shared__ double uwin[kUWin * 16 * NCB];
    const int code = take_slot(a0.slots);
    const int xcc = code & 7, s = code >> 3;
    const int r = s % a0.R, g = (s / a0.R) * 8 + xcc;
    if (g >= 2 * a0.G) return;
    if (g < a0.G)
        split_f32_run<0, false, NCB, kSplitTraced>(a0, g, r, uwin);
    else
        split_f32_run<0, false, NCB, kSplitAdjoint>(a1, g - a0.G, r, uwin);
}

// FP32 split-layout operator (rows x cols) from a column-major FP32 matrix:
// A itself (ld rows), or with `trans` the transpose of a column-major
// cols x rows matrix (ld cols); zero padded: dst[t][w][kg][rb][lane][j]
// (see above).
__global__ void split_pack_f32_kernel(const float *__restrict__ A, int rows, int cols, int T, int kp, int trans,
                                      float *__restrict__ dst) {
    const int KG = kp / 64;
    const int64_t total = (int64_t)T * kWaves * KG * 4 * 64 * 4;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t q = idx;
        const int j = (int)(q % 4); q /= 4;
        const int lane = (int)(q % 64); q /= 64;
        const int rb = (int)(q % 4); q /= 4;
        const int kg = (int)(q % KG); q /= KG;
        const int w = (int)(q % kWaves); q /= kWaves;
        const int t = (int)q;
        const int row = 64 * t + 16 * rb + (lane & 15);
        const int k = w * (kp / 4) + 16 * kg + 4 * j + (lane >> 4);
        dst[idx] = (row < rows && k < cols) ? (trans ? A[k + (int64_t)row * cols] : A[row + (int64_t)k * rows]) : 0.f;
    }
}

// Split-layout BF16 fragments from the low-precision packed operator:
// dst[t][w][rb][kb][lane][e] = op[64 t + 16 rb + lane % 16][w kp/4 + 32 kb +
// 8 (lane / 16) + e], read from the column-block layout
// (BF16: pk[t][k/8][row][8]; FP8: pk[t][k/16][row][16] E4M3 bytes, widened
// exactly to BF16).
__global__ void split_pack_kernel(const unsigned char *__restrict__ src, int fp8, int T, int kp,
                                  unsigned short *__restrict__ dst) {
    const int KB = kp / 128;
    const int64_t total = (int64_t)T * kWaves * 4 * KB * 64 * 8;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t q = idx;
        const int e = (int)(q % 8); q /= 8;
        const int lane = (int)(q % 64); q /= 64;
        const int kb = (int)(q % KB); q /= KB;
        const int rb = (int)(q % 4); q /= 4;
        const int w = (int)(q % kWaves); q /= kWaves;
        const int t = (int)q;
        const int i = 16 * rb + (lane & 15);                    // row within tile
        const int k = w * (kp / 4) + 32 * kb + 8 * (lane >> 4) + e;
        unsigned short v;
        if (!fp8) {
            const unsigned short *s16 = reinterpret_cast<const unsigned short *>(src);
            v = s16[(((int64_t)t * (kp / 8) + k / 8) * 64 + i) * 8 + k % 8];
        } else {
            const unsigned char byte = src[(((int64_t)t * (kp / 16) + k / 16) * 64 + i) * 16 + k % 16];
            typedef float f2 __attribute__((ext_vector_type(2)));
            const f2 wv = __builtin_amdgcn_cvt_pk_f32_fp8((int)byte, false);
            v = (unsigned short)(__float_as_uint(wv.x) >> 16);   // E4M3 values are exact in BF16
        }
        dst[idx] = v;
    }
}

__global__ void split_zero_kernel(unsigned *__restrict__ p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

}  // namespace

size_t rank2_split_lds_bytes() {
    return sizeof(float) * ((size_t)2 * 2 * kCols * kLd + (size_t)kWaves * kCols * kLd + 2 * kRows);
}

bool rank2_split_k_ok(int kvp, bool f32) {
    if (f32) return kvp % kRows == 0 && kvp >= 2 * kRows && kvp <= kMaxSplitK;
    return kvp % 128 == 0 && kvp >= 128 && kvp <= 1024;   // whole 32-term k-blocks per wave
}

// Groups of R = kvp / 64 workgroups one launch holds: a group's workgroups
// share an XCD, so each of the 8 XCDs (32 CUs) holds floor(32 / R) groups.
int rank2_split_groups_per_launch(int kvp) { return kXcds * (kCusPerXcd / (kvp / kRows)); }

// Supported shapes: Kv == Ks == K with K a multiple of 64 in [128, 2048]
// for FP32 operators, a multiple of 128 up to 1024 for BF16 / FP8 ones (register-
// resident fragments), and all 64-column groups in one launch (one
// workgroup per CU, all resident).  Returns the group count, or 0 if the
// row-split schedule does not apply.
int rank2_split_groups(int kv, int ks, int kvp, int ksp, int M, bool f32) {
    if (kv != ks || kvp != ksp || !rank2_split_k_ok(kvp, f32)) return 0;
    const int G = (M + kCols - 1) / kCols;
    if (G > rank2_split_groups_per_launch(kvp)) return 0;
    return G;
}

size_t rank2_split_workspace_bytes(int kvp, int G) {
    return rank2_split_ws_bytes((size_t)G * kCols * kvp, (size_t)G * (kvp / kRows) * kCols);
}

size_t rank2_split_ws_bytes(size_t xfloats, size_t ypd) {
    return sizeof(float) * 2 * xfloats                                 // xv, xs
           + sizeof(double) * ypd                                      // yp
           + sizeof(unsigned) * (256 * kCntStride + 64);               // counters, slots
}

size_t rank2_split_f32_lds_bytes() {
    return sizeof(double) * (size_t)kWaves * kCols * kLdD + sizeof(float) * 2 * kRows;
}

hipError_t launch_split_pack_f32(const float *A, int rows, int cols, int prow, int pcol, void *dst, hipStream_t st,
                                 bool trans) {
    const int T = prow / kRows;
    const int64_t total = (int64_t)T * 64 * pcol;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(split_pack_f32_kernel, dim3(blocks), dim3(256), 0, st, A, rows, cols, T, pcol, trans ? 1 : 0,
                       static_cast<float *>(dst));
    return hipGetLastError();
}

hipError_t launch_split_pack(const void *lp, bool fp8, int kvp, int ksp, void *dst, hipStream_t st) {
    const int T = kvp / kRows;
    const int64_t total = (int64_t)T * 64 * ksp;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(split_pack_kernel, dim3(blocks), dim3(256), 0, st,
                       static_cast<const unsigned char *>(lp), fp8 ? 1 : 0, T, ksp,
                       static_cast<unsigned short *>(dst));
    return hipGetLastError();
}

namespace {

// Carve a workspace of rank2_split_ws_bytes(xfloats, ypd) into the
// exchange buffers (xfloats floats per field), probe partials (ypd
// doubles), group counters and XCD slot counters, and enqueue the clearing
// of the counters and of the abort flag status[2].
hipError_t split_workspace(SplitArgs &a, void *ws, size_t xfloats, size_t ypd, hipStream_t st) {
    unsigned short *x = static_cast<unsigned short *>(ws);
    const size_t xsz = 2 * xfloats;    // in BF16 elements
    a.xv = x;
    a.xs = x + xsz;
    a.yp = reinterpret_cast<double *>(x + 2 * xsz);
    a.cnt = reinterpret_cast<unsigned *>(a.yp + ypd);
    a.slots = a.cnt + 256 * kCntStride;
    a.spin_max = g_forced_timeout ? 256 : kSpinMax;
    a.wait_bias = g_forced_timeout ? 1u : 0u;
    hipLaunchKernelGGL(split_zero_kernel, dim3(64), dim3(256), 0, st, a.cnt, 256 * kCntStride + 64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(split_zero_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned *>(a.status + 2), 1);
    return hipGetLastError();
}

// FP32 kernels: single runs with 16- or 32-column groups at K = 256, 512,
// 1024 take the compile-time k-group count; every other single run
// (64-column groups, other K) and the grouped runs take the run-time one,
// which measured faster with 64-column groups (38.7 against 40.3 us per
// step at K = M = 1024) and slower with narrow ones (14.3 against 12.8 at
// K = 1024, M = 256).  Table: (K = 256, 512, 1024) x (16, 32 columns), then
// the run-time kernels for 16, 32, 64 columns, then the grouped one.
const void *const kSplitF32Kernels[10] = {
    (const void *)rank2_split_f32_kernel<4, false, 1>,  (const void *)rank2_split_f32_kernel<4, false, 2>,
    (const void *)rank2_split_f32_kernel<8, false, 1>,  (const void *)rank2_split_f32_kernel<8, false, 2>,
    (const void *)rank2_split_f32_kernel<16, false, 1>, (const void *)rank2_split_f32_kernel<16, false, 2>,
    (const void *)rank2_split_f32_kernel<0, false, 1>,  (const void *)rank2_split_f32_kernel<0, false, 2>,
    (const void *)rank2_split_f32_kernel<0, false, 4>,  (const void *)rank2_split_f32_kernel<0, true, 4>};

// Traced and adjoint runs (run-time K) by group width.
const void *const kSplitF32ModeKernels[2][3] = {
    {(const void *)rank2_split_f32_kernel<0, false, 1, kSplitTraced>,
     (const void *)rank2_split_f32_kernel<0, false, 2, kSplitTraced>,
     (const void *)rank2_split_f32_kernel<0, false, 4, kSplitTraced>},
    {(const void *)rank2_split_f32_kernel<0, false, 1, kSplitAdjoint>,
     (const void *)rank2_split_f32_kernel<0, false, 2, kSplitAdjoint>,
     (const void *)rank2_split_f32_kernel<0, false, 4, kSplitAdjoint>}};

const void *const kSplitF32DualKernels[3] = {(const void *)rank2_split_f32_dual_kernel<1>,
                                             (const void *)rank2_split_f32_dual_kernel<2>,
                                             (const void *)rank2_split_f32_dual_kernel<4>};

// wi: group width 16 << wi columns (single runs; grouped runs take 64).
template <bool GR>
hipError_t launch_split_f32(int kp, int wi, void **args, hipStream_t st) {
    if (wi < 0 || wi > 2) return hipErrorInvalidValue;
    const int ki = kp == 256 ? 0 : (kp == 512 ? 1 : (kp == 1024 ? 2 : -1));
    const void *f = GR ? kSplitF32Kernels[9] : (ki >= 0 && wi < 2 ? kSplitF32Kernels[2 * ki + wi]
                                                                    : kSplitF32Kernels[6 + wi]);
    return hipLaunchCooperativeKernel(f, dim3(256), dim3(kThreads), args, rank2_split_f32_lds_bytes(), st);
}

// Low-precision kernels by (K = 128 KB, KB = 1 .. 8) x (pair, single-pass) x
// (group width 16, 32, 64 columns).
#define ROM_LP_WIDTHS(KB, SG)                                                           \
    (const void *)rank2_split_kernel<KB, SG, 1>, (const void *)rank2_split_kernel<KB, SG, 2>, \
        (const void *)rank2_split_kernel<KB, SG, 4>
const void *const kSplitLpKernels[48] = {
    ROM_LP_WIDTHS(1, false), ROM_LP_WIDTHS(1, true), ROM_LP_WIDTHS(2, false), ROM_LP_WIDTHS(2, true),
    ROM_LP_WIDTHS(3, false), ROM_LP_WIDTHS(3, true), ROM_LP_WIDTHS(4, false), ROM_LP_WIDTHS(4, true),
    ROM_LP_WIDTHS(5, false), ROM_LP_WIDTHS(5, true), ROM_LP_WIDTHS(6, false), ROM_LP_WIDTHS(6, true),
    ROM_LP_WIDTHS(7, false), ROM_LP_WIDTHS(7, true), ROM_LP_WIDTHS(8, false), ROM_LP_WIDTHS(8, true)};
#undef ROM_LP_WIDTHS

// Width index (group width 16 << wi columns) of the narrowest group whose
// ceil(M / width) groups fit in one launch; the caller's check that the
// 64-column groups fit guarantees that one does.
int split_width_index(int M, int kvp) {
    const int cap = rank2_split_groups_per_launch(kvp);
    int wi = 0;
    while (wi < 2 && (M + (16 << wi) - 1) / (16 << wi) > cap) ++wi;
    return wi;
}

// Scratch of the allocation-free row-split run (rom_run_rank2_noalloc):
// exchange rows, probe partials and barrier counters of the largest launch
// the schedule makes (rank2_split_workspace_bytes over every eligible shape:
// 8 MiB of exchange at G K = 256 x 64, 128 KiB of probe partials, 64 KiB of
// counters).  One copy per GPU, held until the process ends; every call on a
// GPU uses that GPU's copy.
constexpr size_t kStaticScratchBytes = (size_t)8448 * 1024;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

}  // namespace

size_t rank2_split_static_bytes() { return kStaticScratchBytes; }

// Device address of this GPU's static scratch, looked up once per device
// with that device current (the array's host-side name is not a device
// address).  Only the returned pointer is passed to kernels.
hipError_t rank2_split_static_scratch(int device, void **ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_grouped_split_f32(const SplitGroup *grp_dev, int g0, int G, const int *smap_dev, size_t xfloats,
                                    void *ws, int *status, int64_t n0, int64_t nsteps, hipStream_t st) {
    if (G <= 0 || nsteps <= 0) return hipSuccess;
    if (G > kXcds * kCusPerXcd / 2) return hipErrorInvalidValue;
    SplitArgs a{};
    a.grp = grp_dev;
    a.smap = smap_dev;
    a.g0 = g0;
    a.G = G;
    a.n0 = n0;
    a.nsteps = nsteps;
    a.scale = 1.0f;
    a.status = status;
    hipError_t e = split_workspace(a, ws, xfloats, 0, st);
    if (e != hipSuccess) return e;
    void *args[] = {&a};
    return launch_split_f32<true>(0, 2, args, st);
}

hipError_t launch_rank2_split(const void *opv, const void *ops, const Rank2Args &r2, float scale, void *ws,
                              int G, int *status, bool f32, hipStream_t st, int mode) {
    SplitArgs a{};
    a.opv = static_cast<const u4 *>(opv);
    a.ops = static_cast<const u4 *>(ops);
    a.b = static_cast<const float *>(r2.b);
    a.c = static_cast<const float *>(r2.c);
    a.mu = r2.mu;
    a.V = static_cast<float *>(r2.V);
    a.S = static_cast<float *>(r2.S);
    a.J = r2.J;
    a.y = r2.y;
    a.kv = r2.kv;
    a.kp = r2.kvp;
    a.M = r2.M;
    a.G = G;
    a.R = r2.kvp / kRows;
    a.n0 = r2.n0;
    a.nsteps = r2.nsteps;
    a.dt = r2.dt;
    a.source = r2.source;
    a.scale = scale;
    a.status = status;
    a.grp = nullptr;
    a.smap = nullptr;
    a.g0 = 0;
    if (!rank2_split_k_ok(a.kp, f32) || G > rank2_split_groups_per_launch(a.kp)) return hipErrorInvalidValue;
    hipError_t e = split_workspace(a, ws, (size_t)G * kCols * a.kp, (size_t)G * a.R * kCols, st);
    if (e != hipSuccess) return e;
    void *args[] = {&a};
    // the narrowest column group (16, 32 or 64 columns) whose workgroups all
    // fit; the workspace, carved for G 64-column groups, covers it
    // (ceil(M / nc) nc <= ceil(M / 64) 64)
    const int wi = split_width_index(a.M, a.kp);
    a.G = (a.M + (16 << wi) - 1) / (16 << wi);
    if (mode != kSplitPlain) {
        if (!f32 || (mode != kSplitTraced && mode != kSplitAdjoint)) return hipErrorInvalidValue;
        a.vtr = static_cast<float *>(r2.vtr);
        a.str = static_cast<float *>(r2.str);
        a.ytr = r2.ytr;
        a.wtr = static_cast<float *>(r2.wtr);
        a.qtr = static_cast<float *>(r2.qtr);
        a.dmu = r2.dmu;
        return hipLaunchCooperativeKernel(kSplitF32ModeKernels[mode - 1][wi], dim3(256), dim3(kThreads), args,
                                          rank2_split_f32_lds_bytes(), st);
    }
    if (f32) return launch_split_f32<false>(a.kp, wi, args, st);
    const size_t lds = rank2_split_lds_bytes();
    const int idx = a.kp / 128 - 1;   // k-blocks per wave - 1 (K a multiple of 128, checked above)
    return hipLaunchCooperativeKernel(kSplitLpKernels[6 * idx + 3 * (r2.single ? 1 : 0) + wi], dim3(256),
                                      dim3(kThreads), args, lds, st);
}

namespace {

void fill_split_args(SplitArgs &a, const void *opv, const void *ops, const Rank2Args &r2, int *status) {
    a = SplitArgs{};
    a.opv = static_cast<const u4 *>(opv);
    a.ops = static_cast<const u4 *>(ops);
    a.b = static_cast<const float *>(r2.b);
    a.c = static_cast<const float *>(r2.c);
    a.mu = r2.mu;
    a.V = static_cast<float *>(r2.V);
    a.S = static_cast<float *>(r2.S);
    a.J = r2.J;
    a.y = r2.y;
    a.kv = r2.kv;
    a.kp = r2.kvp;
    a.M = r2.M;
    a.R = r2.kvp / kRows;
    a.n0 = r2.n0;
    a.nsteps = r2.nsteps;
    a.dt = r2.dt;
    a.source = r2.source;
    a.scale = 1.0f;
    a.status = status;
    a.vtr = static_cast<float *>(r2.vtr);
    a.str = static_cast<float *>(r2.str);
    a.ytr = r2.ytr;
    a.wtr = static_cast<float *>(r2.wtr);
    a.qtr = static_cast<float *>(r2.qtr);
    a.dmu = r2.dmu;
}

}  // namespace

int rank2_split_dual_width(int kvp, int M) {
    if (!rank2_split_k_ok(kvp, true)) return -1;
    const int cap = rank2_split_groups_per_launch(kvp);
    for (int wi = 0; wi < 3; ++wi)
        if (2 * ((M + (16 << wi) - 1) / (16 << wi)) <= cap) return wi;
    return -1;
}

hipError_t launch_rank2_split_dual(const void *opv0, const void *ops0, const Rank2Args &r0, void *ws0,
                                   const void *opv1, const void *ops1, const Rank2Args &r1, void *ws1, int G,
                                   int *status, hipStream_t st) {
    const int wi = rank2_split_dual_width(r0.kvp, r0.M);
    if (wi < 0 || r1.kvp != r0.kvp || r1.M != r0.M || r1.nsteps <= 0 || r0.nsteps <= 0) return hipErrorInvalidValue;
    SplitArgs a0, a1;
    fill_split_args(a0, opv0, ops0, r0, status);
    fill_split_args(a1, opv1, ops1, r1, status);
    const int R = r0.kvp / kRows;
    // each run's workspace, carved for G 64-column groups
    hipError_t e = split_workspace(a0, ws0, (size_t)G * kCols * a0.kp, (size_t)G * R * kCols, st);
    if (e == hipSuccess) e = split_workspace(a1, ws1, (size_t)G * kCols * a1.kp, (size_t)G * R * kCols, st);
    if (e != hipSuccess) return e;
    a0.G = a1.G = (r0.M + (16 << wi) - 1) / (16 << wi);
    void *args[] = {&a0, &a1};
    return hipLaunchCooperativeKernel(kSplitF32DualKernels[wi], dim3(256), dim3(kThreads), args,
                                      rank2_split_f32_lds_bytes(), st);
}

// The schedule needs all 256 workgroups resident at once, one per CU, 32 on
// each of the 8 XCDs (the group-slot logic counts on it), and cooperative
// launch support.
bool rank2_split_device_ok() {
    int dev = 0, ncu = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess) return false;
    if (ncu != 256 || !coop) return false;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0) return false;
    const size_t lds = rank2_split_lds_bytes();
    for (const void *f : kSplitLpKernels) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kThreads, lds) != hipSuccess || nb < 1) return false;
    }
    for (const void *f : kSplitF32Kernels) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kThreads, rank2_split_f32_lds_bytes()) != hipSuccess ||
            nb < 1)
            return false;
    }
    for (const void *f : kSplitF32DualKernels) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kThreads, rank2_split_f32_lds_bytes()) != hipSuccess ||
            nb < 1)
            return false;
    }
    for (const auto &row : kSplitF32ModeKernels)
        for (const void *f : row) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kThreads, rank2_split_f32_lds_bytes()) !=
                    hipSuccess ||
                nb < 1)
                return false;
        }
    return true;
}

hipError_t rank2_split_configure() {
    // exactly the dynamic LDS the launch asks for (the kernel also has a few
    // bytes of static LDS, so the 160 KB maximum would be refused)
    const int lds = (int)rank2_split_lds_bytes();
    hipError_t e;
    for (const void *f : kSplitLpKernels) {
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    const int lf = (int)rank2_split_f32_lds_bytes();
    for (const void *f : kSplitF32Kernels) {
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lf);
        if (e != hipSuccess) return e;
    }
    for (const auto &row : kSplitF32ModeKernels)
        for (const void *f : row) {
            e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lf);
            if (e != hipSuccess) return e;
        }
    for (const void *f : kSplitF32DualKernels) {
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lf);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rom
