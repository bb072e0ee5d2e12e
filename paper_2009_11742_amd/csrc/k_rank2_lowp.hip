// Rank-2 leapfrog stepper with low-precision operators (BF16 or FP8-E4M3)
// and FP32 states: the precision extension of the rank-2 products (the
// paper points to tensor-core style units for batched products, Sec. 5).
//
// Same column-block decomposition as the FP32 kernel (one workgroup owns 4
// samples for the whole run, states in LDS, no cross-workgroup traffic), with
// the products on v_mfma_f32_4x4x4bf16_1k: 16 blocks = 64 operator rows x 4
// sample columns x 4 reduction terms per instruction.
//
//  * Operators: BF16 (round to nearest even from FP32), packed
//    pk[t][k/8][lane][8] (16 bytes per lane per 8 terms); or FP8-E4M3 with one
//    per-tensor scale shared by both operators (amax / 448), packed
//    pk[t][k/16][lane][16].  FP8 fragments are widened to BF16 in registers
//    (every E4M3 value is exactly a BF16 value), so the product sees the
//    stored FP8 values exactly; the scale multiplies the FP32 result.
//  * State operand: each FP32 state value x is fed as the BF16 pair
//    x_hi = bf16(x), x_lo = bf16(x - x_hi) (two MFMA passes), about 16
//    significant bits; the products accumulate in FP32 and are folded every
//    32 terms into a compensated (hi, lo) pair.  The single-pass variant
//    (SINGLE) feeds x_hi alone: one MFMA per operator fragment, about 8
//    significant bits of the state per product.
//  * State: FP32 hi/lo pairs in LDS with the double-float update of the FP32
//    kernel; the BF16 split of every updated entry is written next to it.
#include "k_tile_f32.h"

namespace rom {
namespace {

using dev::f4;
using tile::kThreads;
using tile::kWaves;
using tile::NB;

typedef short s4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kLpChunk = 32;   // reduction terms per compensated chunk

// bf16 (as the high half of an FP32 word) with round to nearest even.
__device__ __forceinline__ unsigned short bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// 16 bytes of packed BF16 fragment -> two A operands (terms k..k+3, k+4..k+7)
// (BF16 path: the bytes already are BF16).  FP8 path: 16 E4M3 bytes ->
// four A operands, exactly, via the hardware E4M3 -> FP32 conversion and the
// high halves of the FP32 words.
__device__ __forceinline__ s4 pack_hi_halves(float a, float b, float c, float d) {
    unsigned lo = __builtin_amdgcn_perm(__float_as_uint(b), __float_as_uint(a), 0x07060302u);
    unsigned hi = __builtin_amdgcn_perm(__float_as_uint(d), __float_as_uint(c), 0x07060302u);
    s4 r;
    r.x = (short)(lo & 0xffffu);
    r.y = (short)(lo >> 16);
    r.z = (short)(hi & 0xffffu);
    r.w = (short)(hi >> 16);
    return r;
}

__device__ __forceinline__ void widen_fp8(unsigned w, s4 &out) {
    // w holds 4 E4M3 bytes: terms 0..3
    typedef float f2 __attribute__((ext_vector_type(2)));
    f2 a = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
    f2 b = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
    out = pack_hi_halves(a.x, a.y, b.x, b.y);
}

__device__ __forceinline__ s4 as_s4(unsigned lo, unsigned hi) {
    s4 r;
    r.x = (short)(lo & 0xffffu);
    r.y = (short)(lo >> 16);
    r.z = (short)(hi & 0xffffu);
    r.w = (short)(hi >> 16);
    return r;
}

// Product of one 32-term chunk for a 64 x 4 tile: A fragments `a` (8 operand
// quads), state splits xh / xl (8 quads each, this lane's column; xl unused
// when SINGLE).
template <bool SINGLE>
__device__ __forceinline__ void mma_chunk_lp(const s4 (&a)[8], const s4 (&xh)[8], const s4 (&xl)[8],
                                             f4 &hi, f4 &lo) {
    f4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        c0 = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a[q], xh[q], c0, 0, 0, 0);
        if constexpr (!SINGLE) c1 = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a[q], xl[q], c1, 0, 0, 0);
    }
    tile::fold(hi, lo, c0);
    if constexpr (!SINGLE) tile::fold(hi, lo, c1);
}

template <int OP>
struct Frag;   // raw fragment storage of one chunk for one lane

template <>
struct Frag<ROM_BF16> {
    u4 r[4];   // 4 x 16 bytes = 32 BF16 terms
    __device__ __forceinline__ void load(const u4 *ap, int ch) {
        const u4 *s = ap + (size_t)ch * 4 * 64;
#pragma unroll
        for (int q = 0; q < 4; ++q) r[q] = s[q * 64];
    }
    __device__ __forceinline__ void operands(s4 (&a)[8]) const {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[2 * q] = as_s4(r[q].x, r[q].y);
            a[2 * q + 1] = as_s4(r[q].z, r[q].w);
        }
    }
};

template <>
struct Frag<ROM_F8E4M3> {
    u4 r[2];   // 2 x 16 bytes = 32 E4M3 terms
    __device__ __forceinline__ void load(const u4 *ap, int ch) {
        const u4 *s = ap + (size_t)ch * 2 * 64;
#pragma unroll
        for (int q = 0; q < 2; ++q) r[q] = s[q * 64];
    }
    __device__ __forceinline__ void operands(s4 (&a)[8]) const {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            widen_fp8(r[q].x, a[4 * q + 0]);
            widen_fp8(r[q].y, a[4 * q + 1]);
            widen_fp8(r[q].z, a[4 * q + 2]);
            widen_fp8(r[q].w, a[4 * q + 3]);
        }
    }
};

// 8 operand quads of this lane's BF16 split column (terms ch*32 .. +31).
__device__ __forceinline__ void lds_split(s4 (&x)[8], const unsigned short *col, int ch) {
    const u4 *s = reinterpret_cast<const u4 *>(col + ch * kLpChunk);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        u4 v = s[q];
        x[2 * q] = as_s4(v.x, v.y);
        x[2 * q + 1] = as_s4(v.z, v.w);
    }
}

template <int OP, bool SINGLE>
__device__ __forceinline__ void tile_product_lp(const u4 *__restrict__ pk, int t, int kp,
                                                const unsigned short *xh_col,
                                                const unsigned short *xl_col, int lane, f4 &H,
                                                f4 &L) {
    constexpr int per_chunk = OP == ROM_BF16 ? 4 : 2;   // u4 loads per lane per chunk
    const u4 *ap = pk + (size_t)t * (size_t)(kp / kLpChunk) * per_chunk * 64 + lane;
    f4 hi = {0.f, 0.f, 0.f, 0.f}, lo = {0.f, 0.f, 0.f, 0.f};
    const int nch = kp / kLpChunk;   // even
    Frag<OP> f0, f1;
    s4 a[8], x0h[8], x0l[8], x1h[8], x1l[8];
    f0.load(ap, 0);
    f1.load(ap, 1);
    lds_split(x0h, xh_col, 0);
    if constexpr (!SINGLE) lds_split(x0l, xl_col, 0);
    __builtin_amdgcn_sched_barrier(0);
    for (int ch = 0; ch < nch; ch += 2) {
        lds_split(x1h, xh_col, ch + 1);
        if constexpr (!SINGLE) lds_split(x1l, xl_col, ch + 1);
        __builtin_amdgcn_sched_barrier(0);
        f0.operands(a);
        mma_chunk_lp<SINGLE>(a, x0h, x0l, hi, lo);
        __builtin_amdgcn_sched_barrier(0);
        const int n2 = min(ch + 2, nch - 1);
        f0.load(ap, n2);
        lds_split(x0h, xh_col, n2);
        if constexpr (!SINGLE) lds_split(x0l, xl_col, n2);
        __builtin_amdgcn_sched_barrier(0);
        f1.operands(a);
        mma_chunk_lp<SINGLE>(a, x1h, x1l, hi, lo);
        __builtin_amdgcn_sched_barrier(0);
        f1.load(ap, min(ch + 3, nch - 1));
        __builtin_amdgcn_sched_barrier(0);
    }
    H = hi;
    L = lo;
}

struct LpField {
    const u4 *pk;          // packed operator of this half-step
    int T, kp;
    const unsigned short *Xh, *Xl;   // other field's BF16 split, ld ldbx
    int ldbx;
    float *Yh, *Yl;        // updated field FP32 pair, ld ldy
    int ldy;
    unsigned short *Bh, *Bl;         // updated field's BF16 split, ld ldby
    int ldby;
};

// (Yh, Yl) += dt * (scale * (H + L) + forcing), then refresh the BF16 split
// (x_hi only when SINGLE).
template <bool FORCED, bool SINGLE>
__device__ __forceinline__ void finish_tile_lp(const LpField &f, int t, f4 H, f4 L, int lane,
                                               const float *bl, const float *cl, float uh, float ul,
                                               float dtf, float scale, double &ypart) {
    const int j = lane & 3;
    const int i0 = t * kTileRows + 4 * (lane >> 2);
    f4 yh = *(f4 *)(f.Yh + j * f.ldy + i0);
    f4 yl = *(f4 *)(f.Yl + j * f.ldy + i0);
    f4 bb = {0.f, 0.f, 0.f, 0.f}, cc = {0.f, 0.f, 0.f, 0.f};
    if (FORCED) {
        bb = *(const f4 *)(bl + i0);
        cc = *(const f4 *)(cl + i0);
    }
    unsigned short sh[4], sl[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        // scale the compensated product exactly enough: (H + L) * scale
        float Hs = H[r] * scale;
        float Ls = fmaf(L[r], scale, fmaf(H[r], scale, -Hs));
        float F = 0.f, Fe = 0.f;
        if (FORCED) {
            F = bb[r] * uh;
            Fe = fmaf(bb[r], uh, -F) + bb[r] * ul;
        }
        float h = yh[r], l = yl[r];
        dev::comp_update(h, l, Hs, Ls, F, Fe, dtf);
        yh[r] = h;
        yl[r] = l;
        if (FORCED) ypart += (double)cc[r] * ((double)h + (double)l);
        sh[r] = bf16_rne(h);
        sl[r] = bf16_rne(h - bf16_to_f32(sh[r]));
    }
    *(f4 *)(f.Yh + j * f.ldy + i0) = yh;
    *(f4 *)(f.Yl + j * f.ldy + i0) = yl;
    unsigned p0 = (unsigned)sh[0] | ((unsigned)sh[1] << 16), p1 = (unsigned)sh[2] | ((unsigned)sh[3] << 16);
    *reinterpret_cast<unsigned long long *>(f.Bh + j * f.ldby + i0) = (unsigned long long)p0 | ((unsigned long long)p1 << 32);
    if constexpr (!SINGLE) {
        unsigned q0 = (unsigned)sl[0] | ((unsigned)sl[1] << 16), q1 = (unsigned)sl[2] | ((unsigned)sl[3] << 16);
        *reinterpret_cast<unsigned long long *>(f.Bl + j * f.ldby + i0) = (unsigned long long)q0 | ((unsigned long long)q1 << 32);
    }
}

template <int OP, bool FORCED, bool SINGLE>
__device__ __forceinline__ void half_step_lp(const LpField &f, int lane, int w, const float *bl,
                                             const float *cl, float uh, float ul, float dtf,
                                             float scale, double &ypart) {
    const int j = lane & 3;
    for (int t = w; t < f.T; t += kWaves) {
        f4 H, L;
        tile_product_lp<OP, SINGLE>(f.pk, t, f.kp, f.Xh + j * f.ldbx, f.Xl + j * f.ldbx, lane, H, L);
        finish_tile_lp<FORCED, SINGLE>(f, t, H, L, lane, bl, cl, uh, ul, dtf, scale, ypart);
    }
    __syncthreads();
}

// Initial FP32 pair (x, 0) and BF16 split of a column block.
__device__ __forceinline__ void load_field(const float *src, int K, int Kp, int col0, int M, float *hi,
                                           float *lo, int ld, unsigned short *bh, unsigned short *bl_,
                                           int ldb, int tid) {
    for (int idx = tid; idx < NB * Kp; idx += kThreads) {
        int jj = idx / Kp, i = idx - jj * Kp, mm = col0 + jj;
        float x = (mm < M && i < K) ? src[(size_t)mm * K + i] : 0.f;
        hi[jj * ld + i] = x;
        lo[jj * ld + i] = 0.f;
        unsigned short h = bf16_rne(x);
        bh[jj * ldb + i] = h;
        bl_[jj * ldb + i] = bf16_rne(x - bf16_to_f32(h));
    }
}

template <int OP, bool SINGLE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void rank2_lowp_kernel(Rank2Args a, float scale) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int kvp = a.kvp, ksp = a.ksp;
    const int ldv = kvp + 4, lds_ = ksp + 4;
    const int ldbv = kvp + 8, ldbs = ksp + 8;   // BF16 columns, 16-byte aligned
    float *Vh = reinterpret_cast<float *>(smem);
    float *Vl = Vh + NB * ldv;
    float *Sh = Vl + NB * ldv;
    float *Sl = Sh + NB * lds_;
    double *yp = reinterpret_cast<double *>(Sl + NB * lds_);
    float *bl = reinterpret_cast<float *>(yp + kWaves * NB);
    float *cl = bl + kvp;
    unsigned short *VBh = reinterpret_cast<unsigned short *>(cl + kvp);
    unsigned short *VBl = VBh + NB * ldbv;
    unsigned short *SBh = VBl + NB * ldbv;
    unsigned short *SBl = SBh + NB * ldbs;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int col0 = blockIdx.x * NB;
    const float *bv = static_cast<const float *>(a.b);
    const float *cv = static_cast<const float *>(a.c);
    load_field(static_cast<const float *>(a.V), a.kv, kvp, col0, a.M, Vh, Vl, ldv, VBh, VBl, ldbv, tid);
    load_field(static_cast<const float *>(a.S), a.ks, ksp, col0, a.M, Sh, Sl, lds_, SBh, SBl, ldbs, tid);
    for (int i = tid; i < kvp; i += kThreads) {
        bl[i] = i < a.kv ? bv[i] : 0.f;
        cl[i] = (cv != nullptr && i < a.kv) ? cv[i] : 0.f;
    }
    const int j = lane & 3;
    const int m = col0 + j;
    const bool mok = m < a.M;
    const double muj = mok ? a.mu[m] : 1.0;
    const float dtf = (float)a.dt;
    const bool probe = cv != nullptr;
    double Jacc = 0.0;
    const LpField fv = {static_cast<const u4 *>(a.avs), kvp / kTileRows, ksp, SBh, SBl, ldbs, Vh, Vl, ldv, VBh, VBl, ldbv};
    const LpField fs = {static_cast<const u4 *>(a.asv), ksp / kTileRows, kvp, VBh, VBl, ldbv, Sh, Sl, lds_, SBh, SBl, ldbs};
    __syncthreads();

    for (int64_t k = 0; k < a.nsteps; ++k) {
        const double t = (double)(a.n0 + k) * a.dt;
        const double u64 = mok ? dev::forcing(a.source, t, muj) : 0.0;
        const float uh = (float)u64;
        const float ul = (float)(u64 - (double)uh);
        double ypart = 0.0;
        half_step_lp<OP, true, SINGLE>(fv, lane, w, bl, cl, uh, ul, dtf, scale, ypart);
        if (probe) {
            for (int off = 4; off < 64; off <<= 1) ypart += __shfl_xor(ypart, off, 64);
            if (lane < NB) yp[w * NB + lane] = ypart;
        }
        double dummy = 0.0;
        half_step_lp<OP, false, SINGLE>(fs, lane, w, bl, cl, 0.f, 0.f, dtf, scale, dummy);
        if (probe && tid < NB && col0 + tid < a.M) {
            double yv = 0.0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) yv += yp[q * NB + tid];
            Jacc += a.dt * (yv * yv);
            if (a.y) a.y[(size_t)k * a.M + col0 + tid] = yv;
        }
    }
    float *Vout = static_cast<float *>(a.V);
    float *Sout = static_cast<float *>(a.S);
    for (int idx = tid; idx < NB * kvp; idx += kThreads) {
        int jj = idx / kvp, i = idx - jj * kvp, mm = col0 + jj;
        if (mm < a.M && i < a.kv) Vout[(size_t)mm * a.kv + i] = Vh[jj * ldv + i] + Vl[jj * ldv + i];
    }
    for (int idx = tid; idx < NB * ksp; idx += kThreads) {
        int jj = idx / ksp, i = idx - jj * ksp, mm = col0 + jj;
        if (mm < a.M && i < a.ks) Sout[(size_t)mm * a.ks + i] = Sh[jj * lds_ + i] + Sl[jj * lds_ + i];
    }
    if (probe && a.J && tid < NB && col0 + tid < a.M) a.J[col0 + tid] += Jacc;
}

// ---- setup: quantise and pack -------------------------------------------

// max |fp32(x)| over n values, as the bit pattern of a non-negative float
__global__ void amax_kernel(const double *__restrict__ x, int64_t n, unsigned *out) {
    float m = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf((float)x[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// E4M3 ("fn": max 448, no infinities), round to nearest even, saturating,
// from an FP32 value already in the representable range scale.
__device__ __forceinline__ unsigned char e4m3_rne_sat(float f) {
    unsigned char s = f < 0.f ? 0x80 : 0x00;
    float a = fminf(fabsf(f), 448.f);
    if (!(a > 0.f)) return s;                      // +-0
    int e;
    frexpf(a, &e);                                 // a in [2^(e-1), 2^e)
    int ex = e - 1;                                // unbiased exponent
    int qexp = (ex < -6 ? -6 : ex) - 3;            // quantum 2^qexp (3 mantissa bits)
    float q = rintf(ldexpf(a, -qexp));             // RNE to a multiple of the quantum
    float r = ldexpf(q, qexp);
    if (r > 448.f) r = 448.f;
    // encode r
    if (r < ldexpf(1.f, -6)) {                     // subnormal: m * 2^-9
        int mm = (int)rintf(ldexpf(r, 9));
        return s | (unsigned char)mm;
    }
    int e2;
    float fr = frexpf(r, &e2);                     // r = fr * 2^e2, fr in [0.5, 1)
    int biased = (e2 - 1) + 7;
    int mant = (int)rintf((fr * 2.f - 1.f) * 8.f);
    if (mant == 8) { mant = 0; ++biased; }
    return s | (unsigned char)((biased << 3) | mant);
}

// BF16 packing: pk[t][kq][lane][8] = bf16(fp32(A[64 t + lane][8 kq + e]))
__global__ void pack_bf16_kernel(const double *__restrict__ A, int rows, int cols, int prow, int pcol,
                                 unsigned short *__restrict__ pk) {
    const int64_t total = (int64_t)prow * pcol;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = idx;
        const int e = (int)(r % 8); r /= 8;
        const int lane = (int)(r % 64); r /= 64;
        const int kq = (int)(r % (pcol / 8)); r /= (pcol / 8);
        const int i = (int)r * kTileRows + lane, k = kq * 8 + e;
        float v = (i < rows && k < cols) ? (float)A[i + (int64_t)k * rows] : 0.f;
        pk[idx] = bf16_rne(v);
    }
}

// FP8 packing: pk[t][kq][lane][16] = e4m3(fp32(A[64 t + lane][16 kq + e]) / scale)
__global__ void pack_fp8_kernel(const double *__restrict__ A, int rows, int cols, int prow, int pcol,
                                const unsigned *amax_bits, unsigned char *__restrict__ pk) {
    const float amax = __uint_as_float(*amax_bits);
    const float scale = amax > 0.f ? amax / 448.f : 1.f;
    const int64_t total = (int64_t)prow * pcol;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = idx;
        const int e = (int)(r % 16); r /= 16;
        const int lane = (int)(r % 64); r /= 64;
        const int kq = (int)(r % (pcol / 16)); r /= (pcol / 16);
        const int i = (int)r * kTileRows + lane, k = kq * 16 + e;
        float v = (i < rows && k < cols) ? (float)A[i + (int64_t)k * rows] : 0.f;
        pk[idx] = e4m3_rne_sat(v / scale);
    }
}

// Inverse of the packings: column-major FP64 operator (rows x cols) as the
// products see it (BF16 value, or E4M3 value times the scale).
__global__ void unpack_lowp_kernel(const void *__restrict__ pk, int rows, int cols, int prow, int pcol,
                                   int op, double scale, double *__restrict__ A) {
    const int64_t total = (int64_t)rows * cols;
    const int per = op == ROM_BF16 ? 8 : 16;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % rows), k = (int)(idx / rows);
        const int t = i / kTileRows, lane = i % kTileRows, kq = k / per, e = k % per;
        const int64_t p = (((int64_t)t * (pcol / per) + kq) * 64 + lane) * per + e;
        double v;
        if (op == ROM_BF16) {
            v = (double)bf16_to_f32(static_cast<const unsigned short *>(pk)[p]);
        } else {
            const unsigned char b = static_cast<const unsigned char *>(pk)[p];
            typedef float f2 __attribute__((ext_vector_type(2)));
            f2 d = __builtin_amdgcn_cvt_pk_f32_fp8((int)b, false);
            v = (double)d.x * scale;
        }
        A[idx] = v;
    }
}

int grid_for(int64_t n, int cap) {
    int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

size_t rank2_lowp_lds_bytes(int kvp, int ksp) {
    return sizeof(float) * (size_t)NB * 2 * ((kvp + 4) + (ksp + 4)) + sizeof(double) * kWaves * NB +
           sizeof(float) * 2 * (size_t)kvp + sizeof(unsigned short) * (size_t)NB * 2 * ((kvp + 8) + (ksp + 8));
}

hipError_t launch_rank2_lowp(const Rank2Args &a, rom_dtype op, float scale, hipStream_t st) {
    const int blocks = (a.M + NB - 1) / NB;
    const size_t lds = rank2_lowp_lds_bytes(a.kvp, a.ksp);
    if (op == ROM_BF16 && a.single)
        hipLaunchKernelGGL((rank2_lowp_kernel<ROM_BF16, true>), dim3(blocks), dim3(kThreads), lds, st, a, 1.0f);
    else if (op == ROM_BF16)
        hipLaunchKernelGGL((rank2_lowp_kernel<ROM_BF16, false>), dim3(blocks), dim3(kThreads), lds, st, a, 1.0f);
    else if (a.single)
        hipLaunchKernelGGL((rank2_lowp_kernel<ROM_F8E4M3, true>), dim3(blocks), dim3(kThreads), lds, st, a, scale);
    else
        hipLaunchKernelGGL((rank2_lowp_kernel<ROM_F8E4M3, false>), dim3(blocks), dim3(kThreads), lds, st, a, scale);
    return hipGetLastError();
}

hipError_t rank2_lowp_configure() {
    const void *fns[] = {(const void *)rank2_lowp_kernel<ROM_BF16, false>,
                         (const void *)rank2_lowp_kernel<ROM_BF16, true>,
                         (const void *)rank2_lowp_kernel<ROM_F8E4M3, false>,
                         (const void *)rank2_lowp_kernel<ROM_F8E4M3, true>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_amax(const double *x, int64_t n, unsigned *out, hipStream_t st) {
    hipLaunchKernelGGL(amax_kernel, dim3(grid_for(n, 2048)), dim3(256), 0, st, x, n, out);
    return hipGetLastError();
}

hipError_t launch_pack_lowp(const double *A, int rows, int cols, int prow, int pcol, rom_dtype op,
                            const unsigned *amax_bits, void *pk, hipStream_t st) {
    const int64_t total = (int64_t)prow * pcol;
    if (op == ROM_BF16)
        hipLaunchKernelGGL(pack_bf16_kernel, dim3(grid_for(total, 8192)), dim3(256), 0, st, A, rows, cols,
                           prow, pcol, static_cast<unsigned short *>(pk));
    else
        hipLaunchKernelGGL(pack_fp8_kernel, dim3(grid_for(total, 8192)), dim3(256), 0, st, A, rows, cols,
                           prow, pcol, amax_bits, static_cast<unsigned char *>(pk));
    return hipGetLastError();
}

hipError_t launch_unpack_lowp(const void *pk, int rows, int cols, int prow, int pcol, rom_dtype op,
                              double scale, double *A, hipStream_t st) {
    const int64_t total = (int64_t)rows * cols;
    hipLaunchKernelGGL(unpack_lowp_kernel, dim3(grid_for(total, 8192)), dim3(256), 0, st, pk, rows, cols, prow,
                       pcol, (int)op, scale, A);
    return hipGetLastError();
}

}  // namespace rom
