// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "rom.h"

namespace rom {

// Row tile of the rank-2 MFMA kernel: one v_mfma_f32_4x4x1f32 (16 blocks)
// covers 64 operator rows x 4 sample columns for one k.
constexpr int kTileRows = 64;
// Sample columns of one column set of the column-block kernels (a
// workgroup of the FP32 kernel owns one or two sets).
constexpr int kColBlock = 4;
// Largest Kv_pad + Ks_pad the LDS-resident state of the rank-2 kernels holds.
constexpr int kMaxPadSum = 4096;
// Largest padded K of the FP32 row-split schedule: a group's K / 64
// workgroups share one XCD (32 CUs).
constexpr int kMaxSplitK = 2048;

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Failure-handling test hook (rom_debug_force_timeout): when set, every
// bounded in-kernel wait of the row-split kernels waits for one arrival too
// many with a short poll budget, so it runs out and reports ROM_E_TIMEOUT
// while the kernel still ends normally.
extern bool g_forced_timeout;

}  // namespace rom

struct rom_ctx {
    int device = 0;
    int kv = 0, ks = 0;        // reduced sizes
    int kvp = 0, ksp = 0;      // padded to multiples of 64
    double dt = 0.0;           // as given
    rom_dtype op_type = ROM_F64, state_type = ROM_F64;
    uint32_t flags = 0;
    bool skew = false;         // Asv == -Avs^T exactly

    // Column-major operators in the state type (rank-1 GEMV and FP64 path):
    // Avs kv x ks (ld kv), Asv ks x kv (ld ks).
    void *avs_cm = nullptr, *asv_cm = nullptr;
    // FP32 operators packed for the 4x4x1 MFMA kernel:
    // avs_pk[t][k/4][lane][k%4] = Avs[64 t + lane][k], zero padded to kvp x ksp;
    // asv_pk likewise for Asv (ksp x kvp).
    float *avs_pk = nullptr, *asv_pk = nullptr;
    // Low-precision operators (op_type BF16 / FP8): packed panels as void*
    // in avs_lp / asv_lp, FP8 per-tensor scale (shared by both operators).
    void *avs_lp = nullptr, *asv_lp = nullptr;
    float op_scale = 1.0f;
    // Source vector in the state type, zero padded to kvp entries.
    void *b = nullptr;
    // Transposed operators packed like avs_pk / asv_pk for the adjoint sweep
    // (lazily): asvT_pk holds Asv^T (Kv x Ks), avsT_pk holds Avs^T (Ks x Kv).
    float *asvT_pk = nullptr, *avsT_pk = nullptr;
    // Adjoint workspace (checkpoints, segment traces), grown on demand.
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // FP64 column-major copy of Avs exactly as the products use it (for the
    // energy), built on first use.
    double *avs_e64 = nullptr;
    // Row-split schedule (low-precision runs): operators as BF16 MFMA
    // fragments in the split layout (built on first use), its workspace
    // (exchange rows, probe partials, barrier counters), and whether this
    // device can host it (-1 unknown, 0 no, 1 yes).
    void *avs_sp = nullptr, *asv_sp = nullptr;
    // Row-split FP32 packs of Asv^T and Avs^T for the adjoint's reverse
    // sweep on the row-split schedule (lazily).
    void *asvT_sp = nullptr, *avsT_sp = nullptr;
    // Second row-split workspace (the reverse sweep beside the recompute).
    void *sp_ws2 = nullptr;
    size_t sp_ws2_bytes = 0;
    void *sp_ws = nullptr;
    size_t sp_ws_bytes = 0;
    int sp_ok = -1;
    // Operator-resident schedule (skew FP32 pairs, Kv, Ks <= 256): Avs in
    // the per-thread tile order of its kernel, built by rom_create.
    void *res_pk = nullptr;
    // Schedule of the last FP32-state rank-2 run (a rom_schedule, -1 none
    // yet).
    int last_schedule = -1;
    // Device status words: [0] scratch of rom_create, [1] in-kernel error
    // (ROM_E_TIMEOUT), [2] abort flag of the row-split barriers.
    int *status = nullptr;
    // Adjoint pipeline (built on first use): side streams (default
    // priority) that recompute the next segment ([0]) and run the gradient
    // products of the last one ([1]) while the caller's stream runs the
    // current segment's reverse sweep, and their events (see rom_adjoint).
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t ev[13] = {};
    // Receiver runs: two sets of chunk traces (states and probe scratch),
    // and events [b] set b stepped, [2 + b] set b read, [4] side stream
    // drained.
    void *rc_ws = nullptr;
    size_t rc_ws_bytes = 0;
    hipEvent_t rc_ev[5] = {};
    // Panel schedule (FP32, any size): row-major padded operator copies
    // (built on first use) and the run workspace (states hi / lo, probe
    // partials), grown on demand.
    void *avs_rm = nullptr, *asv_rm = nullptr;
    void *pn_ws = nullptr;
    size_t pn_ws_bytes = 0;
};

namespace rom {

struct Rank2Args {
    const void *avs;      // packed (F32 MFMA) or column-major (VALU path)
    const void *asv;
    const void *b;        // kvp entries
    const void *c;        // kv entries or null
    const double *mu;     // M
    void *V, *S;          // caller states (column-major, ld kv / ks)
    double *J;            // M or null (accumulated)
    double *y;            // nsteps x M or null
    int kv, ks, kvp, ksp, M;
    int64_t n0, nsteps;
    double dt;            // FP64 step (forcing time t_n = n * dt)
    // forward only: state traces ((nsteps + 1) x K x M) or null
    float *vtr = nullptr, *str = nullptr;
    // adjoint only: forward probe trace (nsteps x M), W / Q traces
    // (nsteps x K x M) and dJ/dmu (M, accumulated)
    const double *ytr = nullptr;
    float *wtr = nullptr, *qtr = nullptr;
    double *dmu = nullptr;
    // column sets per workgroup of the FP32 column-block kernels (grouped
    // runs read it per instance): 1 = 4 samples, 2 = 8 samples
    int nset = 1;
    // source signal: 0 Ricker, 1 first derivative of a Gaussian
    int source = 0;
    // BF16 / FP8 operators: 1 = the state enters the products as bf16(x)
    // alone (one MFMA pass), 0 = as the BF16 pair (x_hi, x_lo)
    int single = 0;
};

// Operator-resident kernel (skew pairs, FP32): whether padded sizes fit it,
// the bytes of its operator pack, the pack from a column-major FP32 Avs, and
// the run (a.avs = the pack).
// Panel schedule (FP32 operators and states, or FP64 states; any Kv, Ks):
// one tiled MFMA product launch per half-step.  Sizes padded to 128;
// operator copies of panel_op_bytes each; run workspace of panel_ws_bytes.
int panel_pad(int k);
// FP64 states take the panel schedule from Kv_pad + Ks_pad = kPanelF64From
// (measured against the vector-ALU column blocks, us per step at M = 256:
// K = 256 36.0 / 58.7, K = 384 104 / 80, K = 1024 1971 / 69)
constexpr int kPanelF64From = 768;
size_t panel_op_bytes(int kv, int ks, bool f64);
size_t panel_ws_bytes(int kv, int ks, int M, bool f64);
hipError_t launch_panel_pack(const void *avs_cm, const void *asv_cm, int kv, int ks, bool f64, void *avs_rm,
                             void *asv_rm, hipStream_t st);
hipError_t launch_rank2_panel(const void *avs_rm, const void *asv_rm, const Rank2Args &a, bool f64, void *ws,
                              hipStream_t st);

bool rank2_resident_applies(int kvp, int ksp);
size_t rank2_resident_pack_bytes(int kvp, int ksp);
hipError_t launch_resident_pack(const float *A, int kv, int ks, int kvp, int ksp, void *pk, hipStream_t st);
hipError_t launch_rank2_resident(const Rank2Args &a, hipStream_t st);
// FP64 states: the operator-resident schedule in FP64 for skew pairs with
// Kv_pad, Ks_pad <= 128 and other pairs with Kv_pad Ks_pad <= 8192 (a.avs,
// a.asv = the column-major FP64 operators).
bool rank2_resident64_applies(int kvp, int ksp, bool skew);
hipError_t launch_rank2_resident64(const Rank2Args &a, bool skew, hipStream_t st);

// Rank-1 formulation of M samples in one launch (a.avs / a.asv the
// column-major FP32 operators, kv, ks <= 1024).
hipError_t launch_rank1_batch(const Rank2Args &a, hipStream_t st);

// Launchers (return hipSuccess or the launch error).
hipError_t launch_rank2_f32_mfma(const Rank2Args &a, int nset, hipStream_t st);
size_t rank2_f32_mfma_lds_bytes(int kvp, int ksp, int nset);
hipError_t launch_adjoint_f32_mfma(const Rank2Args &a, hipStream_t st);
// The forward steps n0 .. n0 + nsteps - 1 undone from the state after them
// (a.V, a.S in/out), the state before each step stored at trace entry
// n - n0 of a.vtr / a.str (entry nsteps: the state given).
hipError_t launch_inverse_f32_mfma(const Rank2Args &a, hipStream_t st);
// ytr (len x M) = c^T of trace entries 1 .. len of vtr ((len + 1) x M x kv).
hipError_t launch_probe_trace(const float *vtr, const float *c, int kv, int M, int64_t len, double *ytr,
                              hipStream_t st);
hipError_t launch_rank2_lowp(const Rank2Args &a, rom_dtype op, float scale, hipStream_t st);
hipError_t launch_amax(const double *x, int64_t n, unsigned *out, hipStream_t st);
hipError_t launch_unpack_lowp(const void *pk, int rows, int cols, int prow, int pcol, rom_dtype op,
                              double scale, double *A, hipStream_t st);
hipError_t launch_pack_lowp(const double *A, int rows, int cols, int prow, int pcol, rom_dtype op,
                            const unsigned *amax_bits, void *pk, hipStream_t st);
// Grouped forward run over device arrays of per-instance arguments and
// (instance, column block) items, steps n0 .. n0+nsteps-1 for all; LDS of
// lds_bytes (the largest instance's need).
hipError_t launch_grouped_f32_mfma(const Rank2Args *inst_dev, const int2 *items_dev, int nitems,
                                   size_t lds_bytes, int64_t n0, int64_t nsteps, hipStream_t st);
// dA (rows x cols, FP64, column-major) += alpha * X * Y^T with X rows x R and
// Y cols x R column-major FP32 (ld rows / cols).  `part` is a workspace of
// gemm_nt_splits(rows, cols) * rows * cols doubles.
int gemm_nt_splits(int rows, int cols);
// Row-split low-precision kernel.
size_t rank2_split_lds_bytes();
int rank2_split_groups(int kv, int ks, int kvp, int ksp, int M, bool f32);
bool rank2_split_k_ok(int kvp, bool f32);
size_t rank2_split_workspace_bytes(int kvp, int G);
// Workspace of a launch with xfloats exchange floats per field and ypd
// probe-partial doubles.
size_t rank2_split_ws_bytes(size_t xfloats, size_t ypd);
hipError_t launch_split_pack(const void *lp, bool fp8, int kvp, int ksp, void *dst, hipStream_t st);
// mode 0: plain run; FP32 only: 1, traced (a.vtr, a.str every step, probe
// trace a.y), 2, adjoint (a.V, a.S hold P, Q; opv, ops the split packs of
// Asv^T, Avs^T; a.b the probe c, a.c the source b; a.ytr, a.wtr, a.qtr,
// a.dmu as for the column-block adjoint launch).
hipError_t launch_rank2_split(const void *opv, const void *ops, const Rank2Args &a, float scale, void *ws,
                              int G, int *status, bool f32, hipStream_t st, int mode = 0);
// Width index (16 << wi columns) at which two FP32 runs of M samples at
// padded K fit one launch side by side, or -1.
int rank2_split_dual_width(int kvp, int M);
// Run r0 traced (mode 1) and r1 in adjoint mode (mode 2) side by side in
// one cooperative launch: same kvp and M, each with its own workspace of
// rank2_split_workspace_bytes(kvp, G) bytes (G = ceil(M / 64)).
hipError_t launch_rank2_split_dual(const void *opv0, const void *ops0, const Rank2Args &r0, void *ws0,
                                   const void *opv1, const void *ops1, const Rank2Args &r1, void *ws1, int G,
                                   int *status, hipStream_t st);
size_t rank2_split_f32_lds_bytes();
// Split-layout FP32 pack of a column-major rows x cols matrix, or with
// `trans` of the transpose of a column-major cols x rows matrix.
hipError_t launch_split_pack_f32(const float *A, int rows, int cols, int prow, int pcol, void *dst, hipStream_t st,
                                 bool trans = false);
hipError_t rank2_split_configure();
// Static scratch of the allocation-free row-split run: its size, and its
// device address on `device` (which must be current at the first call for
// that device; the lookup is done once per device).
size_t rank2_split_static_bytes();
hipError_t rank2_split_static_scratch(int device, void **ptr);
// Receivers: Y and ensemble statistics of L steps from a chunk's state
// traces (see k_receivers.hip).
size_t receivers_lds_bytes(int kv, int M, int R);
hipError_t launch_receivers(const float *vtr, int kv, int M, int L, const float *C, int R, double *Y,
                            double *stats, hipStream_t st);
hipError_t receivers_configure();
bool rank2_split_device_ok();
hipError_t launch_gemm_nt_acc64(const float *X, const float *Y, int rows, int cols, int64_t R,
                                double alpha, double *dA, double *part, hipStream_t st);
hipError_t launch_f64_to_f32(const double *src, float *dst, int64_t n, hipStream_t st);
hipError_t launch_energy(const double *A64, int kv, int ks, double dt, rom_dtype st_type, const void *V,
                         const void *S, int M, double *E, hipStream_t st);
// Pack a column-major FP32 matrix (rows x cols, or its transpose when
// `transpose`) into the 4x4x1 MFMA panel layout with padded sizes.
hipError_t launch_pack_f32_from_f32(const float *A, int rows, int cols, bool transpose, int prow,
                                    int pcol, float *pk, hipStream_t st);
template <typename T>
hipError_t launch_rank2_valu(const Rank2Args &a, hipStream_t st);

template <typename T>
hipError_t launch_rank1_step(const void *avs_cm, const void *asv_cm, const void *b, int kv,
                             int ks, double dt, int64_t n, double mu, int source, void *v, void *s,
                             hipStream_t st);

// Grouped row-split run (FP32 operators, Kv == Ks, each group with its own
// padded K): one descriptor per 64-sample group.  opv / ops are the
// instance's row-split FP32 operator packs, b its padded FP32 source, mu /
// V / S its own arrays (ld kv); the group owns samples col0 .. col0 + 63
// of the instance's M; xoff is the offset (floats) of its exchange block of
// 64 kp floats within each field's exchange buffer of the launch.
struct SplitGroup {
    const void *opv, *ops;
    const float *b;
    const double *mu;
    float *V, *S;
    double dt;
    int64_t xoff;
    int kv, kp, M, col0, source;
};
// Groups one cooperative launch holds at padded size kvp: 8 floor(32 / (kvp / 64)).
int rank2_split_groups_per_launch(int kvp);
// Groups g0 .. g0 + G - 1 of the device table grp_dev, nsteps steps from
// n0.  smap_dev: the launch's slot map, 256 ints, entry 32 xcc + s = 32 lg
// + r (group g0 + lg, row tile r) for the s-th workgroup on XCD xcc, or -1;
// every group's kp / 64 row tiles on one XCD.  ws holds
// rank2_split_ws_bytes(xfloats, 0) bytes (xfloats: the groups' 64 kp
// summed); status as for launch_rank2_split.
hipError_t launch_grouped_split_f32(const SplitGroup *grp_dev, int g0, int G, const int *smap_dev, size_t xfloats,
                                    void *ws, int *status, int64_t n0, int64_t nsteps, hipStream_t st);

// Full-order side.  A sparse operator on the device: CSR, and when no row
// holds more than 8 entries also a padded (ELL) copy of width W in {2, 4, 8}
// (row r's entries at [r W, r W + W), unused slots with column -1), which
// the kernels then use.
struct FomCsr {
    const int *ptr = nullptr, *col = nullptr;
    const double *val = nullptr;
    int nrows = 0;
    const int *ecol = nullptr;
    const double *eval = nullptr;
    int W = 0;
};
// One FOM leapfrog step n (t_n = n dt) of M row-major samples:
// V += dt (Av S + f u^T), then S += dt As V.
hipError_t launch_fom_step(const FomCsr &Av, const FomCsr &As, const double *f, const double *mu, int M, int64_t n,
                           double dt, int source, double *V, double *S, hipStream_t st);
// Y (rows x M, row-major) = A X (X row-major with M columns).
hipError_t launch_fom_spmm(const FomCsr &A, const double *X, int M, double *Y, hipStream_t st);
// C (K1 x K2 column-major) = P^T Q, P (N x K1) and Q (N x K2) row-major;
// part holds gemm_tn_splits(N, K1, K2) K1 K2 doubles.
int gemm_tn_splits(int64_t N, int K1, int K2);
hipError_t launch_gemm_tn(const double *P, const double *Q, int64_t N, int K1, int K2, double *part, double *C,
                          hipStream_t st);
// Y (N x K2 row-major) = X (N x K1 row-major) B (K1 x K2 column-major).
hipError_t launch_gemm_nn(const double *X, const double *B, int64_t N, int K1, int K2, double *Y, hipStream_t st);

// Error reporting of the C-ABI (rom_last_error text), for the API sources.
rom_status api_fail(rom_status s, const std::string &msg);
rom_status api_hip_fail(hipError_t e, const char *where);

// *flag |= 1 if any of the n values is NaN or infinite.
hipError_t launch_nonfinite(const void *x, int64_t n, bool f64, int *flag, hipStream_t st);

// Affine operators: coefficients of up to kMaxAffine terms, by value.
constexpr int kMaxAffine = 16;
struct AffineCoeffs {
    double c[kMaxAffine];
};
// out (n) = sum_q th.c[q] terms[q n ..], q = 0 .. Q-1 in order (FP64).
hipError_t launch_affine_combine(const double *terms, int Q, int64_t n, const AffineCoeffs &th, double *out,
                                 hipStream_t st);

// Setup kernels: FP64 staging -> state-type column-major copies and packed
// MFMA panels.
hipError_t launch_convert(const double *src, void *dst, int64_t n, rom_dtype to, hipStream_t st);
hipError_t launch_convert_f32_to_f64(const float *src, double *dst, int64_t n, hipStream_t st);
hipError_t launch_pack_f32(const double *A, int rows, int cols, int rowsp, int colsp, float *pk,
                           hipStream_t st);

}  // namespace rom

namespace rom {
// Row-split part of a grouped plan: the 64-sample groups of the instances
// it covers, ordered by launch, and per launch its first group, group
// count, exchange floats per field and slot map (256 entries).
struct SplitPlan {
    std::vector<SplitGroup> groups;
    std::vector<int> owner;                 // instance of each group
    std::vector<int> g0, ng;                // per launch
    std::vector<size_t> xfloats;            // per launch
    std::vector<int> smap;                  // 256 per launch
    size_t ws_bytes = 0;                    // the largest launch's workspace
    int kmin = 0;                           // smallest padded K it covers
};
// Device copies of a row-split plan's tables.
struct SplitDev {
    void *groups = nullptr;    // SplitGroup [n]
    int *smap = nullptr;       // 256 per launch
    void *ws = nullptr;
    int *status = nullptr;     // [4]: [1] ROM_E_TIMEOUT, [2] abort flag
};
}  // namespace rom

struct rom_group {
    int device = 0;
    int G = 0, nitems = 0;
    size_t lds_bytes = 0;
    void *dev = nullptr;          // [G] Rank2Args then [nitems] int2 items
    const rom::Rank2Args *inst = nullptr;
    const int2 *items = nullptr;
    // row-split part (used when ngroups > 0): its launches, then column
    // blocks over the nrest items of the other instances
    int ngroups = 0, nrest = 0;
    rom::SplitPlan plan;
    rom::SplitDev sp;
    void *rest = nullptr;         // [nrest] int2 items
    float us[2] = {-1.f, -1.f};   // timed per-step us: column blocks only, best plan with row-split
};

// Affine family of operator pairs (rank-3 direction): the Q terms of both
// operators and the padded source on the device, for assembling instances.
struct rom_affine {
    rom_config cfg{};
    int Q = 0;
    bool skew = false;               // every term pair is skew
    double *terms = nullptr;         // device: Q x (Kv x Ks) Avs terms, then Q x (Ks x Kv) Asv terms
    double *bpad = nullptr;          // device: Kv_pad
    std::vector<double> host_avs;    // Avs terms on the host (skew check), if requested
};
