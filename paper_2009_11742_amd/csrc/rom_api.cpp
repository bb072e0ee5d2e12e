// C-ABI of the rank-2 Galerkin ROM library: argument validation, context
// lifetime, uploads and kernel dispatch.  Every entry point validates
// synchronously before enqueueing anything, so ROM_E_ARG means nothing was
// written.  No exception crosses the ABI.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "rom_internal.h"

namespace rom {
size_t rank2_lowp_lds_bytes(int kvp, int ksp);
hipError_t rank2_lowp_configure();
size_t rank2_valu_lds_bytes(rom_dtype st, int kv, int ks, int kvp, int ksp);
hipError_t rank2_f32_mfma_configure();
hipError_t rank2_valu_configure();
}  // namespace rom

namespace {

thread_local std::string g_err;

rom_status fail(rom_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

rom_status hip_fail(hipError_t e, const char *where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return ROM_E_DEVICE;
}

}  // namespace

namespace rom {
bool g_forced_timeout = false;
rom_status api_fail(rom_status s, const std::string &msg) { return fail(s, msg); }
rom_status api_hip_fail(hipError_t e, const char *where) { return hip_fail(e, where); }
}  // namespace rom

namespace {

bool all_finite(const double *x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) return false;
    return true;
}

size_t tsize(rom_dtype t) { return t == ROM_F64 ? 8 : 4; }

// Largest singular value of A (rows x cols, column-major) by power iteration
// on A^T A in FP64, run to a relative change below 1e-13.
double sigma_max(const double *A, int rows, int cols) {
    std::vector<double> x(cols, 1.0), y(rows), z(cols);
    double nrm = sqrt((double)cols);
    for (double &v : x) v /= nrm;
    double lam = 0.0;
    for (int it = 0; it < 5000; ++it) {
        for (int i = 0; i < rows; ++i) y[i] = 0.0;
        for (int j = 0; j < cols; ++j)
            for (int i = 0; i < rows; ++i) y[i] += A[i + (size_t)j * rows] * x[j];
        for (int j = 0; j < cols; ++j) {
            double s = 0.0;
            for (int i = 0; i < rows; ++i) s += A[i + (size_t)j * rows] * y[i];
            z[j] = s;
        }
        double n2 = 0.0;
        for (double v : z) n2 += v * v;
        n2 = sqrt(n2);
        if (n2 == 0.0) return 0.0;
        for (int j = 0; j < cols; ++j) x[j] = z[j] / n2;
        double prev = lam;
        lam = n2;  // Rayleigh estimate of sigma^2 (x normalised)
        if (it > 10 && fabs(lam - prev) <= 1e-13 * lam) break;
    }
    return sqrt(lam);
}

void hfree(void *p) {
    if (p) (void)hipFree(p);
}

// Read and clear the in-kernel wait words status[1] (ROM_E_TIMEOUT) and
// status[2] (abort flag) once the work that may set them has completed
// (the copies synchronise with the device).  `timed_out` tells whether a
// bounded wait ran out.
rom_status take_timeout(int *status, bool &timed_out, const char *who) {
    int w[2] = {0, 0};
    timed_out = false;
    hipError_t e = hipMemcpy(w, status + 1, sizeof(w), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, who);
    if (w[0] != 0 || w[1] != 0) {
        e = hipMemset(status + 1, 0, sizeof(w));
        if (e != hipSuccess) return hip_fail(e, who);
        timed_out = w[0] == ROM_E_TIMEOUT;
    }
    return ROM_OK;
}

void free_ctx(rom_ctx *c) {
    if (!c) return;
    // work still on the internal streams may read the buffers below
    for (hipStream_t sd : c->side)
        if (sd) (void)hipStreamSynchronize(sd);
    hfree(c->avs_cm);
    hfree(c->asv_cm);
    hfree(c->avs_pk);
    hfree(c->asv_pk);
    hfree(c->avs_lp);
    hfree(c->asv_lp);
    hfree(c->avs_e64);
    hfree(c->b);
    hfree(c->asvT_pk);
    hfree(c->avsT_pk);
    hfree(c->ws);
    hfree(c->avs_sp);
    hfree(c->asv_sp);
    hfree(c->asvT_sp);
    hfree(c->avsT_sp);
    hfree(c->sp_ws2);
    hfree(c->res_pk);
    hfree(c->sp_ws);
    hfree(c->status);
    for (hipStream_t &sd : c->side)
        if (sd) (void)hipStreamDestroy(sd);
    for (hipEvent_t &ev : c->ev)
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t &ev : c->rc_ev)
        if (ev) (void)hipEventDestroy(ev);
    hfree(c->rc_ws);
    hfree(c->avs_rm);
    hfree(c->asv_rm);
    hfree(c->pn_ws);
    delete c;
}

bool g_configured = false;

// Source signal of a context (rom_config flag ROM_SOURCE_GAUSS1).
int ctx_source(const rom_ctx *c) { return (c->flags & ROM_SOURCE_GAUSS1) ? 1 : 0; }

// Row-split groups for a rank-2 run of M samples with FP32 states, or 0 if
// the row-split kernels do not apply (Kv == Ks, padded K a multiple of 64 in
// [128, 2048] with FP32 operators, a multiple of 128 up to 1024 with BF16 / FP8 ones;
// all groups in one launch; a 256-CU gfx950).
int split_candidate(rom_ctx *ctx, int32_t M) {
    const int G = rom::rank2_split_groups(ctx->kv, ctx->ks, ctx->kvp, ctx->ksp, M, ctx->op_type == ROM_F32);
    if (G == 0) return 0;
    if (ctx->sp_ok < 0) ctx->sp_ok = rom::rank2_split_device_ok() ? 1 : 0;
    return ctx->sp_ok == 1 ? G : 0;
}

// Row-split operator packs of a context (built on first use).
rom_status prepare_split_pack(rom_ctx *ctx, hipStream_t st) {
    hipError_t e;
    if (!ctx->avs_sp) {
        const bool f32 = ctx->op_type == ROM_F32;
        const size_t bytes = (f32 ? sizeof(float) : sizeof(uint16_t)) * (size_t)ctx->kvp * ctx->ksp;
        e = hipMalloc(&ctx->avs_sp, bytes);
        if (e == hipSuccess) e = hipMalloc(&ctx->asv_sp, bytes);
        if (e != hipSuccess) {
            hfree(ctx->avs_sp); hfree(ctx->asv_sp);
            ctx->avs_sp = ctx->asv_sp = nullptr;
            return fail(ROM_E_NOMEM, "rom_run_rank2: device allocation failed");
        }
        if (f32) {
            e = rom::launch_split_pack_f32(static_cast<const float *>(ctx->avs_cm), ctx->kv, ctx->ks, ctx->kvp,
                                           ctx->ksp, ctx->avs_sp, st);
            if (e == hipSuccess)
                e = rom::launch_split_pack_f32(static_cast<const float *>(ctx->asv_cm), ctx->ks, ctx->kv, ctx->ksp,
                                               ctx->kvp, ctx->asv_sp, st);
        } else {
            const bool fp8 = ctx->op_type == ROM_F8E4M3;
            e = rom::launch_split_pack(ctx->avs_lp, fp8, ctx->kvp, ctx->ksp, ctx->avs_sp, st);
            if (e == hipSuccess) e = rom::launch_split_pack(ctx->asv_lp, fp8, ctx->ksp, ctx->kvp, ctx->asv_sp, st);
        }
        if (e != hipSuccess) return hip_fail(e, "rom_run_rank2: split pack");
    }
    return ROM_OK;
}

// Row-split operands and workspace of a context (built on first use).
rom_status prepare_split(rom_ctx *ctx, int G, hipStream_t st) {
    rom_status rs = prepare_split_pack(ctx, st);
    if (rs != ROM_OK) return rs;
    hipError_t e;
    const size_t need = rom::rank2_split_workspace_bytes(ctx->kvp, G);
    if (ctx->sp_ws_bytes < need) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "rom_run_rank2: synchronize");
        hfree(ctx->sp_ws);
        ctx->sp_ws = nullptr;
        ctx->sp_ws_bytes = 0;
        e = hipMalloc(&ctx->sp_ws, need);
        if (e != hipSuccess) { ctx->sp_ws = nullptr; return fail(ROM_E_NOMEM, "rom_run_rank2: workspace allocation failed"); }
        ctx->sp_ws_bytes = need;
    }
    return ROM_OK;
}

// Whether the 8-column blocks apply: FP32 operators and the states of 8
// samples within the LDS.
bool cols8_ok(const rom_ctx *ctx) {
    return ctx->op_type == ROM_F32 && ctx->kvp + ctx->ksp <= rom::kMaxPadSum &&
           rom::rank2_f32_mfma_lds_bytes(ctx->kvp, ctx->ksp, 2) <= 160 * 1024;
}

// Launch one rank-2 run with FP32 states on schedule `sched` (a
// rom_schedule that applies; G: row-split groups).
// Panel schedule run (FP32 operators and states, any size).  The operator
// copies and the workspace are allocated on first use; a stream being
// captured cannot allocate, so a captured run needs an earlier uncaptured
// run of at least as many samples on the context.
bool stream_capturing(hipStream_t st);

// Whether the autotuner weighs the panel schedule for a run: FP32
// operators at Kv_pad + Ks_pad >= 2048 (below, its two launches per step
// and its state traffic lose to every resident schedule), and under graph
// capture only once its workspace covers the run.
bool panel_candidate(const rom_ctx *ctx, int M, bool capturing) {
    if (ctx->op_type != ROM_F32 || ctx->state_type != ROM_F32 || ctx->kvp + ctx->ksp < 2048) return false;
    return !capturing || (ctx->avs_rm && ctx->pn_ws_bytes >= rom::panel_ws_bytes(ctx->kv, ctx->ks, M, false));
}

// FP32 operators and states, or FP64 states (the operators as the FP64
// path uses them).
rom_status run_panel(rom_ctx *ctx, const rom::Rank2Args &a, hipStream_t st) {
    const bool capturing = stream_capturing(st);
    const bool f64 = ctx->state_type == ROM_F64;
    const size_t need = rom::panel_ws_bytes(ctx->kv, ctx->ks, a.M, f64);
    if (!ctx->avs_rm || ctx->pn_ws_bytes < need) {
        if (capturing)
            return fail(ROM_E_UNSUPPORTED, "rom_run_rank2: the panel schedule allocates its workspace on first use; "
                                           "run it once outside graph capture with at least this many samples");
        hipError_t e = hipSuccess;
        if (!ctx->avs_rm) {
            const size_t ob = rom::panel_op_bytes(ctx->kv, ctx->ks, f64);
            e = hipMalloc(&ctx->avs_rm, ob);
            if (e == hipSuccess) e = hipMalloc(&ctx->asv_rm, ob);
            if (e == hipSuccess)
                e = rom::launch_panel_pack(ctx->avs_cm, ctx->asv_cm, ctx->kv, ctx->ks, f64, ctx->avs_rm, ctx->asv_rm,
                                           st);
            if (e != hipSuccess) {
                hfree(ctx->avs_rm); hfree(ctx->asv_rm);
                ctx->avs_rm = ctx->asv_rm = nullptr;
                return e == hipErrorOutOfMemory ? fail(ROM_E_NOMEM, "rom_run_rank2: panel operator allocation failed")
                                                : hip_fail(e, "rom_run_rank2: panel pack");
            }
        }
        if (ctx->pn_ws_bytes < need) {
            // the previous workspace may still be read by queued work
            e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(e, "rom_run_rank2: synchronize");
            hfree(ctx->pn_ws);
            ctx->pn_ws = nullptr;
            ctx->pn_ws_bytes = 0;
            e = hipMalloc(&ctx->pn_ws, need);
            if (e != hipSuccess) {
                ctx->pn_ws = nullptr;
                return fail(ROM_E_NOMEM, "rom_run_rank2: panel workspace allocation failed");
            }
            ctx->pn_ws_bytes = need;
        }
    }
    hipError_t e = rom::launch_rank2_panel(ctx->avs_rm, ctx->asv_rm, a, f64, ctx->pn_ws, st);
    if (e != hipSuccess) return hip_fail(e, "rom_run_rank2: panel launch");
    ctx->last_schedule = ROM_SCHEDULE_PANEL;
    return ROM_OK;
}

rom_status launch_fp32_state_run(rom_ctx *ctx, rom::Rank2Args a, int sched, int G, hipStream_t st) {
    hipError_t e;
    const bool lowp = ctx->op_type == ROM_BF16 || ctx->op_type == ROM_F8E4M3;
    a.single = (lowp && (ctx->flags & ROM_STATE_BF16)) ? 1 : 0;
    if (sched == ROM_SCHEDULE_PANEL) {
        return run_panel(ctx, a, st);
    } else if (sched == ROM_SCHEDULE_RESIDENT) {
        a.avs = ctx->res_pk; a.asv = nullptr;
        e = rom::launch_rank2_resident(a, st);
    } else if (sched == ROM_SCHEDULE_ROWSPLIT) {
        rom_status rs = prepare_split(ctx, G, st);
        if (rs != ROM_OK) return rs;
        e = rom::launch_rank2_split(ctx->avs_sp, ctx->asv_sp, a, lowp ? ctx->op_scale : 1.0f, ctx->sp_ws, G,
                                    ctx->status, !lowp, st);
    } else if (lowp) {
        a.avs = ctx->avs_lp; a.asv = ctx->asv_lp;
        e = rom::launch_rank2_lowp(a, ctx->op_type, ctx->op_scale, st);
    } else {
        a.avs = ctx->avs_pk; a.asv = ctx->asv_pk;
        e = rom::launch_rank2_f32_mfma(a, sched == ROM_SCHEDULE_COLUMNS8 ? 2 : 1, st);
    }
    if (e != hipSuccess) return hip_fail(e, "rom_run_rank2: launch");
    return ROM_OK;
}

// Schedule autotuner.  Which kernel schedule is fastest depends on K, M and
// the operator type in ways a fixed rule misses: the row-split kernels pay
// two group barriers per step but stream no operator; the column-block
// kernels never wait but stream the whole operator per CU, 8-column blocks
// half as much per flop on half as many CUs.  Entries are keyed by
// (Kv_pad, Ks_pad, M rounded up to 64, operator type); m_pad = 0 keys the
// per-workgroup tile times of the grouped launch.
struct TuneKey {
    int kvp, ksp, mpad, op;
    bool operator<(const TuneKey &o) const {
        return std::tie(kvp, ksp, mpad, op) < std::tie(o.kvp, o.ksp, o.mpad, o.op);
    }
};
struct TuneEntry {
    int sched;
    float us[ROM_NSCHEDULES];     // per step, < 0: not applicable / not timed
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;
constexpr int kTuneSteps = 32;    // timed steps per schedule of a run shape
constexpr int kTileSteps = 256;   // timed steps per tile of one workgroup

bool tune_find(const TuneKey &k, TuneEntry &out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(k);
    if (it == g_tune.end()) return false;
    out = it->second;
    return true;
}

void tune_store(const TuneKey &k, const TuneEntry &te) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[k] = te;
}

bool stream_capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

// Time each schedule of `cands` (bit per rom_schedule) for `nsteps` steps of
// `run` (its M) on scratch states, after a 2-step warm-up; best of two runs,
// per step, into us (entries not in cands untouched).
rom_status time_schedules(rom_ctx *ctx, const rom::Rank2Args &run, unsigned cands, int G, int64_t nsteps,
                          hipStream_t st, float (&us)[ROM_NSCHEDULES]) {
    const size_t vb = sizeof(float) * (size_t)ctx->kv * run.M, sb = sizeof(float) * (size_t)ctx->ks * run.M;
    const size_t mb = sizeof(double) * (size_t)run.M;
    void *V = nullptr, *S = nullptr, *mu = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rom_status rs = ROM_OK;
    hipError_t e = hipMalloc(&V, vb);
    if (e == hipSuccess) e = hipMalloc(&S, sb);
    if (e == hipSuccess && !run.mu) e = hipMalloc(&mu, mb);
    if (e == hipSuccess && mu) e = hipMemsetAsync(mu, 0, mb, st);   // any finite mu times the same
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) rs = hip_fail(e, "schedule tuning: setup");
    rom::Rank2Args a = run;
    a.V = V; a.S = S; a.c = nullptr; a.J = nullptr; a.y = nullptr; a.n0 = 0;
    if (mu) a.mu = static_cast<const double *>(mu);
    for (int sc = 0; sc < ROM_NSCHEDULES && rs == ROM_OK; ++sc) {
        if (!(cands >> sc & 1u)) continue;
        float best = 1e30f;
        for (int rep = 0; rep < 3 && rs == ROM_OK; ++rep) {   // rep 0: warm-up
            e = hipMemsetAsync(V, 0, vb, st);
            if (e == hipSuccess) e = hipMemsetAsync(S, 0, sb, st);
            if (e == hipSuccess && rep > 0) e = hipEventRecord(e0, st);
            if (e != hipSuccess) { rs = hip_fail(e, "schedule tuning"); break; }
            a.nsteps = rep == 0 ? 2 : nsteps;
            rs = launch_fp32_state_run(ctx, a, sc, G, st);
            if (rs != ROM_OK || rep == 0) continue;
            float ms = 0.f;
            e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { rs = hip_fail(e, "schedule tuning"); break; }
            best = std::min(best, ms * 1e3f / (float)nsteps);
        }
        if (rs == ROM_OK) us[sc] = best;
    }
    if (rs == ROM_OK) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) rs = hip_fail(e, "schedule tuning");
    }
    if (rs == ROM_OK && (cands >> ROM_SCHEDULE_ROWSPLIT & 1u)) {
        // a row-split run whose barrier timed out is not applicable here,
        // and its status must not be blamed on the caller's next run
        bool to = false;
        rs = take_timeout(ctx->status, to, "schedule tuning: status");
        if (rs == ROM_OK && to) us[ROM_SCHEDULE_ROWSPLIT] = -1.f;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    hfree(V);
    hfree(S);
    hfree(mu);
    return rs;
}

// Fastest timed schedule among `cands` (bit per rom_schedule); COLUMNS4 if
// none of them was timed.
int fastest(const float (&us)[ROM_NSCHEDULES], unsigned cands = ~0u) {
    int best = -1;
    for (int sc = 0; sc < ROM_NSCHEDULES; ++sc)
        if ((cands >> sc & 1u) && us[sc] >= 0.f && (best < 0 || us[sc] < us[best])) best = sc;
    return best < 0 ? ROM_SCHEDULE_COLUMNS4 : best;
}

// Schedule of an FP32-state rank-2 run (flags, table, or tuned now).
// A stream being captured into a graph gets a column-block schedule: the
// row-split path may allocate its workspace and synchronise, and its
// cooperative launch is not used inside graphs.
rom_status pick_schedule(rom_ctx *ctx, const rom::Rank2Args &a, hipStream_t st, int &sched, int &G) {
    const bool capturing = stream_capturing(st);
    G = capturing ? 0 : split_candidate(ctx, a.M);
    unsigned cands = 1u << ROM_SCHEDULE_COLUMNS4;
    if (G > 0) cands |= 1u << ROM_SCHEDULE_ROWSPLIT;
    if (cols8_ok(ctx)) cands |= 1u << ROM_SCHEDULE_COLUMNS8;
    if (ctx->res_pk) cands |= 1u << ROM_SCHEDULE_RESIDENT;
    if (panel_candidate(ctx, a.M, capturing)) cands |= 1u << ROM_SCHEDULE_PANEL;
    sched = ROM_SCHEDULE_COLUMNS4;
    if (ctx->flags & ROM_SCHED_COLUMNS) return ROM_OK;
    if (ctx->flags & ROM_SCHED_RESIDENT) {
        if (ctx->res_pk) sched = ROM_SCHEDULE_RESIDENT;
        return ROM_OK;
    }
    if (ctx->flags & ROM_SCHED_ROWSPLIT) {
        if (G > 0) sched = ROM_SCHEDULE_ROWSPLIT;
        return ROM_OK;
    }
    if (ctx->flags & ROM_SCHED_COLUMNS8) {
        if (cols8_ok(ctx)) sched = ROM_SCHEDULE_COLUMNS8;
        return ROM_OK;
    }
    const TuneKey key{ctx->kvp, ctx->ksp, rom::round_up(a.M, 64), (int)ctx->op_type};
    TuneEntry te;
    if (!tune_find(key, te)) {
        if (capturing) return ROM_OK;
        te.sched = ROM_SCHEDULE_COLUMNS4;
        for (float &u : te.us) u = -1.f;
        rom_status rs = time_schedules(ctx, a, cands, G, kTuneSteps, st, te.us);
        if (rs != ROM_OK) return rs;
        te.sched = fastest(te.us, cands);
        tune_store(key, te);
    }
    // the table's choice where it applies to this context (a shape's entry
    // is shared by skew and non-skew pairs), else the fastest that does
    sched = (cands >> te.sched & 1u) ? te.sched : fastest(te.us, cands);
    return ROM_OK;
}

// Per-workgroup step times of the 4- and 8-column tiles of a context's
// shape (grouped launch), from the table or tuned now on `st`.  Untimed
// entries stay negative.
rom_status tile_times(rom_ctx *c, hipStream_t st, TuneEntry &te) {
    const TuneKey key{c->kvp, c->ksp, 0, (int)ROM_F32};
    if (tune_find(key, te)) return ROM_OK;
    te.sched = ROM_SCHEDULE_COLUMNS4;
    for (float &u : te.us) u = -1.f;
    if (stream_capturing(st)) return ROM_OK;
    rom::Rank2Args a;
    a.b = c->b; a.mu = nullptr;
    a.kv = c->kv; a.ks = c->ks; a.kvp = c->kvp; a.ksp = c->ksp; a.dt = c->dt; a.source = ctx_source(c);
    a.M = rom::kColBlock;
    rom_status rs = time_schedules(c, a, 1u << ROM_SCHEDULE_COLUMNS4, 0, kTileSteps, st, te.us);
    if (rs == ROM_OK && cols8_ok(c)) {
        a.M = 2 * rom::kColBlock;
        rs = time_schedules(c, a, 1u << ROM_SCHEDULE_COLUMNS8, 0, kTileSteps, st, te.us);
    }
    if (rs != ROM_OK) return rs;
    // per-sample throughput decides the entry's tile
    te.sched = (te.us[ROM_SCHEDULE_COLUMNS8] >= 0.f &&
                te.us[ROM_SCHEDULE_COLUMNS8] < 2.f * te.us[ROM_SCHEDULE_COLUMNS4])
                   ? ROM_SCHEDULE_COLUMNS8 : ROM_SCHEDULE_COLUMNS4;
    tune_store(key, te);
    return ROM_OK;
}

}  // namespace

extern "C" {

const char *rom_last_error(void) { return g_err.c_str(); }

const char *rom_version(void) { return "rank2rom-mi355x 0.1 (gfx950)"; }

}  // extern "C"

namespace {

// Checks of a configuration shared by rom_create and affine instances.
rom_status check_config(const rom_config *cfg, const char *who) {
    const int kv = cfg->kv, ks = cfg->ks;
    std::string w(who);
    if (kv < 1 || ks < 1) return fail(ROM_E_ARG, w + ": kv and ks must be >= 1");
    if (kv > 65536 || ks > 65536) return fail(ROM_E_UNSUPPORTED, w + ": kv/ks above 65536");
    if (!(cfg->dt > 0.0) || !isfinite(cfg->dt)) return fail(ROM_E_ARG, w + ": dt must be finite and > 0");
    if (cfg->state_type != ROM_F64 && cfg->state_type != ROM_F32)
        return fail(ROM_E_ARG, w + ": state_type must be ROM_F64 or ROM_F32");
    if (cfg->op_type != ROM_F64 && cfg->op_type != ROM_F32 && cfg->op_type != ROM_BF16 &&
        cfg->op_type != ROM_F8E4M3)
        return fail(ROM_E_ARG, w + ": unknown op_type");
    const bool lowp = cfg->op_type == ROM_BF16 || cfg->op_type == ROM_F8E4M3;
    if (!lowp && cfg->op_type != cfg->state_type)
        return fail(ROM_E_UNSUPPORTED, w + ": supported (op, state) pairs are (F64, F64), "
                                          "(F32, F32), and (BF16 or F8E4M3, F32 or F64)");
    if (cfg->flags & ~(uint32_t)(ROM_SKEW_CHECK | ROM_SCHED_COLUMNS | ROM_SCHED_ROWSPLIT | ROM_SCHED_COLUMNS8 |
                                 ROM_SCHED_RESIDENT | ROM_SCHED_PANEL | ROM_SOURCE_GAUSS1 | ROM_STATE_BF16))
        return fail(ROM_E_ARG, w + ": unknown flag bits");
    if ((cfg->flags & ROM_STATE_BF16) && !(lowp && cfg->state_type == ROM_F32))
        return fail(ROM_E_ARG, w + ": ROM_STATE_BF16 needs BF16 or F8E4M3 operators with F32 states");
    const uint32_t sf =
        cfg->flags & (ROM_SCHED_COLUMNS | ROM_SCHED_ROWSPLIT | ROM_SCHED_COLUMNS8 | ROM_SCHED_RESIDENT | ROM_SCHED_PANEL);
    if (sf & (sf - 1)) return fail(ROM_E_ARG, w + ": at most one ROM_SCHED_* flag");
    return ROM_OK;
}

// Whether Asv == -Avs^T exactly (host arrays).
bool is_skew(const double *Avs, const double *Asv, int kv, int ks) {
    for (int i = 0; i < ks; ++i)
        for (int j = 0; j < kv; ++j)
            if (Asv[i + (size_t)j * ks] != -Avs[j + (size_t)i * kv]) return false;
    return true;
}

// Build a context from FP64 operators already in device memory: sA (Kv x
// Ks) and sB (Ks x Kv) column-major, sb the source padded to Kv_pad
// entries.  The device arrays stay the caller's; the call synchronises st.
rom_status build_ctx(const rom_config *cfg, bool skew, const double *sA, const double *sB, const double *sb,
                     hipStream_t st, const char *who, rom_ctx **out) {
    const int kv = cfg->kv, ks = cfg->ks;
    const size_t nA = (size_t)kv * ks;
    const bool lowp = cfg->op_type == ROM_BF16 || cfg->op_type == ROM_F8E4M3;
    std::string w(who);
    rom_ctx *c = new (std::nothrow) rom_ctx();
    if (!c) return fail(ROM_E_NOMEM, w + ": host allocation failed");
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) { free_ctx(c); return hip_fail(e, (w + ": hipGetDevice").c_str()); }
    if (!g_configured) {
        e = rom::rank2_f32_mfma_configure();
        if (e == hipSuccess) e = rom::rank2_valu_configure();
        if (e == hipSuccess) e = rom::rank2_lowp_configure();
        if (e == hipSuccess) e = rom::rank2_split_configure();
        if (e == hipSuccess) e = rom::receivers_configure();
        if (e != hipSuccess) { free_ctx(c); return hip_fail(e, (w + ": kernel attributes").c_str()); }
        g_configured = true;
    }
    c->kv = kv; c->ks = ks;
    c->kvp = rom::round_up(kv, 64); c->ksp = rom::round_up(ks, 64);
    c->dt = cfg->dt; c->op_type = cfg->op_type; c->state_type = cfg->state_type;
    c->flags = cfg->flags; c->skew = skew;
    const size_t ts = tsize(c->state_type);
#define CHK(call, what)                                                           \
    do {                                                                          \
        e = (call);                                                               \
        if (e != hipSuccess) { free_ctx(c);                                       \
            return e == hipErrorOutOfMemory ? fail(ROM_E_NOMEM, w + what) : hip_fail(e, (w + what).c_str()); } \
    } while (0)
    CHK(hipMalloc(&c->avs_cm, nA * ts), ": device allocation");
    CHK(hipMalloc(&c->asv_cm, nA * ts), ": device allocation");
    CHK(hipMalloc(&c->b, (size_t)c->kvp * ts), ": device allocation");
    CHK(hipMalloc(&c->status, sizeof(int) * 4), ": device allocation");
    CHK(hipMemsetAsync(c->status, 0, sizeof(int) * 4, st), ": memset");
    if (!(lowp && c->state_type == ROM_F64)) {
        CHK(rom::launch_convert(sA, c->avs_cm, nA, c->state_type, st), ": convert");
        CHK(rom::launch_convert(sB, c->asv_cm, nA, c->state_type, st), ": convert");
    }
    CHK(rom::launch_convert(sb, c->b, c->kvp, c->state_type, st), ": convert");
    if (lowp) {
        // BF16: round each operator (via FP32) to BF16; FP8: one scale
        // amax(|fp32(Avs)|, |fp32(Asv)|) / 448 for both operators, so a skew
        // pair stays exactly skew after quantisation.
        const size_t eb = c->op_type == ROM_BF16 ? 2 : 1;
        unsigned *amax = reinterpret_cast<unsigned *>(c->status);
        CHK(hipMalloc(&c->avs_lp, eb * (size_t)c->kvp * c->ksp), ": device allocation");
        CHK(hipMalloc(&c->asv_lp, eb * (size_t)c->kvp * c->ksp), ": device allocation");
        if (c->op_type == ROM_F8E4M3) {
            CHK(rom::launch_amax(sA, (int64_t)nA, amax, st), ": amax");
            CHK(rom::launch_amax(sB, (int64_t)nA, amax, st), ": amax");
        }
        CHK(rom::launch_pack_lowp(sA, kv, ks, c->kvp, c->ksp, c->op_type, amax, c->avs_lp, st), ": pack");
        CHK(rom::launch_pack_lowp(sB, ks, kv, c->ksp, c->kvp, c->op_type, amax, c->asv_lp, st), ": pack");
        if (c->op_type == ROM_F8E4M3) {
            unsigned bits = 0;
            CHK(hipMemcpyAsync(&bits, amax, sizeof(bits), hipMemcpyDeviceToHost, st), ": readback");
            CHK(hipStreamSynchronize(st), ": synchronize");
            float am;
            memcpy(&am, &bits, sizeof(am));
            c->op_scale = am > 0.f ? am / 448.0f : 1.0f;
            CHK(hipMemsetAsync(c->status, 0, sizeof(int) * 4, st), ": memset");
        }
        if (c->state_type == ROM_F64) {
            // FP64 states with rounded operators (the long-horizon reference of
            // the rounded model): the FP64 path runs on the dequantised values
            CHK(rom::launch_unpack_lowp(c->avs_lp, kv, ks, c->kvp, c->ksp, c->op_type, (double)c->op_scale,
                                        static_cast<double *>(c->avs_cm), st), ": unpack");
            CHK(rom::launch_unpack_lowp(c->asv_lp, ks, kv, c->ksp, c->kvp, c->op_type, (double)c->op_scale,
                                        static_cast<double *>(c->asv_cm), st), ": unpack");
        }
    } else if (c->state_type == ROM_F32) {
        CHK(hipMalloc(&c->avs_pk, sizeof(float) * (size_t)c->kvp * c->ksp), ": device allocation");
        CHK(hipMalloc(&c->asv_pk, sizeof(float) * (size_t)c->kvp * c->ksp), ": device allocation");
        CHK(rom::launch_pack_f32(sA, kv, ks, c->kvp, c->ksp, c->avs_pk, st), ": pack");
        CHK(rom::launch_pack_f32(sB, ks, kv, c->ksp, c->kvp, c->asv_pk, st), ": pack");
        if (skew && rom::rank2_resident_applies(c->kvp, c->ksp)) {
            CHK(hipMalloc(&c->res_pk, rom::rank2_resident_pack_bytes(c->kvp, c->ksp)), ": device allocation");
            CHK(rom::launch_resident_pack(static_cast<const float *>(c->avs_cm), kv, ks, c->kvp, c->ksp, c->res_pk,
                                          st), ": pack");
        }
    }
    if (c->state_type == ROM_F32 && split_candidate(c, 1) > 0) {
        // row-split operator packs up front (the allocation-free run needs
        // them), and this device's static row-split scratch looked up once
        // while the device is current (a failure is reported by the run that
        // needs it)
        rom_status rs = prepare_split_pack(c, st);
        if (rs != ROM_OK) { free_ctx(c); return rs; }
        void *scr = nullptr;
        (void)rom::rank2_split_static_scratch(c->device, &scr);
    }
    CHK(hipStreamSynchronize(st), ": synchronize");
#undef CHK
    *out = c;
    return ROM_OK;
}

}  // namespace

extern "C" {

rom_status rom_create(const rom_config *cfg, const double *Avs, const double *Asv,
                      const double *b, void *stream, rom_ctx **out) {
    if (out) *out = nullptr;
    if (!cfg || !Avs || !Asv || !b || !out) return fail(ROM_E_ARG, "rom_create: NULL argument");
    rom_status rs = check_config(cfg, "rom_create");
    if (rs != ROM_OK) return rs;
    const int kv = cfg->kv, ks = cfg->ks;
    const size_t nA = (size_t)kv * ks;
    if (!all_finite(Avs, nA) || !all_finite(Asv, nA) || !all_finite(b, kv))
        return fail(ROM_E_NONFINITE, "rom_create: non-finite value in Avs, Asv or b");
    const bool skew = is_skew(Avs, Asv, kv, ks);
    if ((cfg->flags & ROM_SKEW_CHECK) && skew) {
        double smax = sigma_max(Avs, kv, ks);
        if (cfg->dt * smax * (1.0 + 1e-9) >= 2.0)
            return fail(ROM_E_UNSTABLE, "rom_create: dt * sigma_max(Avs) >= 2 for a skew pair "
                                        "(leapfrog energy not positive)");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t kvp = (size_t)rom::round_up(kv, 64);
    double *stage = nullptr;
    hipError_t e = hipMalloc(&stage, (2 * nA + kvp) * sizeof(double));
    if (e != hipSuccess) return fail(ROM_E_NOMEM, "rom_create: device allocation failed");
    double *sA = stage, *sB = stage + nA, *sb = stage + 2 * nA;
    std::vector<double> bpad(kvp, 0.0);
    memcpy(bpad.data(), b, sizeof(double) * kv);
    e = hipMemcpyAsync(sA, Avs, nA * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sB, Asv, nA * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sb, bpad.data(), kvp * sizeof(double), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) { hfree(stage); return hip_fail(e, "rom_create: upload"); }
    rs = build_ctx(cfg, skew, sA, sB, sb, st, "rom_create", out);
    (void)hipStreamSynchronize(st);   // the staging buffer is read until here
    hfree(stage);
    return rs;
}

rom_status rom_get_operators(rom_ctx *ctx, double *Avs, double *Asv, double *scale) {
    if (!ctx || !Avs || !Asv) return fail(ROM_E_ARG, "rom_get_operators: NULL argument");
    const size_t nA = (size_t)ctx->kv * ctx->ks;
    double *d = nullptr;
    hipError_t e = hipMalloc(&d, 2 * nA * sizeof(double));
    if (e != hipSuccess) return fail(ROM_E_NOMEM, "rom_get_operators: device allocation failed");
    if (ctx->op_type == ROM_BF16 || ctx->op_type == ROM_F8E4M3) {
        e = rom::launch_unpack_lowp(ctx->avs_lp, ctx->kv, ctx->ks, ctx->kvp, ctx->ksp, ctx->op_type,
                                    (double)ctx->op_scale, d, nullptr);
        if (e == hipSuccess)
            e = rom::launch_unpack_lowp(ctx->asv_lp, ctx->ks, ctx->kv, ctx->ksp, ctx->kvp, ctx->op_type,
                                        (double)ctx->op_scale, d + nA, nullptr);
    } else if (ctx->state_type == ROM_F32) {
        e = rom::launch_convert_f32_to_f64(static_cast<const float *>(ctx->avs_cm), d, (int64_t)nA, nullptr);
        if (e == hipSuccess)
            e = rom::launch_convert_f32_to_f64(static_cast<const float *>(ctx->asv_cm), d + nA, (int64_t)nA, nullptr);
    } else {
        e = hipMemcpy(d, ctx->avs_cm, nA * sizeof(double), hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(d + nA, ctx->asv_cm, nA * sizeof(double), hipMemcpyDeviceToDevice);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(Avs, d, nA * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(Asv, d + nA, nA * sizeof(double), hipMemcpyDeviceToHost);
    hfree(d);
    if (e != hipSuccess) return hip_fail(e, "rom_get_operators");
    if (scale) *scale = ctx->op_type == ROM_F8E4M3 ? (double)ctx->op_scale : 1.0;
    return ROM_OK;
}

rom_status rom_energy(rom_ctx *ctx, int32_t M, const void *V, const void *S, double *E, void *stream) {
    if (!ctx || !V || !S || !E) return fail(ROM_E_ARG, "rom_energy: NULL argument");
    if (M < 1) return fail(ROM_E_ARG, "rom_energy: M must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (!ctx->avs_e64) {
        const size_t nA = (size_t)ctx->kv * ctx->ks;
        e = hipMalloc(&ctx->avs_e64, nA * sizeof(double));
        if (e != hipSuccess) { ctx->avs_e64 = nullptr; return fail(ROM_E_NOMEM, "rom_energy: allocation failed"); }
        if ((ctx->op_type == ROM_BF16 || ctx->op_type == ROM_F8E4M3))
            e = rom::launch_unpack_lowp(ctx->avs_lp, ctx->kv, ctx->ks, ctx->kvp, ctx->ksp, ctx->op_type,
                                        (double)ctx->op_scale, ctx->avs_e64, st);
        else if (ctx->state_type == ROM_F32)
            e = rom::launch_convert_f32_to_f64(static_cast<const float *>(ctx->avs_cm), ctx->avs_e64, (int64_t)nA, st);
        else
            e = hipMemcpyAsync(ctx->avs_e64, ctx->avs_cm, nA * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "rom_energy: prepare");
    }
    e = rom::launch_energy(ctx->avs_e64, ctx->kv, ctx->ks, ctx->dt, ctx->state_type, V, S, M, E, st);
    if (e != hipSuccess) return hip_fail(e, "rom_energy: launch");
    return ROM_OK;
}

rom_status rom_affine_create(const rom_config *cfg, int32_t Q, const double *Avs_q, const double *Asv_q,
                             const double *b, void *stream, rom_affine **out) {
    if (out) *out = nullptr;
    if (!cfg || !Avs_q || !Asv_q || !b || !out) return fail(ROM_E_ARG, "rom_affine_create: NULL argument");
    if (Q < 1 || Q > rom::kMaxAffine) return fail(ROM_E_ARG, "rom_affine_create: Q must be in [1, 16]");
    rom_status rs = check_config(cfg, "rom_affine_create");
    if (rs != ROM_OK) return rs;
    const int kv = cfg->kv, ks = cfg->ks;
    const size_t nA = (size_t)kv * ks;
    if (!all_finite(Avs_q, nA * Q) || !all_finite(Asv_q, nA * Q) || !all_finite(b, kv))
        return fail(ROM_E_NONFINITE, "rom_affine_create: non-finite value in the terms or b");
    bool skew = true;
    for (int q = 0; q < Q && skew; ++q) skew = is_skew(Avs_q + q * nA, Asv_q + q * nA, kv, ks);
    rom_affine *A = new (std::nothrow) rom_affine();
    if (!A) return fail(ROM_E_NOMEM, "rom_affine_create: host allocation failed");
    A->cfg = *cfg;
    A->Q = Q;
    A->skew = skew;
    if ((cfg->flags & ROM_SKEW_CHECK) && skew) A->host_avs.assign(Avs_q, Avs_q + nA * Q);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t kvp = (size_t)rom::round_up(kv, 64);
    std::vector<double> bp(kvp, 0.0);
    memcpy(bp.data(), b, sizeof(double) * kv);
    hipError_t e = hipMalloc(&A->terms, 2 * nA * Q * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&A->bpad, kvp * sizeof(double));
    if (e != hipSuccess) {
        hfree(A->terms); hfree(A->bpad); delete A;
        return fail(ROM_E_NOMEM, "rom_affine_create: device allocation failed");
    }
    e = hipMemcpyAsync(A->terms, Avs_q, nA * Q * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(A->terms + nA * Q, Asv_q, nA * Q * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(A->bpad, bp.data(), kvp * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        hfree(A->terms); hfree(A->bpad); delete A;
        return hip_fail(e, "rom_affine_create: upload");
    }
    *out = A;
    return ROM_OK;
}

rom_status rom_affine_instance(rom_affine *A, const double *theta, double dt, void *stream, rom_ctx **out) {
    if (out) *out = nullptr;
    if (!A || !theta || !out) return fail(ROM_E_ARG, "rom_affine_instance: NULL argument");
    if (!all_finite(theta, A->Q)) return fail(ROM_E_NONFINITE, "rom_affine_instance: non-finite coefficient");
    if (dt < 0.0 || !isfinite(dt)) return fail(ROM_E_ARG, "rom_affine_instance: dt must be finite and >= 0");
    rom_config cfg = A->cfg;
    if (dt > 0.0) cfg.dt = dt;
    const int kv = cfg.kv, ks = cfg.ks;
    const size_t nA = (size_t)kv * ks;
    if ((cfg.flags & ROM_SKEW_CHECK) && A->skew) {
        // the same sum, in the same order, on the host
        std::vector<double> Avs(nA);
        for (size_t i = 0; i < nA; ++i) {
            double acc = theta[0] * A->host_avs[i];
            for (int q = 1; q < A->Q; ++q) acc = acc + theta[q] * A->host_avs[(size_t)q * nA + i];
            Avs[i] = acc;
        }
        if (cfg.dt * sigma_max(Avs.data(), kv, ks) * (1.0 + 1e-9) >= 2.0)
            return fail(ROM_E_UNSTABLE, "rom_affine_instance: dt * sigma_max(Avs) >= 2 for a skew pair "
                                        "(leapfrog energy not positive)");
    }
    rom::AffineCoeffs th{};
    for (int q = 0; q < A->Q; ++q) th.c[q] = theta[q];
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *stage = nullptr;
    hipError_t e = hipMalloc(&stage, 2 * nA * sizeof(double));
    if (e != hipSuccess) return fail(ROM_E_NOMEM, "rom_affine_instance: device allocation failed");
    e = rom::launch_affine_combine(A->terms, A->Q, (int64_t)nA, th, stage, st);
    if (e == hipSuccess) e = rom::launch_affine_combine(A->terms + nA * A->Q, A->Q, (int64_t)nA, th, stage + nA, st);
    if (e != hipSuccess) { hfree(stage); return hip_fail(e, "rom_affine_instance: assemble"); }
    rom_status rs = build_ctx(&cfg, A->skew, stage, stage + nA, A->bpad, st, "rom_affine_instance", out);
    (void)hipStreamSynchronize(st);
    hfree(stage);
    return rs;
}

rom_status rom_affine_destroy(rom_affine *A) {
    if (!A) return ROM_OK;
    hfree(A->terms);
    hfree(A->bpad);
    delete A;
    return ROM_OK;
}

rom_status rom_destroy(rom_ctx *ctx) {
    if (!ctx) return ROM_OK;
    free_ctx(ctx);
    return ROM_OK;
}

rom_status rom_debug_force_timeout(int32_t on) {
    rom::g_forced_timeout = on != 0;
    return ROM_OK;
}

int32_t rom_last_schedule(rom_ctx *ctx) { return ctx ? ctx->last_schedule : -1; }

rom_status rom_schedule_times(rom_ctx *ctx, int32_t M, double us[ROM_NSCHEDULES]) {
    if (!ctx || M < 1 || !us) return fail(ROM_E_ARG, "rom_schedule_times: bad argument");
    TuneEntry te;
    if (!tune_find(TuneKey{ctx->kvp, ctx->ksp, rom::round_up(M, 64), (int)ctx->op_type}, te))
        return fail(ROM_E_ARG, "rom_schedule_times: this shape is not in the tuning table");
    for (int sc = 0; sc < ROM_NSCHEDULES; ++sc) us[sc] = te.us[sc];
    return ROM_OK;
}

int32_t rom_tune_count(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return (int32_t)g_tune.size();
}

rom_status rom_tune_get(int32_t i, rom_tune_entry *out) {
    if (!out) return fail(ROM_E_ARG, "rom_tune_get: NULL out");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (i < 0 || i >= (int32_t)g_tune.size()) return fail(ROM_E_ARG, "rom_tune_get: index out of range");
    auto it = g_tune.begin();
    std::advance(it, i);
    out->kv_pad = it->first.kvp;
    out->ks_pad = it->first.ksp;
    out->m_pad = it->first.mpad;
    out->op_type = (rom_dtype)it->first.op;
    out->schedule = it->second.sched;
    for (int sc = 0; sc < ROM_NSCHEDULES; ++sc) out->us[sc] = it->second.us[sc];
    return ROM_OK;
}

rom_status rom_tune_put(const rom_tune_entry *e) {
    if (!e) return fail(ROM_E_ARG, "rom_tune_put: NULL entry");
    if (e->kv_pad < 64 || e->ks_pad < 64 || e->kv_pad % 64 || e->ks_pad % 64 || e->m_pad < 0 || e->m_pad % 64)
        return fail(ROM_E_ARG, "rom_tune_put: sizes must be positive multiples of 64 (m_pad may be 0)");
    if (e->op_type < ROM_F64 || e->op_type > ROM_F8E4M3)
        return fail(ROM_E_ARG, "rom_tune_put: bad op_type");
    if (e->schedule < 0 || e->schedule >= ROM_NSCHEDULES)
        return fail(ROM_E_ARG, "rom_tune_put: bad schedule");
    if (e->m_pad == 0 && e->schedule != ROM_SCHEDULE_COLUMNS4 && e->schedule != ROM_SCHEDULE_COLUMNS8)
        return fail(ROM_E_ARG, "rom_tune_put: a grouped tile entry names a column tile");
    TuneEntry te;
    te.sched = e->schedule;
    for (int sc = 0; sc < ROM_NSCHEDULES; ++sc) te.us[sc] = (float)e->us[sc];
    tune_store(TuneKey{e->kv_pad, e->ks_pad, e->m_pad, (int)e->op_type}, te);
    return ROM_OK;
}

void rom_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

rom_status rom_check(rom_ctx *ctx, void *stream) {
    if (!ctx) return fail(ROM_E_ARG, "rom_check: NULL context");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "rom_check: synchronize");
    bool to = false;
    rom_status rs = take_timeout(ctx->status, to, "rom_check: status");
    if (rs != ROM_OK) return rs;
    if (to) return fail(ROM_E_TIMEOUT, "rom_check: a row-split group barrier timed out; the run's results are invalid");
    return ROM_OK;
}

rom_status rom_check_finite(rom_ctx *ctx, int32_t M, const void *V, const void *S, void *stream) {
    if (!ctx || !V || !S) return fail(ROM_E_ARG, "rom_check_finite: NULL argument");
    if (M < 1) return fail(ROM_E_ARG, "rom_check_finite: M must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool f64 = ctx->state_type == ROM_F64;
    int *flag = ctx->status + 3;
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), st);
    if (e == hipSuccess) e = rom::launch_nonfinite(V, (int64_t)ctx->kv * M, f64, flag, st);
    if (e == hipSuccess) e = rom::launch_nonfinite(S, (int64_t)ctx->ks * M, f64, flag, st);
    int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "rom_check_finite");
    if (h) return fail(ROM_E_NONFINITE, "rom_check_finite: the states hold NaN or infinite values");
    return ROM_OK;
}

rom_status rom_step_rank1(rom_ctx *ctx, void *v, void *s, int64_t n, double mu, void *stream) {
    if (!ctx || !v || !s) return fail(ROM_E_ARG, "rom_step_rank1: NULL argument");
    if (n < 0) return fail(ROM_E_ARG, "rom_step_rank1: n must be >= 0");
    if (!isfinite(mu)) return fail(ROM_E_NONFINITE, "rom_step_rank1: mu not finite");
    if (ctx->op_type != ctx->state_type)
        return fail(ROM_E_UNSUPPORTED, "rom_step_rank1: needs op_type == state_type");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = ctx->state_type == ROM_F64
        ? rom::launch_rank1_step<double>(ctx->avs_cm, ctx->asv_cm, ctx->b, ctx->kv, ctx->ks, ctx->dt, n, mu,
                                         ctx_source(ctx), v, s, st)
        : rom::launch_rank1_step<float>(ctx->avs_cm, ctx->asv_cm, ctx->b, ctx->kv, ctx->ks, ctx->dt, n, mu,
                                        ctx_source(ctx), v, s, st);
    if (e != hipSuccess) return hip_fail(e, "rom_step_rank1: launch");
    return ROM_OK;
}

rom_status rom_run_rank1(rom_ctx *ctx, void *v, void *s, double mu, int64_t n0, int64_t nsteps,
                         void *stream) {
    if (!ctx || !v || !s) return fail(ROM_E_ARG, "rom_run_rank1: NULL argument");
    if (n0 < 0 || nsteps < 0) return fail(ROM_E_ARG, "rom_run_rank1: n0 and nsteps must be >= 0");
    if (!isfinite(mu)) return fail(ROM_E_NONFINITE, "rom_run_rank1: mu not finite");
    for (int64_t k = 0; k < nsteps; ++k) {
        rom_status r = rom_step_rank1(ctx, v, s, n0 + k, mu, stream);
        if (r != ROM_OK) return r;
    }
    return ROM_OK;
}

rom_status rom_run_rank1_batch(rom_ctx *ctx, int32_t M, const double *mu, int64_t n0, int64_t nsteps, void *V,
                               void *S, void *stream) {
    if (!ctx) return fail(ROM_E_ARG, "rom_run_rank1_batch: NULL context");
    if (M < 1) return fail(ROM_E_ARG, "rom_run_rank1_batch: M must be >= 1");
    if (!mu || !V || !S) return fail(ROM_E_ARG, "rom_run_rank1_batch: NULL mu, V or S");
    if (n0 < 0 || nsteps < 0) return fail(ROM_E_ARG, "rom_run_rank1_batch: n0 and nsteps must be >= 0");
    if (ctx->state_type != ROM_F32 || ctx->op_type != ROM_F32)
        return fail(ROM_E_UNSUPPORTED, "rom_run_rank1_batch: FP32 states and operators only");
    if (ctx->kv > 1024 || ctx->ks > 1024) return fail(ROM_E_UNSUPPORTED, "rom_run_rank1_batch: Kv, Ks <= 1024");
    if (nsteps == 0) return ROM_OK;
    rom::Rank2Args a;
    a.avs = ctx->avs_cm; a.asv = ctx->asv_cm; a.b = ctx->b; a.mu = mu; a.V = V; a.S = S;
    a.kv = ctx->kv; a.ks = ctx->ks; a.kvp = ctx->kvp; a.ksp = ctx->ksp; a.M = M;
    a.n0 = n0; a.nsteps = nsteps; a.dt = ctx->dt; a.source = ctx_source(ctx);
    hipError_t e = rom::launch_rank1_batch(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "rom_run_rank1_batch: launch");
    return ROM_OK;
}

rom_status rom_run_rank2(rom_ctx *ctx, int32_t M, const double *mu, int64_t n0, int64_t nsteps,
                         void *V, void *S, const void *c, double *J, double *y, void *stream) {
    if (!ctx) return fail(ROM_E_ARG, "rom_run_rank2: NULL context");
    if (M < 1) return fail(ROM_E_ARG, "rom_run_rank2: M must be >= 1");
    if (!mu || !V || !S) return fail(ROM_E_ARG, "rom_run_rank2: NULL mu, V or S");
    if (n0 < 0 || nsteps < 0) return fail(ROM_E_ARG, "rom_run_rank2: n0 and nsteps must be >= 0");
    if ((J || y) && !c) return fail(ROM_E_ARG, "rom_run_rank2: J and y require the probe c");
    if (nsteps == 0) return ROM_OK;
    rom::Rank2Args a;
    a.b = ctx->b; a.c = c; a.mu = mu; a.V = V; a.S = S; a.J = J; a.y = y;
    a.kv = ctx->kv; a.ks = ctx->ks; a.kvp = ctx->kvp; a.ksp = ctx->ksp; a.M = M;
    a.n0 = n0; a.nsteps = nsteps; a.dt = ctx->dt; a.source = ctx_source(ctx);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((ctx->op_type == ROM_BF16 || ctx->op_type == ROM_F8E4M3 || ctx->op_type == ROM_F32) &&
        ctx->state_type == ROM_F32) {
        const bool lowp = ctx->op_type != ROM_F32;
        if (lowp && rom::rank2_lowp_lds_bytes(ctx->kvp, ctx->ksp) > 160 * 1024)
            return fail(ROM_E_UNSUPPORTED, "rom_run_rank2: Kv + Ks above the LDS-resident limit");
        // FP32 operators: the panel schedule where the column blocks' states
        // do not fit in LDS, or where the context pins it
        if (!lowp && ((ctx->flags & ROM_SCHED_PANEL) || ctx->kvp + ctx->ksp > rom::kMaxPadSum ||
                      rom::rank2_f32_mfma_lds_bytes(ctx->kvp, ctx->ksp, 1) > 160 * 1024))
            return run_panel(ctx, a, st);
        int sched = ROM_SCHEDULE_COLUMNS4, G = 0;
        rom_status rs = pick_schedule(ctx, a, st, sched, G);
        if (rs != ROM_OK) return rs;
        ctx->last_schedule = sched;
        return launch_fp32_state_run(ctx, a, sched, G, st);
    } else {
        // FP64 states: the vector-ALU column blocks (pinned by
        // ROM_SCHED_COLUMNS), else the panel schedule on the FP64 matrix
        // cores where pinned, from Kv_pad + Ks_pad >= kPanelF64From, or where
        // the column blocks' states do not fit in LDS (any size)
        const bool fits = rom::rank2_valu_lds_bytes(ctx->state_type, ctx->kv, ctx->ks, ctx->kvp, ctx->ksp) <= 150 * 1024;
        // a stream being captured cannot allocate the panel workspace: an
        // unpinned run that fits the column blocks stays on them until an
        // uncaptured panel run has set the workspace up
        const bool panel_ready = ctx->avs_rm && ctx->pn_ws_bytes >= rom::panel_ws_bytes(ctx->kv, ctx->ks, M, true);
        const bool auto_panel = !(ctx->flags & ROM_SCHED_COLUMNS) && ctx->kvp + ctx->ksp >= rom::kPanelF64From &&
                                (panel_ready || !stream_capturing(st));
        if (!fits || (ctx->flags & ROM_SCHED_PANEL) || auto_panel)
            return run_panel(ctx, a, st);
        a.avs = ctx->avs_cm; a.asv = ctx->asv_cm;
        // small K (skew pairs: Kv_pad, Ks_pad <= 128; others: Kv_pad Ks_pad
        // <= 8192): the operator-resident kernel unless the context pins
        // the column blocks
        if (!(ctx->flags & ROM_SCHED_COLUMNS) && rom::rank2_resident64_applies(ctx->kvp, ctx->ksp, ctx->skew)) {
            e = rom::launch_rank2_resident64(a, ctx->skew, st);
            ctx->last_schedule = ROM_SCHEDULE_RESIDENT;
        } else {
            e = rom::launch_rank2_valu<double>(a, st);
            ctx->last_schedule = -1;
        }
    }
    if (e != hipSuccess) return hip_fail(e, "rom_run_rank2: launch");
    return ROM_OK;
}

rom_status rom_run_rank2_noalloc(rom_ctx *ctx, int32_t M, const double *mu, int64_t n0, int64_t nsteps,
                                 void *V, void *S, const void *c, double *J, double *y, void *stream) {
    if (!ctx) return fail(ROM_E_ARG, "rom_run_rank2_noalloc: NULL context");
    if (M < 1) return fail(ROM_E_ARG, "rom_run_rank2_noalloc: M must be >= 1");
    if (!mu || !V || !S) return fail(ROM_E_ARG, "rom_run_rank2_noalloc: NULL mu, V or S");
    if (n0 < 0 || nsteps < 0) return fail(ROM_E_ARG, "rom_run_rank2_noalloc: n0 and nsteps must be >= 0");
    if ((J || y) && !c) return fail(ROM_E_ARG, "rom_run_rank2_noalloc: J and y require the probe c");
    if (ctx->state_type != ROM_F32 || ctx->op_type == ROM_F64)
        return fail(ROM_E_UNSUPPORTED, "rom_run_rank2_noalloc: FP32 states with F32, BF16 or F8E4M3 operators only");
    const int G = split_candidate(ctx, M);
    if (G == 0 || !ctx->avs_sp)
        return fail(ROM_E_UNSUPPORTED, "rom_run_rank2_noalloc: the row-split schedule does not apply (Kv == Ks, "
                                       "padded K a multiple of 64 in [128, 2048] (F32) or of 128 in [128, 1024] "
                                       "(BF16, FP8), ceil(M/64) <= 8 floor(32 / (K/64)), a 256-CU gfx950)");
    const size_t need = rom::rank2_split_workspace_bytes(ctx->kvp, G);
    if (need > rom::rank2_split_static_bytes())
        return fail(ROM_E_UNSUPPORTED, "rom_run_rank2_noalloc: needs " + std::to_string(need) +
                                           " bytes of scratch, above the static " +
                                           std::to_string(rom::rank2_split_static_bytes()));
    if (nsteps == 0) return ROM_OK;
    void *scr = nullptr;
    hipError_t e = rom::rank2_split_static_scratch(ctx->device, &scr);
    if (e != hipSuccess) return hip_fail(e, "rom_run_rank2_noalloc: static scratch");
    rom::Rank2Args a;
    a.b = ctx->b; a.c = c; a.mu = mu; a.V = V; a.S = S; a.J = J; a.y = y;
    a.kv = ctx->kv; a.ks = ctx->ks; a.kvp = ctx->kvp; a.ksp = ctx->ksp; a.M = M;
    a.n0 = n0; a.nsteps = nsteps; a.dt = ctx->dt; a.source = ctx_source(ctx);
    const bool lowp = ctx->op_type != ROM_F32;
    a.single = (lowp && (ctx->flags & ROM_STATE_BF16)) ? 1 : 0;
    e = rom::launch_rank2_split(ctx->avs_sp, ctx->asv_sp, a, lowp ? ctx->op_scale : 1.0f, scr, G, ctx->status,
                                !lowp, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "rom_run_rank2_noalloc: launch");
    ctx->last_schedule = ROM_SCHEDULE_ROWSPLIT;
    return ROM_OK;
}

rom_status rom_adjoint(rom_ctx *ctx, int32_t M, const double *mu, int64_t nsteps, const void *c,
                       const void *V0, const void *S0, double *J, void *dAvs, void *dAsv,
                       double *dmu, int32_t ckpt_stride, void *stream) {
    if (!ctx) return fail(ROM_E_ARG, "rom_adjoint: NULL context");
    if (M < 1) return fail(ROM_E_ARG, "rom_adjoint: M must be >= 1");
    if (!mu || !c || !J) return fail(ROM_E_ARG, "rom_adjoint: mu, c and J are required");
    if (nsteps < 1) return fail(ROM_E_ARG, "rom_adjoint: nsteps must be >= 1");
    if (ckpt_stride < -1) return fail(ROM_E_ARG, "rom_adjoint: ckpt_stride must be >= -1");
    if (ctx->state_type != ROM_F32 || ctx->op_type != ROM_F32)
        return fail(ROM_E_UNSUPPORTED, "rom_adjoint: FP32 states and operators only in this version");
    if (ctx->kvp + ctx->ksp > rom::kMaxPadSum ||
        rom::rank2_f32_mfma_lds_bytes(ctx->kvp, ctx->ksp, 1) > 160 * 1024)
        return fail(ROM_E_UNSUPPORTED, "rom_adjoint: Kv + Ks above the LDS-resident limit");
    // ckpt_stride -1: no checkpoints, the states are recovered by stepping
    // the leapfrog backwards from the final state (segments of sqrt(N) steps)
    const bool rev = ckpt_stride == -1;
    int64_t C = ckpt_stride > 0 ? ckpt_stride : (int64_t)ceil(sqrt((double)nsteps));
    if (C < 1) C = 1;
    if (C > nsteps) C = nsteps;
    const int64_t nseg = (nsteps + C - 1) / C;
    const int kv = ctx->kv, ks = ctx->ks;
    const size_t mK = (size_t)M, v1 = (size_t)kv * mK, s1 = (size_t)ks * mK;
    // workspace layout (floats, then doubles)
    // The recompute of segment g - 1 (side stream 0), the reverse sweep of
    // segment g (the caller's stream) and the gradient products of segment
    // g + 1 (side stream 1) run at the same time: the state and probe traces
    // of a segment live in one of kTr buffer sets, its W and Q traces in one
    // of kWq, each reused only after the products of its previous segment.
    constexpr int kTr = 3, kWq = 2;
    const size_t n_ck = rev ? 0 : (size_t)nseg * (v1 + s1);
    const size_t n_vtr = (size_t)(C + 1) * v1, n_str = (size_t)(C + 1) * s1;
    const size_t n_wtr = (size_t)C * v1, n_qtr = (size_t)C * s1;
    const size_t n_cur = v1 + s1, n_pq = v1 + s1;
    size_t nf = n_ck + kTr * (n_vtr + n_str) + kWq * (n_wtr + n_qtr) + n_cur + n_pq;
    nf = (nf + 3) / 4 * 4;
    const size_t n_ytr = (size_t)C * mK, n_da = 2 * (size_t)kv * ks;
    const int nsplit = std::max(rom::gemm_nt_splits(kv, ks), rom::gemm_nt_splits(ks, kv));
    const size_t n_part = (size_t)nsplit * kv * ks;   // gradient-product partials
    const size_t bytes = nf * sizeof(float) + (kTr * n_ytr + n_da + n_part) * sizeof(double);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (!ctx->side[0]) {
        e = hipSuccess;
        for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking);
        for (int i = 0; i < 13 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ctx->ev[i], hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "rom_adjoint: stream / event creation");
    }
    if (!ctx->asvT_pk) {
        size_t pk = sizeof(float) * (size_t)ctx->kvp * ctx->ksp;
        e = hipMalloc(&ctx->asvT_pk, pk);
        if (e == hipSuccess) e = hipMalloc(&ctx->avsT_pk, pk);
        if (e != hipSuccess) {
            hfree(ctx->asvT_pk); hfree(ctx->avsT_pk);
            ctx->asvT_pk = ctx->avsT_pk = nullptr;
            return fail(ROM_E_NOMEM, "rom_adjoint: device allocation failed");
        }
        // Asv^T is Kv x Ks (rows kvp, reduction ksp); Avs^T is Ks x Kv
        e = rom::launch_pack_f32_from_f32((const float *)ctx->asv_cm, ks, kv, true, ctx->kvp,
                                          ctx->ksp, ctx->asvT_pk, st);
        if (e == hipSuccess)
            e = rom::launch_pack_f32_from_f32((const float *)ctx->avs_cm, kv, ks, true, ctx->ksp,
                                              ctx->kvp, ctx->avsT_pk, st);
        if (e != hipSuccess) return hip_fail(e, "rom_adjoint: pack");
    }
    if (ctx->ws_bytes < bytes) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "rom_adjoint: synchronize");
        hfree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
        e = hipMalloc(&ctx->ws, bytes);
        if (e != hipSuccess) { ctx->ws = nullptr; return fail(ROM_E_NOMEM, "rom_adjoint: workspace allocation failed"); }
        ctx->ws_bytes = bytes;
    }
    float *f = static_cast<float *>(ctx->ws);
    float *ck = f;
    float *vtrb[kTr], *strb[kTr], *wtrb[kWq], *qtrb[kWq];
    float *fp = ck + n_ck;
    for (int i = 0; i < kTr; ++i) { vtrb[i] = fp; strb[i] = fp + n_vtr; fp += n_vtr + n_str; }
    for (int i = 0; i < kWq; ++i) { wtrb[i] = fp; qtrb[i] = fp + n_wtr; fp += n_wtr + n_qtr; }
    float *curV = fp, *curS = curV + v1, *P = curS + s1, *Q = P + v1;
    double *ytrb[kTr];
    for (int i = 0; i < kTr; ++i) ytrb[i] = reinterpret_cast<double *>(f + nf) + i * n_ytr;
    double *dA64 = ytrb[kTr - 1] + n_ytr;
    double *dAvs64 = dA64, *dAsv64 = dA64 + (size_t)kv * ks;
    double *part = dA64 + n_da;

#define ACHK(call, what) do { e = (call); if (e != hipSuccess) return hip_fail(e, what); } while (0)
    // forward sweep: checkpoint before every segment, accumulate J
    if (V0) ACHK(hipMemcpyAsync(curV, V0, v1 * 4, hipMemcpyDeviceToDevice, st), "rom_adjoint: copy");
    else ACHK(hipMemsetAsync(curV, 0, v1 * 4, st), "rom_adjoint: memset");
    if (S0) ACHK(hipMemcpyAsync(curS, S0, s1 * 4, hipMemcpyDeviceToDevice, st), "rom_adjoint: copy");
    else ACHK(hipMemsetAsync(curS, 0, s1 * 4, st), "rom_adjoint: memset");
    ACHK(hipMemsetAsync(J, 0, mK * 8, st), "rom_adjoint: memset");
    rom::Rank2Args a;
    a.b = ctx->b; a.c = c; a.mu = mu; a.kv = kv; a.ks = ks; a.kvp = ctx->kvp; a.ksp = ctx->ksp;
    a.M = M; a.dt = ctx->dt; a.avs = ctx->avs_pk; a.asv = ctx->asv_pk; a.y = nullptr; a.source = ctx_source(ctx);
    // The forward sweep is a plain run with a probe: it takes the schedule a
    // rom_run_rank2 of this shape would (flags, table or tuner), e.g. the
    // row-split kernels where they beat the column blocks.  The recompute
    // and reverse sweeps need the traced column-block kernels.
    int fsched = ROM_SCHEDULE_COLUMNS4, fG = 0;
    a.V = curV; a.S = curS; a.J = J; a.n0 = 0; a.nsteps = nsteps;
    {
        rom_status rs = pick_schedule(ctx, a, st, fsched, fG);
        if (rs != ROM_OK) return rs;
    }
    if (rev) {
        rom_status rs = launch_fp32_state_run(ctx, a, fsched, fG, st);
        if (rs != ROM_OK) return rs;
    }
    for (int64_t g = 0; g < nseg && !rev; ++g) {
        const int64_t nb = g * C, len = (nb + C <= nsteps) ? C : nsteps - nb;
        float *cg = ck + (size_t)g * (v1 + s1);
        ACHK(hipMemcpyAsync(cg, curV, v1 * 4, hipMemcpyDeviceToDevice, st), "rom_adjoint: checkpoint");
        ACHK(hipMemcpyAsync(cg + v1, curS, s1 * 4, hipMemcpyDeviceToDevice, st), "rom_adjoint: checkpoint");
        a.V = curV; a.S = curS; a.J = J; a.n0 = nb; a.nsteps = len;
        rom_status rs = launch_fp32_state_run(ctx, a, fsched, fG, st);
        if (rs != ROM_OK) return rs;
    }
    if (fsched == ROM_SCHEDULE_ROWSPLIT) {
        // the forward sweep ran on the row-split kernels: a group barrier
        // that timed out leaves invalid checkpoints and J, so the reverse
        // sweep is not started (this synchronises `stream`)
        ACHK(hipStreamSynchronize(st), "rom_adjoint: synchronize");
        bool to = false;
        rom_status rs = take_timeout(ctx->status, to, "rom_adjoint: status");
        if (rs != ROM_OK) return rs;
        if (to) return fail(ROM_E_TIMEOUT, "rom_adjoint: a row-split group barrier of the forward sweep timed out");
    }
    // With a checkpointed forward sweep on the row-split kernels, the
    // recompute and reverse sweeps run on them too: the traced and adjoint
    // row-split variants, one after the other on `stream` (cooperative
    // launches may not share the chip), with the gradient products of each
    // segment on side stream 1 beside the next segment's launches.
    const bool split_adj = fsched == ROM_SCHEDULE_ROWSPLIT && !rev;
    if (split_adj && !ctx->asvT_sp) {
        const size_t pk = sizeof(float) * (size_t)ctx->kvp * ctx->ksp;
        e = hipMalloc(&ctx->asvT_sp, pk);
        if (e == hipSuccess) e = hipMalloc(&ctx->avsT_sp, pk);
        if (e != hipSuccess) {
            hfree(ctx->asvT_sp); hfree(ctx->avsT_sp);
            ctx->asvT_sp = ctx->avsT_sp = nullptr;
            return fail(ROM_E_NOMEM, "rom_adjoint: device allocation failed");
        }
        // Asv^T (Kv x Ks) from Asv (Ks x Kv), Avs^T (Ks x Kv) from Avs
        ACHK(rom::launch_split_pack_f32(static_cast<const float *>(ctx->asv_cm), kv, ks, ctx->kvp, ctx->ksp,
                                        ctx->asvT_sp, st, true), "rom_adjoint: split pack");
        ACHK(rom::launch_split_pack_f32(static_cast<const float *>(ctx->avs_cm), ks, kv, ctx->ksp, ctx->kvp,
                                        ctx->avsT_sp, st, true), "rom_adjoint: split pack");
    }
    // reverse sweep, segment by segment from the last.  Segment g's state
    // and probe traces (set g % kTr) are written by its recompute (side
    // stream 0) and read by its reverse sweep (this stream) and its gradient
    // products (side stream 1), as are its W and Q traces (set g % kWq,
    // written by the reverse sweep); a set is rewritten only after the
    // products of the segment that used it before.  Events: ev[0] forward
    // sweep done; ev[1 + i] trace set i free; ev[4 + i] trace set i
    // recomputed; ev[7 + i] W/Q set i free; ev[9 + i] reverse sweep into W/Q
    // set i done; ev[11], ev[12] side streams drained.
    hipStream_t s2 = ctx->side[0], s3 = ctx->side[1];
    hipEvent_t ev_fwd = ctx->ev[0], *ev_tr_free = ctx->ev + 1, *ev_rec = ctx->ev + 4;
    hipEvent_t *ev_wq_free = ctx->ev + 7, *ev_rev = ctx->ev + 9;
    auto recompute = [&](int64_t g) -> hipError_t {
        const int64_t nb = g * C, len = (nb + C <= nsteps) ? C : nsteps - nb;
        const int b = (int)(g % kTr);
        hipError_t r = hipSuccess;
        if (g + kTr < nseg) r = hipStreamWaitEvent(s2, ev_tr_free[b], 0);
        if (rev) {
            // (curV, curS) hold the state after the segment: step it back,
            // keeping every state, then recover the probe trace from them
            rom::Rank2Args iv = a;
            iv.V = curV; iv.S = curS; iv.c = nullptr; iv.J = nullptr; iv.y = nullptr; iv.n0 = nb; iv.nsteps = len;
            iv.vtr = vtrb[b]; iv.str = strb[b];
            if (r == hipSuccess) r = rom::launch_inverse_f32_mfma(iv, s2);
            if (r == hipSuccess) r = rom::launch_probe_trace(vtrb[b], static_cast<const float *>(c), kv, M, len,
                                                             ytrb[b], s2);
            if (r == hipSuccess) r = hipEventRecord(ev_rec[b], s2);
            return r;
        }
        const float *cg = ck + (size_t)g * (v1 + s1);
        if (r == hipSuccess) r = hipMemcpyAsync(curV, cg, v1 * 4, hipMemcpyDeviceToDevice, s2);
        if (r == hipSuccess) r = hipMemcpyAsync(curS, cg + v1, s1 * 4, hipMemcpyDeviceToDevice, s2);
        // recompute the segment, keeping every state and the probe trace
        rom::Rank2Args fw = a;
        fw.V = curV; fw.S = curS; fw.J = nullptr; fw.y = ytrb[b]; fw.n0 = nb; fw.nsteps = len;
        fw.vtr = vtrb[b]; fw.str = strb[b];
        if (r == hipSuccess) r = rom::launch_rank2_f32_mfma(fw, 1, s2);
        if (r == hipSuccess) r = hipEventRecord(ev_rec[b], s2);
        return r;
    };
    ACHK(hipMemsetAsync(P, 0, (v1 + s1) * 4, st), "rom_adjoint: memset");
    ACHK(hipMemsetAsync(dA64, 0, n_da * 8, st), "rom_adjoint: memset");
    if (dmu) ACHK(hipMemsetAsync(dmu, 0, mK * 8, st), "rom_adjoint: memset");
    ACHK(hipEventRecord(ev_fwd, st), "rom_adjoint: event");
    ACHK(hipStreamWaitEvent(s2, ev_fwd, 0), "rom_adjoint: event");
    ACHK(hipStreamWaitEvent(s3, ev_fwd, 0), "rom_adjoint: event");
    // gradient products of a reversed segment (side stream 1), then its
    // trace sets are free again
    auto products = [&](int64_t g) -> hipError_t {
        const int64_t len = (g * C + C <= nsteps) ? C : nsteps - g * C;
        const int b = (int)(g % kTr), bw = (int)(g % kWq);
        // dAvs += dt sum_n W^n (S^n)^T ;  dAsv += dt sum_n Q^{n+1} (V^{n+1})^T
        hipError_t r = hipStreamWaitEvent(s3, ev_rev[bw], 0);
        if (r == hipSuccess && dAvs) r = rom::launch_gemm_nt_acc64(wtrb[bw], strb[b], kv, ks, len * M, ctx->dt, dAvs64, part, s3);
        if (r == hipSuccess && dAsv)
            r = rom::launch_gemm_nt_acc64(qtrb[bw], vtrb[b] + v1, ks, kv, len * M, ctx->dt, dAsv64, part, s3);
        if (r == hipSuccess) r = hipEventRecord(ev_tr_free[b], s3);
        if (r == hipSuccess) r = hipEventRecord(ev_wq_free[bw], s3);
        return r;
    };
    // row-split arguments of segment g's recompute (from its checkpoint,
    // keeping every state and the probe trace) and reverse sweep (steps
    // nb + len - 1 .. nb: source c, probe b)
    auto split_rec = [&](int64_t g) {
        const int64_t nb = g * C, len = (nb + C <= nsteps) ? C : nsteps - nb;
        rom::Rank2Args fw = a;
        fw.V = curV; fw.S = curS; fw.J = nullptr; fw.y = ytrb[g % kTr]; fw.n0 = nb; fw.nsteps = len;
        fw.vtr = vtrb[g % kTr]; fw.str = strb[g % kTr];
        return fw;
    };
    auto split_rev = [&](int64_t g) {
        const int64_t nb = g * C, len = (nb + C <= nsteps) ? C : nsteps - nb;
        rom::Rank2Args ad = a;
        ad.b = c; ad.c = ctx->b; ad.V = P; ad.S = Q; ad.J = nullptr; ad.y = nullptr;
        ad.n0 = nb; ad.nsteps = len; ad.ytr = ytrb[g % kTr]; ad.wtr = wtrb[g % kWq]; ad.qtr = qtrb[g % kWq];
        ad.dmu = dmu;
        return ad;
    };
    auto load_ckpt = [&](int64_t g) -> hipError_t {
        const float *cg = ck + (size_t)g * (v1 + s1);
        hipError_t r = hipMemcpyAsync(curV, cg, v1 * 4, hipMemcpyDeviceToDevice, st);
        if (r == hipSuccess) r = hipMemcpyAsync(curS, cg + v1, s1 * 4, hipMemcpyDeviceToDevice, st);
        return r;
    };
    // Side by side: where two runs of this shape fit one launch, segment g's
    // reverse sweep and segment g - 1's recompute share a launch (disjoint
    // workgroups, a second workspace); otherwise they run one after the
    // other.
    bool dual = split_adj && nseg > 1 && rom::rank2_split_dual_width(ctx->kvp, M) >= 0;
    if (dual) {
        const size_t need = rom::rank2_split_workspace_bytes(ctx->kvp, fG);
        if (ctx->sp_ws2_bytes < need) {
            ACHK(hipStreamSynchronize(st), "rom_adjoint: synchronize");
            hfree(ctx->sp_ws2);
            ctx->sp_ws2 = nullptr;
            ctx->sp_ws2_bytes = 0;
            e = hipMalloc(&ctx->sp_ws2, need);
            if (e != hipSuccess) {
                ctx->sp_ws2 = nullptr;
                return fail(ROM_E_NOMEM, "rom_adjoint: workspace allocation failed");
            }
            ctx->sp_ws2_bytes = need;
        }
    }
    if (split_adj) {
        if (dual) {
            ACHK(load_ckpt(nseg - 1), "rom_adjoint: copy");
            ACHK(rom::launch_rank2_split(ctx->avs_sp, ctx->asv_sp, split_rec(nseg - 1), 1.0f, ctx->sp_ws, fG,
                                         ctx->status, true, st, 1), "rom_adjoint: recompute");
        }
        for (int64_t g = nseg - 1; g >= 0; --g) {
            const int b = (int)(g % kTr), bw = (int)(g % kWq);
            if (g + kWq < nseg) ACHK(hipStreamWaitEvent(st, ev_wq_free[bw], 0), "rom_adjoint: event");
            if (dual && g >= 1) {
                const int b1 = (int)((g - 1) % kTr);
                if (g - 1 + kTr < nseg) ACHK(hipStreamWaitEvent(st, ev_tr_free[b1], 0), "rom_adjoint: event");
                ACHK(load_ckpt(g - 1), "rom_adjoint: copy");
                ACHK(rom::launch_rank2_split_dual(ctx->avs_sp, ctx->asv_sp, split_rec(g - 1), ctx->sp_ws,
                                                  ctx->asvT_sp, ctx->avsT_sp, split_rev(g), ctx->sp_ws2, fG,
                                                  ctx->status, st), "rom_adjoint: recompute + reverse launch");
            } else {
                if (!dual) {
                    if (g + kTr < nseg) ACHK(hipStreamWaitEvent(st, ev_tr_free[b], 0), "rom_adjoint: event");
                    ACHK(load_ckpt(g), "rom_adjoint: copy");
                    ACHK(rom::launch_rank2_split(ctx->avs_sp, ctx->asv_sp, split_rec(g), 1.0f, ctx->sp_ws, fG,
                                                 ctx->status, true, st, 1), "rom_adjoint: recompute");
                }
                ACHK(rom::launch_rank2_split(ctx->asvT_sp, ctx->avsT_sp, split_rev(g), 1.0f, ctx->sp_ws, fG,
                                             ctx->status, true, st, 2), "rom_adjoint: reverse launch");
            }
            ACHK(hipEventRecord(ev_rev[bw], st), "rom_adjoint: event");
            ACHK(products(g), "rom_adjoint: gradient product");
        }
    }
    if (!split_adj) ACHK(recompute(nseg - 1), "rom_adjoint: recompute");
    for (int64_t g = nseg - 1; g >= 0 && !split_adj; --g) {
        const int64_t nb = g * C, len = (nb + C <= nsteps) ? C : nsteps - nb;
        const int b = (int)(g % kTr), bw = (int)(g % kWq);
        if (g >= 1) ACHK(recompute(g - 1), "rom_adjoint: recompute");
        ACHK(hipStreamWaitEvent(st, ev_rec[b], 0), "rom_adjoint: event");
        if (g + kWq < nseg) ACHK(hipStreamWaitEvent(st, ev_wq_free[bw], 0), "rom_adjoint: event");
        // reverse steps nb + len - 1 .. nb
        rom::Rank2Args ad = a;
        ad.avs = ctx->asvT_pk; ad.asv = ctx->avsT_pk; ad.V = P; ad.S = Q; ad.J = nullptr;
        ad.n0 = nb; ad.nsteps = len; ad.ytr = ytrb[b]; ad.wtr = wtrb[bw]; ad.qtr = qtrb[bw]; ad.dmu = dmu;
        ACHK(rom::launch_adjoint_f32_mfma(ad, st), "rom_adjoint: reverse launch");
        ACHK(hipEventRecord(ev_rev[bw], st), "rom_adjoint: event");
        ACHK(products(g), "rom_adjoint: gradient product");
    }
    // join: nothing of this call stays on the side streams
    ACHK(hipEventRecord(ctx->ev[11], s2), "rom_adjoint: event");
    ACHK(hipEventRecord(ctx->ev[12], s3), "rom_adjoint: event");
    ACHK(hipStreamWaitEvent(st, ctx->ev[11], 0), "rom_adjoint: event");
    ACHK(hipStreamWaitEvent(st, ctx->ev[12], 0), "rom_adjoint: event");
    if (dAvs) ACHK(rom::launch_f64_to_f32(dAvs64, (float *)dAvs, (int64_t)kv * ks, st), "rom_adjoint: convert");
    if (dAsv) ACHK(rom::launch_f64_to_f32(dAsv64, (float *)dAsv, (int64_t)kv * ks, st), "rom_adjoint: convert");
    if (split_adj) {
        // the recompute and reverse sweeps ran on the row-split kernels: a
        // timed-out group barrier makes the gradients invalid (this
        // synchronises `stream`)
        ACHK(hipStreamSynchronize(st), "rom_adjoint: synchronize");
        bool to = false;
        rom_status rs = take_timeout(ctx->status, to, "rom_adjoint: status");
        if (rs != ROM_OK) return rs;
        if (to) return fail(ROM_E_TIMEOUT, "rom_adjoint: a row-split group barrier of the reverse sweep timed out");
    }
#undef ACHK
    return ROM_OK;
}

rom_status rom_run_receivers(rom_ctx *ctx, int32_t M, const double *mu, int64_t n0, int64_t nsteps, void *V,
                             void *S, int32_t R, const void *C, double *Y, double *stats, void *stream) {
    if (!ctx) return fail(ROM_E_ARG, "rom_run_receivers: NULL context");
    if (M < 1 || M > 1024) return fail(ROM_E_ARG, "rom_run_receivers: M must be in [1, 1024]");
    if (R < 1 || R > 64) return fail(ROM_E_ARG, "rom_run_receivers: R must be in [1, 64]");
    if (!mu || !V || !S || !C) return fail(ROM_E_ARG, "rom_run_receivers: NULL mu, V, S or C");
    if (n0 < 0 || nsteps < 0) return fail(ROM_E_ARG, "rom_run_receivers: n0 and nsteps must be >= 0");
    if (ctx->state_type != ROM_F32 || ctx->op_type != ROM_F32)
        return fail(ROM_E_UNSUPPORTED, "rom_run_receivers: FP32 states and operators only");
    if (ctx->kvp + ctx->ksp > rom::kMaxPadSum || rom::rank2_f32_mfma_lds_bytes(ctx->kvp, ctx->ksp, 1) > 160 * 1024)
        return fail(ROM_E_UNSUPPORTED, "rom_run_receivers: Kv + Ks above the LDS-resident limit");
    if ((int64_t)R * M > 8192 || rom::receivers_lds_bytes(ctx->kv, M, R) > 160 * 1024)
        return fail(ROM_E_UNSUPPORTED, "rom_run_receivers: R x M or R x Kv too large for one workgroup's LDS");
    if (nsteps == 0) return ROM_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    const int kv = ctx->kv, ks = ctx->ks;
    // chunk length: one set of state traces within 256 MiB
    const size_t per_step = (size_t)(kv + ks) * M * sizeof(float);
    int64_t L = (int64_t)((256u << 20) / per_step);
    L = std::max<int64_t>(1, std::min<int64_t>(L, std::min<int64_t>(nsteps, 4096)));
    const size_t n_tr = (size_t)(L + 1) * (kv + ks) * M;              // floats per set: V then S traces
    const size_t n_set = ((n_tr + 3) / 4 * 4 * sizeof(float) + (size_t)L * M * sizeof(double) + 255) / 256 * 256;
    const size_t bytes = 2 * n_set;
    if (!ctx->side[0]) {
        e = hipSuccess;
        for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking);
        for (int i = 0; i < 13 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ctx->ev[i], hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "rom_run_receivers: stream / event creation");
    }
    if (!ctx->rc_ev[0]) {
        e = hipSuccess;
        for (int i = 0; i < 5 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ctx->rc_ev[i], hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "rom_run_receivers: event creation");
    }
    if (ctx->rc_ws_bytes < bytes) {
        e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->side[0]);
        if (e != hipSuccess) return hip_fail(e, "rom_run_receivers: synchronize");
        hfree(ctx->rc_ws);
        ctx->rc_ws = nullptr;
        ctx->rc_ws_bytes = 0;
        e = hipMalloc(&ctx->rc_ws, bytes);
        if (e != hipSuccess) { ctx->rc_ws = nullptr; return fail(ROM_E_NOMEM, "rom_run_receivers: workspace allocation failed"); }
        ctx->rc_ws_bytes = bytes;
    }
    float *vtr[2], *str[2];
    double *ysc[2];
    for (int b = 0; b < 2; ++b) {
        char *base = static_cast<char *>(ctx->rc_ws) + b * n_set;
        vtr[b] = reinterpret_cast<float *>(base);
        str[b] = vtr[b] + (size_t)(L + 1) * kv * M;
        ysc[b] = reinterpret_cast<double *>(base + (n_tr + 3) / 4 * 4 * sizeof(float));
    }
    // Chunk c is stepped on the caller's stream into trace set c % 2 (the
    // first receiver row doubles as the stepper's probe, whose trace goes to
    // scratch), and its seismograms and statistics are taken on the side
    // stream while the next chunk steps; a set is stepped into again only
    // after the side stream has read it.
    hipStream_t s2 = ctx->side[0];
    rom::Rank2Args a;
    a.b = ctx->b; a.c = C; a.mu = mu; a.V = V; a.S = S; a.J = nullptr;
    a.kv = kv; a.ks = ks; a.kvp = ctx->kvp; a.ksp = ctx->ksp; a.M = M; a.dt = ctx->dt; a.source = ctx_source(ctx);
    a.avs = ctx->avs_pk; a.asv = ctx->asv_pk;
    const int64_t nchunk = (nsteps + L - 1) / L;
    for (int64_t c = 0; c < nchunk; ++c) {
        const int b = (int)(c & 1);
        const int64_t len = std::min<int64_t>(L, nsteps - c * L);
        if (c >= 2) {
            e = hipStreamWaitEvent(st, ctx->rc_ev[2 + b], 0);
            if (e != hipSuccess) return hip_fail(e, "rom_run_receivers: event");
        }
        a.n0 = n0 + c * L; a.nsteps = len; a.vtr = vtr[b]; a.str = str[b]; a.y = ysc[b];
        e = rom::launch_rank2_f32_mfma(a, 1, st);
        if (e == hipSuccess) e = hipEventRecord(ctx->rc_ev[b], st);
        if (e == hipSuccess) e = hipStreamWaitEvent(s2, ctx->rc_ev[b], 0);
        if (e == hipSuccess)
            e = rom::launch_receivers(vtr[b], kv, M, (int)len, static_cast<const float *>(C), R,
                                      Y ? Y + (size_t)c * L * R * M : nullptr,
                                      stats ? stats + (size_t)c * L * R * 5 : nullptr, s2);
        if (e == hipSuccess) e = hipEventRecord(ctx->rc_ev[2 + b], s2);
        if (e != hipSuccess) return hip_fail(e, "rom_run_receivers: launch");
    }
    e = hipEventRecord(ctx->rc_ev[4], s2);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ctx->rc_ev[4], 0);
    if (e != hipSuccess) return hip_fail(e, "rom_run_receivers: event");
    return ROM_OK;
}

}  // extern "C"

namespace {

// Validate a grouped request and build the per-instance arguments (each
// with its column tile) and the (instance, first column) items, longest
// tuned step time first.  Tile times missing from the table are tuned on
// `st` (synchronously).
rom_status build_group(rom_ctx *const *ctx, int32_t G, const int32_t *M, const double *const *mu,
                       void *const *V, void *const *S, hipStream_t st, std::vector<rom::Rank2Args> &inst,
                       std::vector<int2> &items, size_t &lds) {
    if (!ctx || !M || !mu || !V || !S) return fail(ROM_E_ARG, "grouped: NULL array");
    if (G < 1) return fail(ROM_E_ARG, "grouped: G must be >= 1");
    inst.assign(G, rom::Rank2Args());
    std::vector<float> cost(G, 0.f);
    lds = 0;
    for (int i = 0; i < G; ++i) {
        rom_ctx *c = ctx[i];
        if (!c) return fail(ROM_E_ARG, "grouped: NULL context");
        if (M[i] < 1) return fail(ROM_E_ARG, "grouped: every M[i] must be >= 1");
        if (!mu[i] || !V[i] || !S[i]) return fail(ROM_E_ARG, "grouped: NULL mu, V or S");
        if (c->state_type != ROM_F32 || c->op_type != ROM_F32)
            return fail(ROM_E_UNSUPPORTED, "grouped: FP32 states and operators only");
        if (c->kvp + c->ksp > rom::kMaxPadSum || rom::rank2_f32_mfma_lds_bytes(c->kvp, c->ksp, 1) > 160 * 1024)
            return fail(ROM_E_UNSUPPORTED, "grouped: an instance exceeds the LDS-resident limit");
    }
    for (int i = 0; i < G; ++i) {
        rom_ctx *c = ctx[i];
        int nset = 1;
        float t4 = -1.f, t8 = -1.f;
        if (c->flags & ROM_SCHED_COLUMNS8) {
            nset = cols8_ok(c) ? 2 : 1;
        } else if (!(c->flags & ROM_SCHED_COLUMNS)) {
            TuneEntry te;
            rom_status rs = tile_times(c, st, te);
            if (rs != ROM_OK) return rs;
            t4 = te.us[ROM_SCHEDULE_COLUMNS4];
            t8 = cols8_ok(c) ? te.us[ROM_SCHEDULE_COLUMNS8] : -1.f;
            const int b4 = (M[i] + rom::kColBlock - 1) / rom::kColBlock;
            const int b8 = (M[i] + 2 * rom::kColBlock - 1) / (2 * rom::kColBlock);
            if (t4 >= 0.f && t8 >= 0.f && (float)b8 * t8 < (float)b4 * t4) nset = 2;
        }
        // item cost: the tuned per-workgroup step time, else operator size x columns
        const float tt = nset == 2 ? t8 : t4;
        cost[i] = tt >= 0.f ? tt : 1e-6f * (float)c->kvp * (float)c->ksp * (float)nset;
        const size_t b = rom::rank2_f32_mfma_lds_bytes(c->kvp, c->ksp, nset);
        if (b > lds) lds = b;
        rom::Rank2Args &a = inst[i];
        a.avs = c->avs_pk; a.asv = c->asv_pk; a.b = c->b; a.c = nullptr; a.mu = mu[i];
        a.V = V[i]; a.S = S[i]; a.J = nullptr; a.y = nullptr;
        a.kv = c->kv; a.ks = c->ks; a.kvp = c->kvp; a.ksp = c->ksp; a.M = M[i];
        a.n0 = 0; a.nsteps = 0; a.dt = c->dt; a.source = ctx_source(c);
        a.nset = nset;
    }
    std::vector<int> order(G);
    for (int i = 0; i < G; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    items.clear();
    for (int i : order) {
        const int nc = rom::kColBlock * inst[i].nset;
        for (int c0 = 0; c0 < inst[i].M; c0 += nc) items.push_back(make_int2(i, c0));
    }
    return ROM_OK;
}

using rom::SplitPlan;
using rom::SplitDev;

// Whether instance i can run in a grouped row-split launch: square FP32,
// padded K the row-split kernels take, a device that runs them, and not
// pinned to column blocks.
bool split_eligible(rom_ctx *c) {
    if (c->kv != c->ks || (c->flags & (ROM_SCHED_COLUMNS | ROM_SCHED_COLUMNS8))) return false;
    return split_candidate(c, 64) > 0;
}

// Packing of row-split groups into cooperative launches (host logic only):
// kp[q] is group q's padded K (K / 64 slots on one XCD of 32).  Groups go in
// order of decreasing K (stable), each into the first launch with an XCD
// that has K / 64 free slots, on the XCD of that launch with the most free
// slots; a launch's step takes as long as its largest-K group's, so the
// smaller groups fill what the larger ones left.  Returns per launch its
// members (indices into kp, in placement order) and their XCDs.
struct PackedLaunch {
    std::vector<int> mem, xcd;
};
std::vector<PackedLaunch> pack_groups(const std::vector<int> &kp) {
    std::vector<int> order(kp.size());
    for (size_t q = 0; q < kp.size(); ++q) order[q] = (int)q;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return kp[x] > kp[y]; });
    std::vector<PackedLaunch> ls;
    std::vector<std::array<int, 8>> freec;
    for (int q : order) {
        const int R = kp[q] / 64;
        int li = -1, xb = -1;
        for (int l = 0; l < (int)ls.size() && li < 0; ++l) {
            for (int x = 0; x < 8; ++x)
                if (freec[l][x] >= R && (xb < 0 || freec[l][x] > freec[l][xb])) xb = x;
            if (xb >= 0) li = l;
        }
        if (li < 0) {
            ls.emplace_back();
            freec.push_back({32, 32, 32, 32, 32, 32, 32, 32});
            li = (int)ls.size() - 1;
            xb = 0;
        }
        freec[li][xb] -= R;
        ls[li].mem.push_back(q);
        ls[li].xcd.push_back(xb);
    }
    return ls;
}

// Slot map of a packed launch: entry 32 xcd + s = 32 lg + r for row tile r
// of the launch's lg-th member, the members' tiles in consecutive slots of
// their XCD; -1 for idle slots.
std::vector<int> launch_slot_map(const PackedLaunch &L, const std::vector<int> &kp) {
    std::vector<int> sm(256, -1);
    int used[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t j = 0; j < L.mem.size(); ++j) {
        const int x = L.xcd[j], R = kp[L.mem[j]] / 64;
        for (int r = 0; r < R; ++r) sm[32 * x + used[x] + r] = 32 * (int)j + r;
        used[x] += R;
    }
    return sm;
}

// Row-split part of a grouped plan for the instances with use[i]: their
// 64-sample groups packed into launches (pack_groups).
void plan_split(rom_ctx *const *ctx, int32_t G, const int32_t *M, const double *const *mu, void *const *V,
                void *const *S, const std::vector<char> &use, SplitPlan &sp) {
    struct Cand { int inst, col0; };
    std::vector<Cand> cand;
    std::vector<int> kp;
    for (int i = 0; i < G; ++i)
        if (use[i])
            for (int c0 = 0; c0 < M[i]; c0 += 64) {
                cand.push_back({i, c0});
                kp.push_back(ctx[i]->kvp);
            }
    const std::vector<PackedLaunch> ls = pack_groups(kp);
    sp = SplitPlan();
    sp.kmin = kp.empty() ? 0 : *std::min_element(kp.begin(), kp.end());
    for (const PackedLaunch &L : ls) {
        const int g0 = (int)sp.groups.size();
        int64_t xoff = 0;
        for (size_t j = 0; j < L.mem.size(); ++j) {
            const Cand &c = cand[L.mem[j]];
            const int i = c.inst;
            rom::SplitGroup g{};
            g.opv = ctx[i]->avs_sp; g.ops = ctx[i]->asv_sp;
            g.b = static_cast<const float *>(ctx[i]->b);
            g.mu = mu[i];
            g.V = static_cast<float *>(V[i]); g.S = static_cast<float *>(S[i]);
            g.dt = ctx[i]->dt;
            g.source = ctx_source(ctx[i]);
            g.kv = ctx[i]->kv; g.kp = kp[L.mem[j]]; g.M = M[i]; g.col0 = c.col0;
            g.xoff = xoff;
            xoff += 64 * (int64_t)g.kp;
            sp.groups.push_back(g);
            sp.owner.push_back(i);
        }
        const std::vector<int> sm = launch_slot_map(L, kp);
        sp.g0.push_back(g0);
        sp.ng.push_back((int)L.mem.size());
        sp.xfloats.push_back((size_t)xoff);
        sp.smap.insert(sp.smap.end(), sm.begin(), sm.end());
        sp.ws_bytes = std::max(sp.ws_bytes, rom::rank2_split_ws_bytes((size_t)xoff, 0));
    }
}

void free_split_dev(SplitDev &d) {
    hfree(d.groups); hfree(d.smap); hfree(d.ws); hfree(d.status);
    d = SplitDev();
}

hipError_t upload_split(const SplitPlan &sp, SplitDev &d) {
    hipError_t e = hipMalloc(&d.groups, sizeof(rom::SplitGroup) * sp.groups.size());
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&d.smap), sizeof(int) * sp.smap.size());
    if (e == hipSuccess) e = hipMalloc(&d.ws, sp.ws_bytes);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&d.status), sizeof(int) * 4);
    if (e == hipSuccess) e = hipMemset(d.status, 0, sizeof(int) * 4);
    if (e == hipSuccess)
        e = hipMemcpy(d.groups, sp.groups.data(), sizeof(rom::SplitGroup) * sp.groups.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.smap, sp.smap.data(), sizeof(int) * sp.smap.size(), hipMemcpyHostToDevice);
    return e;
}

// Row-split launches of a grouped run, one after another on `st`.
hipError_t launch_split_plan(const SplitPlan &sp, const SplitDev &d, int64_t n0, int64_t nsteps, hipStream_t st) {
    for (size_t l = 0; l < sp.g0.size(); ++l) {
        hipError_t e = rom::launch_grouped_split_f32(static_cast<const rom::SplitGroup *>(d.groups), sp.g0[l], sp.ng[l],
                                                     d.smap + 256 * l, sp.xfloats[l], d.ws, d.status, n0, nsteps, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Which plan a grouped shape runs: timed once per shape (the instances'
// padded K and sample counts) and remembered for the process, as the
// smallest padded K on row-split (0: column blocks only).
std::mutex g_gsched_mu;
std::map<std::vector<int>, int> g_gsched;

// Column-block items of the instances with use[i] == 0.
std::vector<int2> rest_items(const std::vector<int2> &items, const std::vector<char> &use) {
    std::vector<int2> r;
    for (const int2 &it : items)
        if (!use[it.x]) r.push_back(it);
    return r;
}

// Time a grouped plan (per step: best of two runs of kTuneSteps steps after
// a 2-step warm-up) on scratch states: the row-split launches of sp (none
// if it is empty), then column blocks over `items`.  The caller's mu arrays
// are read.  A plan whose row-split barrier timed out is reported as not
// applicable (us < 0).
rom_status time_group_plan(const std::vector<rom::Rank2Args> &inst, const std::vector<int2> &items, size_t lds,
                           const SplitPlan &sp, hipStream_t st, float &us) {
    const int G = (int)inst.size();
    std::vector<size_t> off(G + 1, 0);
    for (int i = 0; i < G; ++i) off[i + 1] = off[i] + (size_t)(inst[i].kv + inst[i].ks) * inst[i].M;
    std::vector<rom::Rank2Args> ic(inst);
    SplitPlan sc(sp);
    SplitDev sd;
    float *scr = nullptr;
    void *dev = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rom_status rs = ROM_OK;
    const size_t ib = sizeof(rom::Rank2Args) * ic.size(), tb = sizeof(int2) * std::max<size_t>(1, items.size());
    hipError_t e = hipMalloc(&scr, sizeof(float) * off[G]);
    if (e == hipSuccess) e = hipMalloc(&dev, ib + tb);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        for (int i = 0; i < G; ++i) {
            ic[i].V = scr + off[i];
            ic[i].S = scr + off[i] + (size_t)inst[i].kv * inst[i].M;
        }
        for (size_t q = 0; q < sc.groups.size(); ++q) {
            sc.groups[q].V = static_cast<float *>(ic[sc.owner[q]].V);
            sc.groups[q].S = static_cast<float *>(ic[sc.owner[q]].S);
        }
        if (!sc.groups.empty()) e = upload_split(sc, sd);
        char *d = static_cast<char *>(dev);
        if (e == hipSuccess) e = hipMemsetAsync(scr, 0, sizeof(float) * off[G], st);
        if (e == hipSuccess) e = hipMemcpyAsync(d, ic.data(), ib, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && !items.empty())
            e = hipMemcpyAsync(d + ib, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (e != hipSuccess) rs = hip_fail(e, "grouped plan tuning: setup");
    const char *d = static_cast<const char *>(dev);
    float best = 1e30f;
    for (int rep = 0; rep < 3 && rs == ROM_OK; ++rep) {   // rep 0: warm-up
        const int64_t n = rep == 0 ? 2 : kTuneSteps;
        e = rep > 0 ? hipEventRecord(e0, st) : hipSuccess;
        if (e == hipSuccess && !sc.groups.empty()) e = launch_split_plan(sc, sd, 0, n, st);
        if (e == hipSuccess && !items.empty())
            e = rom::launch_grouped_f32_mfma(reinterpret_cast<const rom::Rank2Args *>(d),
                                             reinterpret_cast<const int2 *>(d + ib), (int)items.size(), lds, 0, n, st);
        if (e == hipSuccess && rep > 0) e = hipEventRecord(e1, st);
        if (e == hipSuccess && rep > 0) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess && rep > 0) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { rs = hip_fail(e, "grouped plan tuning"); break; }
        if (rep > 0) best = std::min(best, ms * 1e3f / (float)n);
    }
    if (rs == ROM_OK) e = hipStreamSynchronize(st);
    if (rs == ROM_OK && e != hipSuccess) rs = hip_fail(e, "grouped plan tuning");
    if (rs == ROM_OK && sd.status) {
        int w[2] = {0, 0};
        e = hipMemcpy(w, sd.status + 1, sizeof(w), hipMemcpyDeviceToHost);
        if (e == hipSuccess && (w[0] != 0 || w[1] != 0)) best = -1.f;
        if (e != hipSuccess) rs = hip_fail(e, "grouped plan tuning: status");
    }
    us = best;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    free_split_dev(sd);
    hfree(scr);
    hfree(dev);
    return rs;
}

// Free a plan's device memory (its work must have completed).
void free_group(rom_group *g) {
    hfree(g->dev);
    hfree(g->rest);
    free_split_dev(g->sp);
    delete g;
}

// Build a plan: the column-block descriptor table of every instance always
// (graph capture runs it); when the row-split kernels apply to some
// instances and are forced or timed faster, the row-split launches for the
// instances from a padded K threshold up and the column-block items of the
// rest.  Candidate thresholds: each padded K of the eligible instances (all
// of them on row-split when every instance asks for that schedule).  Tuning
// runs on `st` and synchronises it.
rom_status make_group(rom_ctx *const *ctx, int32_t G, const int32_t *M, const double *const *mu, void *const *V,
                      void *const *S, hipStream_t st, const char *who, rom_group **out) {
    std::string w(who);
    std::vector<rom::Rank2Args> inst;
    std::vector<int2> items;
    size_t lds = 0;
    rom_status r = build_group(ctx, G, M, mu, V, S, st, inst, items, lds);
    if (r != ROM_OK) return r;
    std::vector<char> elig(G, 0);
    bool forced = true, any = false;
    if (!stream_capturing(st)) {
        for (int i = 0; i < G; ++i) {
            elig[i] = split_eligible(ctx[i]) ? 1 : 0;
            any = any || elig[i];
            if (!elig[i] || !(ctx[i]->flags & ROM_SCHED_ROWSPLIT)) forced = false;
        }
    }
    if (any) {
        for (int i = 0; i < G; ++i)
            if (elig[i]) {
                r = prepare_split_pack(ctx[i], st);
                if (r != ROM_OK) return r;
            }
        hipError_t es = hipStreamSynchronize(st);   // the packs are complete before any plan runs
        if (es != hipSuccess) return hip_fail(es, (w + ": synchronize").c_str());
    }
    rom_group *g = new (std::nothrow) rom_group();
    if (!g) return fail(ROM_E_NOMEM, w + ": host allocation failed");
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) { free_group(g); return hip_fail(e, (w + ": hipGetDevice").c_str()); }
    const size_t ib = sizeof(rom::Rank2Args) * inst.size();
    const size_t bytes = ib + sizeof(int2) * items.size();
    e = hipMalloc(&g->dev, bytes);
    if (e != hipSuccess) { free_group(g); return fail(ROM_E_NOMEM, w + ": device allocation failed"); }
    e = hipMemcpy(g->dev, inst.data(), ib, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(static_cast<char *>(g->dev) + ib, items.data(), sizeof(int2) * items.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) { free_group(g); return hip_fail(e, (w + ": upload").c_str()); }
    g->G = G;
    g->nitems = (int)items.size();
    g->lds_bytes = lds;
    g->inst = static_cast<const rom::Rank2Args *>(g->dev);
    g->items = reinterpret_cast<const int2 *>(static_cast<char *>(g->dev) + ib);
    if (any) {
        std::vector<int> ks;
        for (int i = 0; i < G; ++i)
            if (elig[i]) ks.push_back(ctx[i]->kvp);
        std::sort(ks.begin(), ks.end());
        ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
        auto use_from = [&](int t) {
            std::vector<char> u(G, 0);
            for (int i = 0; i < G; ++i) u[i] = (t > 0 && elig[i] && ctx[i]->kvp >= t) ? 1 : 0;
            return u;
        };
        int t = forced ? ks.front() : -1;
        if (!forced) {
            std::vector<int> key;
            for (int i = 0; i < G; ++i) { key.push_back(elig[i] ? ctx[i]->kvp : -ctx[i]->kvp); key.push_back(M[i]); }
            {
                std::lock_guard<std::mutex> lk(g_gsched_mu);
                auto it = g_gsched.find(key);
                if (it != g_gsched.end()) t = it->second;
            }
            if (t < 0) {
                float tc = -1.f;
                SplitPlan none;
                r = time_group_plan(inst, items, lds, none, st, tc);
                if (r != ROM_OK) { free_group(g); return r; }
                float tb = -1.f;
                int best = 0;
                for (int k : ks) {
                    SplitPlan sp;
                    const std::vector<char> u = use_from(k);
                    plan_split(ctx, G, M, mu, V, S, u, sp);
                    float ts = -1.f;
                    r = time_group_plan(inst, rest_items(items, u), lds, sp, st, ts);
                    if (r != ROM_OK) { free_group(g); return r; }
                    if (ts >= 0.f && (tb < 0.f || ts < tb)) { tb = ts; best = k; }
                }
                g->us[0] = tc;
                g->us[1] = tb;
                t = (tb >= 0.f && tb < tc) ? best : 0;
                std::lock_guard<std::mutex> lk(g_gsched_mu);
                g_gsched[key] = t;
            }
        }
        if (t > 0) {
            const std::vector<char> u = use_from(t);
            plan_split(ctx, G, M, mu, V, S, u, g->plan);
            e = upload_split(g->plan, g->sp);
            const std::vector<int2> rest = rest_items(items, u);
            if (e == hipSuccess && !rest.empty()) {
                e = hipMalloc(&g->rest, sizeof(int2) * rest.size());
                if (e == hipSuccess)
                    e = hipMemcpy(g->rest, rest.data(), sizeof(int2) * rest.size(), hipMemcpyHostToDevice);
            }
            if (e != hipSuccess) { free_group(g); return hip_fail(e, (w + ": row-split plan upload").c_str()); }
            g->nrest = (int)rest.size();
            g->ngroups = (int)g->plan.groups.size();
        }
    }
    *out = g;
    return ROM_OK;
}

// Enqueue a plan's run: with a row-split part and a stream not being
// captured, its launches and then column blocks over the other instances;
// else column blocks over all instances.
hipError_t run_group(rom_group *g, int64_t n0, int64_t nsteps, hipStream_t st) {
    if (g->ngroups > 0 && !stream_capturing(st)) {
        hipError_t e = launch_split_plan(g->plan, g->sp, n0, nsteps, st);
        if (e != hipSuccess || g->nrest == 0) return e;
        return rom::launch_grouped_f32_mfma(g->inst, static_cast<const int2 *>(g->rest), g->nrest, g->lds_bytes, n0,
                                            nsteps, st);
    }
    return rom::launch_grouped_f32_mfma(g->inst, g->items, g->nitems, g->lds_bytes, n0, nsteps, st);
}

}  // namespace

extern "C" {

int32_t rom_debug_pack_groups(const int32_t *kp, int32_t n, int32_t *launch, int32_t *member, int32_t *slot_maps,
                              int32_t max_launches) {
    if (!kp || n < 0 || !launch || !member || !slot_maps || max_launches < 1) return -1;
    std::vector<int> k(kp, kp + n);
    for (int v : k)
        if (v < 128 || v > rom::kMaxSplitK || v % 64 != 0) return -1;
    const std::vector<PackedLaunch> ls = pack_groups(k);
    if ((int)ls.size() > max_launches) return -1;
    for (size_t l = 0; l < ls.size(); ++l) {
        for (size_t j = 0; j < ls[l].mem.size(); ++j) {
            launch[ls[l].mem[j]] = (int32_t)l;
            member[ls[l].mem[j]] = (int32_t)j;
        }
        const std::vector<int> sm = launch_slot_map(ls[l], k);
        std::copy(sm.begin(), sm.end(), slot_maps + 256 * l);
    }
    return (int32_t)ls.size();
}

rom_status rom_group_create(rom_ctx *const *ctx, int32_t G, const int32_t *M, const double *const *mu,
                            void *const *V, void *const *S, rom_group **out) {
    if (out) *out = nullptr;
    if (!out) return fail(ROM_E_ARG, "rom_group_create: NULL out");
    return make_group(ctx, G, M, mu, V, S, nullptr, "rom_group_create", out);
}

rom_status rom_group_run(rom_group *g, int64_t n0, int64_t nsteps, void *stream) {
    if (!g) return fail(ROM_E_ARG, "rom_group_run: NULL plan");
    if (n0 < 0 || nsteps < 0) return fail(ROM_E_ARG, "rom_group_run: n0 and nsteps must be >= 0");
    hipError_t e = run_group(g, n0, nsteps, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "rom_group_run: launch");
    return ROM_OK;
}

int32_t rom_group_schedule(const rom_group *g) {
    if (!g) return -1;
    return g->ngroups > 0 ? ROM_SCHEDULE_ROWSPLIT : ROM_SCHEDULE_COLUMNS4;
}

int32_t rom_group_split_k(const rom_group *g) {
    if (!g) return -1;
    return g->ngroups > 0 ? g->plan.kmin : 0;
}

rom_status rom_group_times(const rom_group *g, double us[2]) {
    if (!g || !us) return fail(ROM_E_ARG, "rom_group_times: NULL argument");
    us[0] = g->us[0];
    us[1] = g->us[1];
    return ROM_OK;
}

rom_status rom_group_check(rom_group *g, void *stream) {
    if (!g) return fail(ROM_E_ARG, "rom_group_check: NULL plan");
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "rom_group_check: synchronize");
    if (!g->sp.status) return ROM_OK;
    int w[2] = {0, 0};
    e = hipMemcpy(w, g->sp.status + 1, sizeof(w), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "rom_group_check: read status");
    if (w[0] != 0 || w[1] != 0) {
        e = hipMemset(g->sp.status + 1, 0, sizeof(w));
        if (e != hipSuccess) return hip_fail(e, "rom_group_check: clear status");
        if (w[0] == ROM_E_TIMEOUT)
            return fail(ROM_E_TIMEOUT, "rom_group_check: a row-split group barrier timed out; the run's results are invalid");
    }
    return ROM_OK;
}

rom_status rom_group_destroy(rom_group *g) {
    if (!g) return ROM_OK;
    free_group(g);
    return ROM_OK;
}

rom_status rom_run_grouped(rom_ctx *const *ctx, int32_t G, const int32_t *M, const double *const *mu,
                           int64_t nsteps, void *const *V, void *const *S, void *stream) {
    if (nsteps < 0) return fail(ROM_E_ARG, "rom_run_grouped: nsteps must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    rom_group *g = nullptr;
    rom_status r = make_group(ctx, G, M, mu, V, S, st, "rom_run_grouped", &g);
    if (r != ROM_OK) return r;
    hipError_t e = nsteps > 0 ? run_group(g, 0, nsteps, st) : hipSuccess;
    // the plan's memory is released once its run has completed
    hipError_t e2 = hipStreamSynchronize(st);
    if (e == hipSuccess && e2 == hipSuccess && g->ngroups > 0) {
        r = rom_group_check(g, stream);
    }
    free_group(g);
    if (e != hipSuccess) return hip_fail(e, "rom_run_grouped: launch");
    if (e2 != hipSuccess) return hip_fail(e2, "rom_run_grouped: synchronize");
    return r;
}

}  // extern "C"
