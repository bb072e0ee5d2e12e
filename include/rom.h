/*
 * rom.h - C ABI of the MI355X (gfx950) rank-2 Galerkin ROM library.
 *
 * The library integrates M forcing samples of one Galerkin-projected,
 * staggered (velocity/stress) linear time-invariant system together.  The
 * reduced states of all samples are stacked as matrices (one sample per
 * column), so every leapfrog half-step is one dense operator x state-matrix
 * product plus a per-sample forcing update (the "rank-2" form of the paper,
 * Sec. 2.4 eq. (2.5), written for the two-field shear-wave system of
 * Sec. 3.1 eq. (3.3)).  The "rank-1" form (Sec. 2.2 eq. (2.3)) advances one
 * sample with two matrix-vector products per step.
 *
 * Problem (eq. (3.3); forcing-only parameters batched as in Sec. 2):
 *
 *   dV/dt = Avs S + b u(t; mu_m)        V: Kv x M (velocity coordinates)
 *   dS/dt = Asv V                       S: Ks x M (stress coordinates)
 *
 *   Avs  (Kv x Ks)  reduced velocity operator  (Phi_v^T A_v Phi_s)
 *   Asv  (Ks x Kv)  reduced stress operator    (Phi_s^T A_s Phi_v)
 *   b    (Kv)       reduced point source (sparse forcing, Sec. 2.2)
 *   u    Ricker wavelet (Sec. 3.2), per-sample centre frequency mu_m:
 *        u(t; mu) = (1 - 2a) exp(-a),  a = pi^2 (mu t - 1.5)^2
 *
 * Time integration: leapfrog, velocity first then stress (Sec. 3.1, the
 * paragraph after eq. (3.3)); the discrete form is
 *
 *   for n = n0 .. n0 + nsteps - 1,  t_n = n dt:
 *     V <- V + dt (Avs S + b u(t_n; mu)^T)
 *     S <- S + dt (Asv V)                 (uses the updated V)
 *
 * and, with a probe row c (a receiver, i.e. one row of Phi_v, Sec. 4.5):
 *     y_m = c^T V[:, m],   J_m += dt y_m^2
 *
 * Conventions shared by every entry point
 *  - Every function returns a rom_status.  On ROM_E_ARG nothing was enqueued
 *    and no output was written.  rom_last_error() returns a thread-local
 *    text for the last non-OK status of the calling thread.
 *  - Matrices are column-major: element (i, j) of an R x C matrix is at
 *    [i + j*R].  In particular a state matrix stores sample m contiguously
 *    at [m*K, (m+1)*K) (as the paper's BLAS layout, Sec. 4.2).
 *  - "dev" pointers are HIP device pointers owned by the caller; "host"
 *    pointers are ordinary host memory.  The library never frees caller
 *    memory.  Device buffers of state type hold `double` for ROM_F64 and
 *    `float` for ROM_F32 states.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    work on it and results are ready when it is synchronised.  Some calls
 *    also run work on internal streams of the context (default priority)
 *    and join them back into `stream` before returning (rom_adjoint,
 *    rom_run_receivers); a few synchronise `stream` (a rank-2 run that tunes
 *    its schedule, rom_create, rom_check, rom_run_grouped), as their
 *    comments say.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef ROM_H
#define ROM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ROM_OK = 0,
    ROM_E_ARG = 1,          /* invalid argument (nothing enqueued)            */
    ROM_E_NOMEM = 2,        /* device or host allocation failed               */
    ROM_E_DEVICE = 3,       /* HIP runtime error (launch, copy, fault)         */
    ROM_E_UNSTABLE = 4,     /* skew pair with dt * sigma_max(Avs) >= 2         */
    ROM_E_UNSUPPORTED = 5,  /* valid but unsupported combination               */
    ROM_E_NONFINITE = 6,    /* non-finite input values                         */
    ROM_E_TIMEOUT = 7       /* an in-kernel wait exceeded its time limit       */
} rom_status;

typedef enum {
    ROM_F64 = 0,
    ROM_F32 = 1,
    ROM_BF16 = 2,           /* operators only                                  */
    ROM_F8E4M3 = 3          /* operators only: OCP e4m3fn, per-tensor scale    */
} rom_dtype;

/* rom_config.flags */
enum {
    ROM_SKEW_CHECK = 1u,    /* if Asv == -Avs^T exactly, require
                               dt * sigma_max(Avs) < 2 (positivity of the
                               leapfrog's discrete energy); ROM_E_UNSTABLE
                               otherwise.  Non-skew pairs are not checked.   */
    ROM_SCHED_COLUMNS = 2u, /* FP32-state rank-2 runs (FP32, BF16, FP8
                               operators): always the 4-column column-block
                               kernels (each workgroup owns 4 samples and
                               streams the whole operator); FP64-state runs:
                               the vector-ALU column blocks where their
                               states fit in LDS                              */
    ROM_SCHED_ROWSPLIT = 4u,/* FP32-state rank-2 runs: the row-split kernels
                               (operator rows split over the workgroups of a
                               sample group, exchanged every half-step)
                               wherever they apply: Kv == Ks, padded K a
                               multiple of 64 in [128, 2048] (FP32
                               operators) or of 128 up to 1024 (BF16 / FP8),
                               all groups in one launch, a 256-CU gfx950;
                               else 4-column blocks.  Groups of 64
                               samples with BF16 / FP8 operators; with FP32
                               operators the narrowest of 16, 32, 64 whose
                               ceil(M/width) * K/64 workgroups fit in 256   */
    ROM_SCHED_COLUMNS8 = 8u,/* FP32 operators and states: 8-column blocks
                               (two column sets per operator fragment) where
                               the states of 8 samples fit in LDS; else 4.
                               At most one ROM_SCHED_* flag; none: the
                               schedule autotuner decides (rom_last_schedule)*/
    ROM_SOURCE_GAUSS1 = 16u /* source signal: the first derivative of a
                               Gaussian (Sec. 3.2), period 1/mu, delay 3/mu,
                               unit peak: u = -sqrt(2e) x exp(-x^2),
                               x = pi (mu t - 3); default: the Ricker wavelet
                               (1 - 2a) exp(-a), a = pi^2 (mu t - 1.5)^2.  The
                               adjoint's dJ/dmu differentiates the chosen one */,
    ROM_SCHED_RESIDENT = 64u,/* FP32 operators and states, skew pairs
                               (Asv == -Avs^T exactly) with Kv, Ks <= 256:
                               the operator-resident kernel (one sample per
                               workgroup, all of Avs in its registers); else
                               4-column blocks.  (FP64-state runs of skew
                               pairs with Kv_pad, Ks_pad <= 128, and of
                               other pairs with Kv_pad Ks_pad <= 8192, take
                               the FP64 resident kernel with or without it.)*/
    ROM_SCHED_PANEL = 128u, /* FP32 operators and states, or FP64 states:
                               the panel schedule (one tiled matrix-product
                               launch per half-step, nothing resident
                               between them), which runs of any Kv, Ks take
                               anyway where the column blocks' states do
                               not fit in LDS (FP32: Kv_pad + Ks_pad >
                               4096) and FP64 runs from Kv_pad + Ks_pad >=
                               768 (ROM_SCHED_COLUMNS keeps FP64 runs on
                               the vector-ALU column blocks where they fit,
                               and so does a stream under graph capture
                               before the panel workspace exists);
                               ignored with BF16 / FP8 operators and FP32
                               states                                       */
    ROM_STATE_BF16 = 32u    /* BF16 / F8E4M3 operators with F32 states: the
                               state operand of every product is bf16(x)
                               alone (one MFMA pass, about 8 significant
                               bits; the precision extension for matrix
                               units, Sec. 5) instead
                               of the pair bf16(x) + bf16(x - bf16(x)) (two
                               passes, about 16 bits).  Faster, at about
                               2e-2 relative state error after 10^3 steps
                               and 3e-2 after 5000 at K = 1024 (the
                               rounding is redone every half-step).  Such contexts share their
                               operator type's tuning-table entries.  Other
                               (op, state) pairs: ROM_E_ARG                  */
};

typedef struct {
    int32_t kv;             /* velocity reduced size Kv >= 1                   */
    int32_t ks;             /* stress reduced size Ks >= 1                     */
    double dt;              /* time step > 0 (the value used, as given)        */
    rom_dtype op_type;      /* operator precision in the products: F64 with F64
                               states, F32 with F32 states, BF16 / F8E4M3 with
                               F32 states (low-precision products) or F64
                               states (FP64 integration of the rounded
                               operators, the long-horizon reference)        */
    rom_dtype state_type;   /* ROM_F64 or ROM_F32: state and I/O precision    */
    uint32_t flags;         /* ROM_SKEW_CHECK | ...                            */
} rom_config;

typedef struct rom_ctx rom_ctx;

/*
 * Create a context on the current HIP device: validate the configuration,
 * copy the operators and source to the device, and prepare them for the
 * products (rounding to op_type, packing).  Operators are the time-
 * independent reduced matrices computed offline (Sec. 2.2, Sec. 4.2).
 *
 *   cfg   host, configuration (copied)
 *   Avs   host, Kv x Ks column-major FP64
 *   Asv   host, Ks x Kv column-major FP64
 *   b     host, Kv FP64
 *   stream  stream for the uploads (the call synchronises it before return)
 *   out   receives the context; set to NULL on failure
 *
 * The host arrays may be freed on return.  Errors: ROM_E_ARG (NULL pointer,
 * Kv or Ks < 1, dt <= 0 or not finite, state_type not F64/F32, op_type
 * narrower than... see rom_run_rank2), ROM_E_NONFINITE (NaN/Inf in inputs),
 * ROM_E_UNSTABLE (see ROM_SKEW_CHECK), ROM_E_UNSUPPORTED, ROM_E_NOMEM,
 * ROM_E_DEVICE.
 */
rom_status rom_create(const rom_config *cfg, const double *Avs, const double *Asv,
                      const double *b, void *stream, rom_ctx **out);

/*
 * Copy the operators exactly as the context's products use them to host
 * FP64 column-major arrays: Avs (Kv x Ks) and Asv (Ks x Kv) after rounding
 * to op_type (FP32, BF16 via FP32) and, for FP8-E4M3, multiplied by the
 * per-tensor scale, which is returned in *scale (1 otherwise; scale may be
 * NULL).  Lets a caller integrate the same operators with another
 * implementation.  Synchronises the device.
 */
rom_status rom_get_operators(rom_ctx *ctx, double *Avs, double *Asv, double *scale);

/*
 * Modified discrete energy of the leapfrog per sample, in FP64:
 *   E_m = |v_m|^2 + |s_m|^2 + dt v_m^T Avs s_m     (Avs as the products use it)
 * V, S dev states of state type (Kv x M, Ks x M); E dev, M FP64 (set).  For
 * a skew pair the unforced leapfrog conserves E exactly, and E is positive
 * definite when dt * sigma_max(Avs) < 2: its drift over a long run measures
 * the arithmetic, its size bounds the state (the stability check of the
 * low-precision runs, used with an FP64-state context of the same rounded
 * operators as the long-horizon reference).
 */
rom_status rom_energy(rom_ctx *ctx, int32_t M, const void *V, const void *S, double *E, void *stream);

/*
 * Release every device buffer and internal stream owned by the context
 * (library housekeeping: no passage of the paper defines it).  Work the
 * context enqueued must have completed.  NULL is accepted.  Errors: none
 * (always ROM_OK).
 */
rom_status rom_destroy(rom_ctx *ctx);

/*
 * Schedule of a rank-2 run with FP32 states.  Three kernel schedules
 * compute it with the same per-sample results up to rounding order:
 *   ROM_SCHEDULE_COLUMNS4  each workgroup owns 4 samples and streams the
 *                          whole operator; workgroups never wait for one
 *                          another;
 *   ROM_SCHEDULE_ROWSPLIT  operator rows split over the workgroups of a
 *                          sample group (16, 32 or 64 samples, see
 *                          ROM_SCHED_ROWSPLIT), kept in registers or
 *                          streamed per quarter, rows exchanged at a group
 *                          barrier every half-step;
 *   ROM_SCHEDULE_COLUMNS8  as COLUMNS4 with 8 samples per workgroup (FP32
 *                          operators): half the operator bytes per flop,
 *                          half the workgroups.  Bitwise equal to COLUMNS4.
 *   ROM_SCHEDULE_RESIDENT  skew pairs (Asv == -Avs^T exactly, the energy-
 *                          conserving structure of Sec. 3.1) with FP32
 *                          operators and Kv, Ks <= 256: one sample per
 *                          workgroup, which keeps all of Avs in registers
 *                          for the whole run and uses it for both half-
 *                          steps (Asv V = -Avs^T V); no operator streaming,
 *                          no exchange between workgroups.  FP64 states
 *                          (FP64 operators, or BF16 / FP8 ones) have an
 *                          FP64 form of it, for skew pairs (which stay
 *                          skew when rounded) with Kv_pad, Ks_pad <= 128
 *                          and for other pairs, holding Asv as well, with
 *                          Kv_pad Ks_pad <= 8192 (sizes padded to 64): every
 *                          such run takes it unless ROM_SCHED_COLUMNS pins
 *                          the vector-ALU column blocks.
 *   ROM_SCHEDULE_PANEL     FP32 operators, any Kv, Ks: each half-step one
 *                          launch of a tiled matrix product (128 operator
 *                          rows x 64 samples per workgroup, FP32 matrix
 *                          cores, FP64 compensated update in its epilogue);
 *                          states and probe partials in a context
 *                          workspace of about 8 (Kv + Ks) M bytes, operator
 *                          copies of 4 Kv Ks bytes each, both allocated on
 *                          the first such run (which must not be captured
 *                          into a graph: ROM_E_UNSUPPORTED).  Always taken
 *                          where Kv_pad + Ks_pad > 4096 or with
 *                          ROM_SCHED_PANEL; the autotuner weighs it from
 *                          Kv_pad + Ks_pad >= 2048 (under capture only
 *                          once its workspace covers the run).
 * Without a ROM_SCHED_* flag the first run of each shape (Kv_pad, Ks_pad, M
 * rounded up to 64, operator type) times every schedule that applies for 32
 * steps on scratch states and keeps the fastest for the process (that run
 * synchronises the stream; a row-split timing run whose group barrier timed
 * out counts as not applicable, and its status is cleared), unless the process-wide tuning table already
 * holds the shape.  A stream being captured into a graph is never tuned and
 * never takes ROWSPLIT (whatever the flags or the table say): it runs the
 * table's column-block choice, else COLUMNS4.
 *
 * The grouped launch (rom_run_grouped, rom_group_create) picks each
 * instance's column tile (4 or 8 samples) from the per-workgroup step times
 * of its (Kv_pad, Ks_pad) bucket, tuned on first use (one workgroup, 256
 * steps per tile) and kept in the same table with m_pad = 0; the instance
 * takes the tile minimising ceil(M / tile) x time.  A context flag
 * ROM_SCHED_COLUMNS / ROM_SCHED_COLUMNS8 fixes the instance's tile.
 *
 * rom_last_schedule: the schedule of the context's last FP32-state rank-2
 * run; after an FP64-state run ROM_SCHEDULE_PANEL (panel schedule),
 * ROM_SCHEDULE_RESIDENT (FP64 resident kernel) or -1 (vector-ALU column
 * blocks); -1 if none.  rom_schedule_times: the table's per-step times
 * (microseconds) of each schedule for the context's shape at M samples,
 * negative where a schedule does not apply; ROM_E_ARG if that shape is not
 * in the table.
 *
 * Tuning table: rom_tune_count / rom_tune_get export the process-wide
 * entries (index order is the key order), rom_tune_put adds or replaces one
 * (its schedule must be one that applies when a run uses it; a run whose
 * table schedule does not apply falls back to COLUMNS4), rom_tune_clear
 * empties the table.  The table is shared by all contexts and threads.
 */
typedef enum {
    ROM_SCHEDULE_COLUMNS4 = 0,
    ROM_SCHEDULE_ROWSPLIT = 1,
    ROM_SCHEDULE_COLUMNS8 = 2,
    ROM_SCHEDULE_RESIDENT = 3,
    ROM_SCHEDULE_PANEL = 4
} rom_schedule;
#define ROM_NSCHEDULES 5

typedef struct {
    int32_t kv_pad, ks_pad; /* Kv, Ks rounded up to multiples of 64           */
    int32_t m_pad;          /* M rounded up to a multiple of 64; 0: grouped
                               per-workgroup tile entry                        */
    rom_dtype op_type;      /* operator type of the shape                      */
    int32_t schedule;       /* rom_schedule chosen                             */
    double us[ROM_NSCHEDULES]; /* per-step time of each schedule (us), < 0 if
                               not applicable or not measured                  */
} rom_tune_entry;

int32_t rom_last_schedule(rom_ctx *ctx);
rom_status rom_schedule_times(rom_ctx *ctx, int32_t M, double us[ROM_NSCHEDULES]);
int32_t rom_tune_count(void);
rom_status rom_tune_get(int32_t i, rom_tune_entry *out);
rom_status rom_tune_put(const rom_tune_entry *e);
void rom_tune_clear(void);

/*
 * Report in-kernel failures of the work enqueued so far: synchronises
 * `stream`, returns ROM_E_TIMEOUT if a row-split run's group barrier ran out
 * of time (its results are then invalid; the kernel still ended), and clears
 * the condition.  ROM_OK otherwise.
 */
rom_status rom_check(rom_ctx *ctx, void *stream);

/*
 * Test hook for the failure handling above (not for production use): with
 * on != 0, every later row-split launch of this process waits at its first
 * group barrier for one arrival more than the group has, with a short poll
 * budget, so the wait runs out, ROM_E_TIMEOUT is recorded and every later
 * wait of that launch returns at once; the kernel ends normally with
 * invalid results.  on = 0 restores normal waits.  Process-wide; returns
 * ROM_OK.
 */
rom_status rom_debug_force_timeout(int32_t on);

/*
 * Test hook for the grouped plans' row-split packing (host logic only; no
 * device work): places n row-split groups of padded K kp[q] (multiples of
 * 64 in [128, 2048]) into cooperative launches of 8 XCDs x 32 workgroups
 * as rom_group_create does (largest K first, each group's K / 64 row tiles
 * on one XCD, first launch with room).  Writes launch[q] and member[q] (the
 * group's launch and its index lg within it) and, per launch l, the slot
 * map slot_maps[256 l + 32 xcd + s] = 32 lg + r (row tile r of member lg
 * in slot s of that XCD) or -1 for an idle slot.  Returns the number of
 * launches, or -1 for an invalid argument or more than max_launches.
 */
int32_t rom_debug_pack_groups(const int32_t *kp, int32_t n, int32_t *launch, int32_t *member,
                              int32_t *slot_maps, int32_t max_launches);

/*
 * End-of-run health check: scans the states V (dev Kv x M) and S (dev Ks x
 * M, the context's state type) for NaN or infinite values (an unstable time
 * step, or non-finite inputs that reached the states) and returns
 * ROM_E_NONFINITE if there is one.  Synchronises `stream`; writes nothing
 * of the caller's.
 */
rom_status rom_check_finite(rom_ctx *ctx, int32_t M, const void *V, const void *S, void *stream);

/*
 * Rank-1 step (Sec. 2.2 eq. (2.3); Sec. 2.3): advance ONE sample by one
 * leapfrog step at t_n = n dt, as two matrix-vector products that re-read
 * the operators from device memory.
 *
 *   v   dev, Kv values of state type (in/out)
 *   s   dev, Ks values of state type (in/out)
 *   n   step index (forcing sampled at n*dt)
 *   mu  Ricker centre frequency of this sample
 *
 * Requires op_type == state_type.  Repeated calls reproduce column m of a
 * rank-2 run to the accuracy of the state type.
 */
rom_status rom_step_rank1(rom_ctx *ctx, void *v, void *s, int64_t n, double mu,
                          void *stream);

/*
 * Rank-1 run: nsteps calls of rom_step_rank1 for one sample, step indices
 * n0 .. n0+nsteps-1, enqueued back to back on `stream` (2 launches per step).
 * The baseline formulation the rank-2 run is compared with.
 */
rom_status rom_run_rank1(rom_ctx *ctx, void *v, void *s, double mu, int64_t n0, int64_t nsteps,
                         void *stream);

/*
 * Rank-1 formulation of M samples in one launch (Sec. 2.2 eq. (2.3); the
 * rank-1 cost model of Sec. 2.3): workgroup m advances sample m through all
 * steps, and every half-step is a matrix-vector product that reads the
 * operator from device memory again, so no operator entry is reused within
 * a step.  The whole chip is busy and there is no launch per step: the
 * memory-bound baseline the rank-2 runs are compared with on this device.
 * V (Kv x M), S (Ks x M), mu (M) as rom_run_rank2; per row the arithmetic
 * of rom_step_rank1 without its split of the reduction over waves (the
 * state is rounded once per half-step).  FP32 states and operators, Kv,
 * Ks <= 1024.  Errors: ROM_E_ARG, ROM_E_UNSUPPORTED, ROM_E_DEVICE.
 */
rom_status rom_run_rank1_batch(rom_ctx *ctx, int32_t M, const double *mu, int64_t n0, int64_t nsteps,
                               void *V, void *S, void *stream);

/*
 * Rank-2 run (Sec. 2.4 eq. (2.5) in the staggered form (3.3)): advance all M
 * samples by `nsteps` leapfrog steps, step indices n0 .. n0+nsteps-1.
 *
 *   M       number of samples (columns), >= 1
 *   mu      dev, M FP64 centre frequencies
 *   V       dev, Kv x M state type, ld = Kv (in/out)
 *   S       dev, Ks x M state type, ld = Ks (in/out)
 *   c       dev, Kv state type probe row, or NULL
 *   J       dev, M FP64, accumulated (+= dt y_m^2 per step), or NULL
 *   y       dev, nsteps x M FP64 probe trace (row k = step n0+k), or NULL
 *
 * J and y require c.  nsteps == 0 is a no-op.  With ROM_F32 states the
 * kernel keeps a compensation term per entry during the run (two-term
 * state) and rounds once when writing back, so splitting a run in two
 * differs from the whole run by at most a rounding of the state.
 * Sizes: FP32 operators and states, and FP64 states, run at any Kv, Ks
 * (the panel schedule where the LDS-resident kernels stop); BF16 / FP8
 * operators with FP32 states within their kernels' LDS limits
 * (ROM_E_UNSUPPORTED above).
 * Errors: ROM_E_ARG, ROM_E_UNSUPPORTED, ROM_E_NOMEM (panel workspace),
 * ROM_E_DEVICE, ROM_E_TIMEOUT.
 */
rom_status rom_run_rank2(rom_ctx *ctx, int32_t M, const double *mu, int64_t n0,
                         int64_t nsteps, void *V, void *S, const void *c, double *J,
                         double *y, void *stream);

/*
 * Allocation-free rank-2 run, for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc during a run): the
 * rank-2 run of rom_run_rank2 on the
 * ROWSPLIT schedule, arguments and results as there (bitwise the same as a
 * rom_run_rank2 that takes ROWSPLIT), without allocating, tuning or
 * synchronising.
 *
 * Its scratch (exchange rows, probe partials, barrier counters) lives in a
 * static device array of 8448 KiB per GPU, held until the process ends and
 * shared by every call on that GPU: calls that overlap on one GPU (several
 * streams, threads or contexts at once) race and give wrong results; calls
 * in stream order are safe (each clears its counters before it runs).  The
 * context's row-split operators are prepared by rom_create.  Requires FP32
 * states, Kv == Ks, a padded K the row-split schedule takes (F32 operators:
 * a multiple of 64 in [128, 2048]; BF16 or F8E4M3: a multiple of 128 in
 * [128, 1024]), the
 * ceil(M / 64) groups of 64 samples in one launch (at most 8 floor(32 /
 * (K / 64))) and a 256-CU gfx950: else ROM_E_UNSUPPORTED,
 * as for a scratch need above the static size (nothing enqueued).  A group
 * barrier that timed out is reported by rom_check.  The launch is
 * cooperative and is not for graph capture.
 * Errors: ROM_E_ARG, ROM_E_UNSUPPORTED, ROM_E_DEVICE.
 */
rom_status rom_run_rank2_noalloc(rom_ctx *ctx, int32_t M, const double *mu, int64_t n0,
                                 int64_t nsteps, void *V, void *S, const void *c, double *J,
                                 double *y, void *stream);

/*
 * Discrete adjoint of a rank-2 run from step 0 for the probe QoI
 *   J = sum_m sum_{n=0}^{N-1} dt (c^T V_m^(n+1))^2
 * (differentiation of the leapfrog, the sensitivity use named in Sec. 5).
 * Reverse sweep with the transposed operators; forward states are rebuilt
 * from checkpoints every `ckpt_stride` steps (0 = ceil(sqrt(nsteps))), or,
 * with ckpt_stride = -1, without checkpoints: by stepping the leapfrog
 * backwards from the final state (it is time-reversible; Sec. 3.1), in
 * segments of ceil(sqrt(nsteps)) steps.  The reversal is exact only in exact
 * arithmetic: the rebuilt states carry the rounding of the forward and
 * backward steps, which grows with N (about 1e-6 relative at N = 5000 in
 * FP32); the checkpoints are the reference.
 *
 *   M, mu, c      as rom_run_rank2 (c required)
 *   nsteps        N >= 1
 *   V0, S0        dev initial states (state type), NULL = zero
 *   J             dev, M FP64 (set, not accumulated)
 *   dAvs          dev, Kv x Ks state type: dJ/dAvs with Asv fixed (set)
 *   dAsv          dev, Ks x Kv state type: dJ/dAsv with Avs fixed (set)
 *   dmu           dev, M FP64: dJ/dmu_m (set)
 * Any of dAvs, dAsv, dmu may be NULL.  dt is held fixed.
 *
 * FP32 states and operators.  The forward sweep runs on the schedule a
 * rom_run_rank2 of the same shape takes; when that is ROWSPLIT the call
 * synchronises `stream` after it and returns ROM_E_TIMEOUT (nothing of the
 * reverse sweep enqueued) if one of its group barriers timed out.  With
 * checkpoints and a ROWSPLIT forward sweep, the recompute and reverse sweep
 * of every segment run on the row-split kernels as well, one after the
 * other on `stream` (the context then also keeps row-split packs of Asv^T
 * and Avs^T, 2 K^2 floats), the call synchronises `stream` at its end and
 * returns ROM_E_TIMEOUT if a group barrier of those sweeps timed out.
 * Otherwise the recompute of the next segment runs on an internal stream
 * beside the reverse sweep on `stream`.  The gradient products of a
 * reversed segment run on a second internal stream; the context keeps the
 * workspace (checkpoints unless ckpt_stride = -1, three sets of state and
 * probe traces, two of W/Q traces: about 0.45 GB at Kv = Ks = 512, M = 256,
 * N = 5000, 0.07 GB less without checkpoints) until rom_destroy.
 */
rom_status rom_adjoint(rom_ctx *ctx, int32_t M, const double *mu, int64_t nsteps,
                       const void *c, const void *V0, const void *S0, double *J,
                       void *dAvs, void *dAsv, double *dmu, int32_t ckpt_stride,
                       void *stream);

/*
 * Seismograms at R receivers and their ensemble statistics (Sec. 4.5: the
 * velocity at a target point is reconstructed from a single row of the
 * velocity basis, and the ensemble over the forcing parameter is summarised
 * by its mean and percentile bounds).  Advances all M samples by `nsteps`
 * steps from step n0 like rom_run_rank2 and records, for every step n and
 * receiver r,
 *   Y[n][r][m] = C[r] . V_m after step n0 + n
 * and over the M samples: mean, population variance (1/M) and the
 * nearest-rank 5th, 50th and 95th percentiles (the ceil(p M / 100)-th
 * smallest value).
 *
 *   M        samples, 1 .. 1024
 *   mu, V, S as rom_run_rank2 (V, S updated in place)
 *   R        receivers, 1 .. 64, with R x M <= 8192
 *   C        dev, R x Kv row-major state type (FP32): one receiver row each
 *   Y        dev, nsteps x R x M FP64 seismograms, or NULL
 *   stats    dev, nsteps x R x 5 FP64 (mean, variance, p5, p50, p95), or
 *            NULL
 *
 * FP32 states and operators only, on the 4-column column-block schedule.
 * The run is stepped in chunks whose state traces stay in device memory
 * (up to 2 x 256 MiB of workspace, kept by the context); the seismograms and
 * statistics of a chunk are computed on an internal stream while the next
 * chunk steps.  Chunk boundaries round the state once, as a split
 * rom_run_rank2 does.  Errors: ROM_E_ARG, ROM_E_UNSUPPORTED (sizes above),
 * ROM_E_NOMEM, ROM_E_DEVICE.
 */
rom_status rom_run_receivers(rom_ctx *ctx, int32_t M, const double *mu, int64_t n0, int64_t nsteps,
                             void *V, void *S, int32_t R, const void *C, double *Y, double *stats,
                             void *stream);

/*
 * Grouped run: G independent ROM instances (each its own context, sizes and
 * samples) advanced `nsteps` steps from step 0 together — the batched
 * direction the paper names for many operator realisations (Sec. 5).  On
 * the column-block plan it is ONE launch whose work items are (instance,
 * column block of 4 or 8 samples: see the tile autotuner above) pairs,
 * dispatched longest tuned step time first; instances of one square K may
 * run on the row-split plan instead (below).  All contexts must have F32
 * states and operators, within the LDS-resident size limit.  Per instance
 * i: M[i] samples, mu[i] dev FP64, V[i] / S[i] dev states as in
 * rom_run_rank2 (host arrays of pointers).  Each instance's result is
 * bitwise identical to its own rom_run_rank2 on the plan's schedule
 * (column blocks, or row-split).
 * The call builds a plan (below), runs it and synchronises `stream`
 * before releasing the plan; use the plan API for asynchronous or
 * graph-captured runs.
 */
rom_status rom_run_grouped(rom_ctx *const *ctx, int32_t G, const int32_t *M,
                           const double *const *mu, int64_t nsteps, void *const *V,
                           void *const *S, void *stream);

/*
 * Grouped plan: the validated descriptor table of a grouped run, uploaded
 * once (synchronously) by rom_group_create.  rom_group_run is then a single
 * kernel launch with no host-side data (so it can be captured in a HIP
 * graph and replayed); it advances every instance over steps
 * n0 .. n0+nsteps-1.  The plan stores the caller's device pointers, which
 * must stay valid while the plan is used.  Contexts must outlive the plan.
 */
typedef struct rom_group rom_group;
rom_status rom_group_create(rom_ctx *const *ctx, int32_t G, const int32_t *M,
                            const double *const *mu, void *const *V, void *const *S,
                            rom_group **out);
rom_status rom_group_run(rom_group *g, int64_t n0, int64_t nsteps, void *stream);
rom_status rom_group_destroy(rom_group *g);

/*
 * Row-split grouped plan.  Instances that are square (Kv == Ks) with FP32
 * operators and a padded K the row-split schedule takes (a multiple of 64
 * in [128, 2048]), and that are not pinned to column blocks
 * (ROM_SCHED_COLUMNS / ROM_SCHED_COLUMNS8), can instead run as the
 * row-split schedule of rom_run_rank2 runs one instance: samples in groups
 * of 64, the operator rows of a group over K / 64 workgroups of one XCD.
 * A plan puts the eligible instances from a padded-K threshold up on
 * row-split: their groups, largest K first, fill cooperative launches (8
 * XCDs x 32 workgroups each, groups of different K side by side), run one
 * after another, followed by one column-block launch over the other
 * instances.  Each instance's result is bitwise identical to its own
 * rom_run_rank2 on the schedule it ran on.  Which threshold: the smallest
 * eligible K if every context has ROM_SCHED_ROWSPLIT, else the fastest of
 * "none" (column blocks only) and each eligible padded K, timed once per
 * shape (the instances' padded K and M) on scratch states when the plan is
 * made (rom_group_create: on the default stream; rom_run_grouped: on
 * `stream`) and remembered for the process.  A plan keeps the all-column
 * form too: a run enqueued on a stream that is being captured into a graph
 * uses it.  Making such a plan also packs each eligible context's row-split
 * operators (2 K^2 floats per context, kept by it).
 *
 * rom_group_schedule: ROM_SCHEDULE_ROWSPLIT (a plan with a row-split
 *   part) or ROM_SCHEDULE_COLUMNS4 (column blocks only, whatever tiles its
 *   instances take); -1 for NULL.
 * rom_group_times: per-step microseconds of the column-block plan (us[0])
 *   and of the fastest plan with a row-split part (us[1]) if this plan
 *   timed them, else negative.
 * rom_group_split_k: the smallest padded K of the instances on the plan's
 *   row-split part (every eligible instance with at least that padded K
 *   runs there), 0 for a column-block plan, -1 for NULL.
 * rom_group_check: as rom_check, for the row-split plan's group barriers
 *   (synchronises `stream`).  rom_run_grouped synchronises `stream` after
 *   its run and returns ROM_E_TIMEOUT itself.
 */
int32_t rom_group_schedule(const rom_group *g);
rom_status rom_group_times(const rom_group *g, double us[2]);
int32_t rom_group_split_k(const rom_group *g);
rom_status rom_group_check(rom_group *g, void *stream);

/*
 * Affine operator families (the rank-3 direction of Sec. 5: many operator
 * parameters at once).  Operators that depend affinely on parameters,
 *   Avs(theta) = sum_q theta_q Avs_q,   Asv(theta) = sum_q theta_q Asv_q,
 * are kept as their Q terms on the device; each parameter point becomes an
 * ordinary context whose operators are assembled on the device in FP64
 * (terms added in order q = 0, 1, ..., each product and sum rounded once)
 * and then rounded and packed exactly as rom_create does with host
 * operators.  All instances of a family run together in one grouped launch
 * (rom_run_grouped / rom_group_create) or alone.
 *
 * rom_affine_create:
 *   cfg      as rom_create (its dt is the instances' default)
 *   Q        terms, 1 .. 16
 *   Avs_q    host, Q consecutive Kv x Ks column-major FP64 matrices
 *   Asv_q    host, Q consecutive Ks x Kv column-major FP64 matrices
 *   b        host, Kv FP64 (shared source)
 *   stream   for the uploads (synchronised before return)
 * rom_affine_instance:
 *   theta    host, Q FP64 coefficients
 *   dt       > 0, or 0 for the family's dt
 *   out      the new context (destroy with rom_destroy); the call
 *            synchronises `stream`.  With ROM_SKEW_CHECK and skew terms the
 *            assembled Avs is checked as in rom_create (ROM_E_UNSTABLE).
 * Instances own their operators: a family may be destroyed while its
 * instances are still in use.  Host arrays may be freed on return.
 * Errors: ROM_E_ARG (NULL pointer, Q outside 1..16, cfg rejected as by
 * rom_create, dt negative or non-finite), ROM_E_NONFINITE (NaN/Inf in the
 * terms, b or theta), ROM_E_UNSTABLE, ROM_E_NOMEM, ROM_E_DEVICE; *out is
 * NULL on any error.  rom_affine_destroy(NULL) is a no-op.
 */
typedef struct rom_affine rom_affine;
rom_status rom_affine_create(const rom_config *cfg, int32_t Q, const double *Avs_q, const double *Asv_q,
                             const double *b, void *stream, rom_affine **out);
rom_status rom_affine_instance(rom_affine *A, const double *theta, double dt, void *stream, rom_ctx **out);
rom_status rom_affine_destroy(rom_affine *A);

/*
 * Full-order model (FOM) and the offline stage (NEXT to the ROM path).
 *
 * The rank-2 FOM of the staggered system (Sec. 3, eq. (3.2)):
 *   dV/dt = Av S + f u(t; mu)^T,   dS/dt = As V,
 * with sparse Av (Nv x Ns) and As (Ns x Nv), stepped by the ROM's leapfrog
 * (V first, then S with the new V; forcing at t_n = n dt).  FOM states are
 * ROW-major, unlike ROM states: element (r, m) of an N x M state is at
 * [r*M + m] (one degree of freedom's M samples contiguous).  FP64 only.
 *
 * rom_fom_create:
 *   Nv, Ns          sizes of the velocity and stress spaces
 *   av_ptr/col/val  host CSR of Av: row pointers (Nv + 1, starting at 0,
 *                   non-decreasing), column indices (< Ns), FP64 values
 *   as_ptr/col/val  host CSR of As (Ns rows, columns < Nv)
 *   f               host, Nv FP64 source vector (the point source e_src / rho
 *                   of Sec. 3.2; any vector is accepted)
 *   dt              time step (> 0)
 *   flags           0 (Ricker source) or ROM_SOURCE_GAUSS1
 *   The arrays are copied (and the call synchronises `stream`); the host
 *   arrays may be freed on return.  Errors: ROM_E_ARG (NULL, bad sizes, bad
 *   CSR structure), ROM_E_NONFINITE, ROM_E_NOMEM, ROM_E_DEVICE.
 * rom_fom_run: nsteps steps from step n0 of M samples: mu dev M FP64, V dev
 *   Nv x M and S dev Ns x M FP64 row-major, updated in place.  Two kernel
 *   launches per step, enqueued on `stream`.
 * rom_fom_project: the Galerkin ROM operators of orthonormal bases
 *   (Sec. 2.2, eq. (3.3)): Avs = Phi_v^T Av Phi_s (dev Kv x Ks, column-major:
 *   the rom_create layout), Asv = Phi_s^T As Phi_v (dev Ks x Kv), b =
 *   Phi_v^T f (dev Kv).  phi_v: dev Nv x Kv and phi_s: dev Ns x Ks, ROW-major
 *   (the layout rom_pod writes).  Enqueued on `stream` (stream-ordered
 *   scratch of (Nv Ks + Ns Kv) doubles plus split partials).
 * rom_fom_destroy(NULL) is a no-op.
 */
typedef struct rom_fom rom_fom;
rom_status rom_fom_create(int32_t nv, int32_t ns, const int32_t *av_ptr, const int32_t *av_col,
                          const double *av_val, const int32_t *as_ptr, const int32_t *as_col,
                          const double *as_val, const double *f, double dt, uint32_t flags,
                          void *stream, rom_fom **out);
rom_status rom_fom_run(rom_fom *F, int32_t M, const double *mu, int64_t n0, int64_t nsteps,
                       double *V, double *S, void *stream);
rom_status rom_fom_project(rom_fom *F, int32_t kv, int32_t ks, const double *phi_v,
                           const double *phi_s, double *Avs, double *Asv, double *b, void *stream);
rom_status rom_fom_destroy(rom_fom *F);

/*
 * POD of a snapshot matrix (Sec. 4.4): the leading left singular vectors of
 * X (dev n x ns FP64, ROW-major, one snapshot per column, n >= ns,
 * ns <= 2048), kept to k columns: with tol >= 0 the smallest k whose
 * singular values hold at least (1 - tol) of sum sigma_i^2, capped at kmax;
 * with tol < 0, k = kmax (capped at the number of nonzero sigma).
 *   phi     dev n x kmax FP64 ROW-major out: columns 0 .. k-1 the modes
 *           (orthonormal), the rest zero
 *   sigma   host ns FP64 out: all singular values, descending
 *   k       host out: the number of modes kept
 * Method: the Gram matrix X^T X (device) and its eigen-decomposition (host
 * Jacobi) give the numerical rank r (eigenvalues above 100 ns u l_1, so
 * modes with sigma_i / sigma_1 below about 1e-6 / sqrt(ns / 100) are never
 * kept) and V_r; Y = X V_r is orthonormalised by two Cholesky QR passes
 * (device products, host factors) into Q; the SVD of Q^T X (host Jacobi)
 * gives sigma_0 .. sigma_{r-1} and the modes Q U (device).  sigma_i for
 * i >= r is the square root of the Gram eigenvalue (inaccurate, and below
 * the rank threshold).  The host Jacobi solves use up to 16 threads (about
 * 0.05 s at ns = 256, 3 s at ns = 1024).  Synchronises `stream`; allocates
 * 2 n ns + 2 ns^2 doubles plus split partials for the call.  Errors: ROM_E_ARG,
 * ROM_E_NONFINITE (zero or non-finite X), ROM_E_UNSUPPORTED (the Cholesky
 * QR of the dominant subspace failed), ROM_E_NOMEM, ROM_E_DEVICE.
 */
rom_status rom_pod(int64_t n, int32_t ns, const double *X, double tol, int32_t kmax, double *phi,
                   double *sigma, int32_t *k, void *stream);

/*
 * Thread-local text describing the last non-OK status of this thread
 * (library housekeeping: no passage of the paper defines it).  The pointer
 * stays valid until the thread's next library call; never NULL.
 */
const char *rom_last_error(void);

/* Library version string. */
const char *rom_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ROM_H */
