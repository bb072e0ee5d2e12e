/*
 * FP64 CPU oracle for the rank-2 Galerkin ROM of a staggered LTI system.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or helper with the HIP library.
 *
 * What is computed (paper: Sec. 3.1, eq. (3.3), leapfrog paragraph after it;
 * rank-2 form eq. (2.5)):
 *
 *   dV/dt = Avs S + b u(t; mu)^T        (velocity, forced)
 *   dS/dt = Asv V                       (stress)
 *
 * with V (Kv x M) and S (Ks x M) holding one sample per column, Avs (Kv x Ks),
 * Asv (Ks x Kv) the two reduced operators, b the reduced point source (the
 * sparse-forcing case of Sec. 2.2) and u a Ricker wavelet whose parameter mu_m
 * (centre frequency) differs per sample (the forcing-only parameter split of
 * Sec. 2).  The integrator is leapfrog, velocity first then stress, from the
 * caller's initial state (zero in the paper).  Discrete form used (the paper
 * does not print one; this is the reading documented with the library):
 *
 *   for n = n0 .. n0+nsteps-1, t_n = n*dt:
 *     V <- V + dt * (Avs S + b u(t_n)^T)
 *     S <- S + dt * (Asv V)              (the freshly updated V)
 *     optional probe: y_m = c^T V[:,m],  J_m += dt * y_m^2
 *
 * Ricker wavelet (Sec. 3.2 names it, with the period as its parameter; no
 * formula is given): unit-peak form u = (1 - 2a) exp(-a), a = pi^2 (mu t - 1.5)^2,
 * i.e. centre frequency mu = 1/T and delay 1.5/mu.
 *
 * All storage is column-major: element (i, j) of an R x C matrix is at
 * [i + j*R].  Every sum runs over its index in increasing order, multiply and
 * add kept separate (build with -ffp-contract=off), so the rank-1 routine and
 * each column of the rank-2 routine produce bitwise identical numbers.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---- forcing (Sec. 3.2): Ricker wavelet and its mu-derivative ---------- */

double orc_ricker(double t, double mu)
{
    double x = M_PI * (mu * t - 1.5);
    double a = x * x;
    return (1.0 - 2.0 * a) * exp(-a);
}

/* d u / d mu, including the mu-dependence of the 1.5/mu delay:
 * a = pi^2 (mu t - 1.5)^2, da/dmu = 2 pi^2 t (mu t - 1.5), du/da = (2a - 3) e^-a */
double orc_ricker_dmu(double t, double mu)
{
    double x = mu * t - 1.5;
    double a = M_PI * M_PI * x * x;
    return (2.0 * a - 3.0) * exp(-a) * (2.0 * M_PI * M_PI * t * x);
}

/* The paper's second signal (Sec. 3.2; the source of its FOM scaling runs,
 * Appendix A): the first derivative of a Gaussian, no formula given.  Read
 * here with the period T = 1/mu and the delay 3T of Appendix A, unit peak:
 *   u = -sqrt(2e) x exp(-x^2),   x = pi (mu t - 3)
 * (the time derivative of exp(-x^2), scaled so that max |u| = 1). */
double orc_gauss1(double t, double mu)
{
    double x = M_PI * (mu * t - 3.0);
    return -sqrt(2.0 * exp(1.0)) * x * exp(-x * x);
}

/* d u / d mu of the above (the delay 3/mu moves with mu): dx/dmu = pi t */
double orc_gauss1_dmu(double t, double mu)
{
    double x = M_PI * (mu * t - 3.0);
    return -sqrt(2.0 * exp(1.0)) * (1.0 - 2.0 * x * x) * exp(-x * x) * (M_PI * t);
}

/* Signal of source kind src (0: Ricker, 1: Gaussian derivative). */
static double src_u(int src, double t, double mu)
{
    return src == 1 ? orc_gauss1(t, mu) : orc_ricker(t, mu);
}

static double src_dmu(int src, double t, double mu)
{
    return src == 1 ? orc_gauss1_dmu(t, mu) : orc_ricker_dmu(t, mu);
}

/* ---- rank-1 (Sec. 2.2 eq. (2.3), M = 1): one trajectory, two GEMVs ------- */

/* One leapfrog step at t_n = n*dt for a single sample. v (Kv), s (Ks) in/out. */
void orc_step_rank1(int kv, int ks, const double *Avs, const double *Asv,
                    const double *b, double dt, int64_t n, double mu,
                    double *v, double *s, int src)
{
    double u = src_u(src, (double)n * dt, mu);
    for (int i = 0; i < kv; ++i) {
        double r = 0.0;
        for (int j = 0; j < ks; ++j) r = r + Avs[i + (int64_t)j * kv] * s[j];
        v[i] = v[i] + dt * (r + b[i] * u);
    }
    for (int i = 0; i < ks; ++i) {
        double r = 0.0;
        for (int j = 0; j < kv; ++j) r = r + Asv[i + (int64_t)j * ks] * v[j];
        s[i] = s[i] + dt * r;
    }
}

/* ---- rank-2 (Sec. 2.4 eq. (2.5) in the staggered form (3.3)) ------------- */

/* One leapfrog step of all M columns, written as matrix products.
 * R is scratch of max(Kv, Ks) * M doubles. */
static void rank2_step(int kv, int ks, const double *Avs, const double *Asv,
                       const double *b, double dt, int M, const double *mu,
                       int64_t n, double *V, double *S, double *R, int src)
{
    double t = (double)n * dt;
    /* R = Avs * S  (Kv x M) */
    #pragma omp parallel for schedule(static)
    for (int m = 0; m < M; ++m) {
        for (int i = 0; i < kv; ++i) {
            double r = 0.0;
            for (int j = 0; j < ks; ++j)
                r = r + Avs[i + (int64_t)j * kv] * S[j + (int64_t)m * ks];
            R[i + (int64_t)m * kv] = r;
        }
        double u = src_u(src, t, mu[m]);
        for (int i = 0; i < kv; ++i)
            V[i + (int64_t)m * kv] = V[i + (int64_t)m * kv] + dt * (R[i + (int64_t)m * kv] + b[i] * u);
    }
    /* R = Asv * V_new  (Ks x M) */
    #pragma omp parallel for schedule(static)
    for (int m = 0; m < M; ++m) {
        for (int i = 0; i < ks; ++i) {
            double r = 0.0;
            for (int j = 0; j < kv; ++j)
                r = r + Asv[i + (int64_t)j * ks] * V[j + (int64_t)m * kv];
            R[i + (int64_t)m * ks] = r;
        }
        for (int i = 0; i < ks; ++i)
            S[i + (int64_t)m * ks] = S[i + (int64_t)m * ks] + dt * R[i + (int64_t)m * ks];
    }
}

/* y_m = c^T V[:, m] */
static void probe(int kv, int M, const double *c, const double *V, double *y)
{
    for (int m = 0; m < M; ++m) {
        double acc = 0.0;
        for (int i = 0; i < kv; ++i) acc = acc + c[i] * V[i + (int64_t)m * kv];
        y[m] = acc;
    }
}

/*
 * Integrate nsteps leapfrog steps starting at step index n0 for M samples.
 * V (Kv x M), S (Ks x M) in/out.  c (Kv) optional probe; J (M) accumulated
 * (+= dt * y^2 per step) when c and J are given; ytrace (nsteps x M, row n is
 * step n0+n) receives y when given.  Returns 0, or -1 on allocation failure.
 */
int orc_run_rank2(int kv, int ks, const double *Avs, const double *Asv,
                  const double *b, double dt, int M, const double *mu,
                  int64_t n0, int64_t nsteps, double *V, double *S,
                  const double *c, double *J, double *ytrace, int src)
{
    int kmax = kv > ks ? kv : ks;
    double *R = (double *)malloc(sizeof(double) * (size_t)kmax * (size_t)(M > 0 ? M : 1));
    double *y = (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
    if (!R || !y) { free(R); free(y); return -1; }
    for (int64_t k = 0; k < nsteps; ++k) {
        int64_t n = n0 + k;
        rank2_step(kv, ks, Avs, Asv, b, dt, M, mu, n, V, S, R, src);
        if (c) {
            probe(kv, M, c, V, y);
            for (int m = 0; m < M; ++m) {
                if (J) J[m] = J[m] + dt * (y[m] * y[m]);
                if (ytrace) ytrace[k * M + m] = y[m];
            }
        }
    }
    free(R);
    free(y);
    return 0;
}

/* Modified discrete energy per column: E = |v|^2 + |s|^2 + dt v^T Avs s.
 * For Asv = -Avs^T it is conserved by the unforced step (derivation in the
 * design notes); E (M) out. */
void orc_energy(int kv, int ks, const double *Avs, double dt, int M,
                const double *V, const double *S, double *E)
{
    for (int m = 0; m < M; ++m) {
        const double *v = V + (int64_t)m * kv;
        const double *s = S + (int64_t)m * ks;
        double vv = 0.0, ss = 0.0, vas = 0.0;
        for (int i = 0; i < kv; ++i) vv = vv + v[i] * v[i];
        for (int j = 0; j < ks; ++j) ss = ss + s[j] * s[j];
        for (int i = 0; i < kv; ++i) {
            double r = 0.0;
            for (int j = 0; j < ks; ++j) r = r + Avs[i + (int64_t)j * kv] * s[j];
            vas = vas + v[i] * r;
        }
        E[m] = vv + ss + dt * vas;
    }
}

/*
 * Discrete adjoint of the loop above for the probe QoI
 *   J = sum_m sum_{n=0}^{N-1} dt (c^T V_m^{(n+1)})^2,
 * starting at step 0 from (V0, S0) (NULL = zero).  Reverse-mode
 * differentiation of each forward statement, in reverse order:
 *
 *   p, q = 0
 *   for n = N-1 .. 0 (V+ = V after step n, S- = S before step n):
 *     dAsv += dt q V+^T
 *     w     = p + 2 dt (c^T V+) c + dt Asv^T q
 *     dAvs += dt w S-^T
 *     dmu_m += dt (b^T w_m) du/dmu(t_n; mu_m)
 *     p = w ;  q = q + dt Avs^T w
 *
 * Forward states come from checkpoints every `stride` steps (stride <= 0
 * selects ceil(sqrt(N))) with the segment recomputed by the same forward
 * step, so the result does not depend on the stride.  Outputs: J (M, set),
 * dAvs (Kv x Ks, set), dAsv (Ks x Kv, set), dmu (M, set).  Gradients are
 * partial derivatives with the other operator and dt held fixed.
 * Returns 0, or -1 on allocation failure / bad arguments.
 */
int orc_adjoint(int kv, int ks, const double *Avs, const double *Asv,
                const double *b, double dt, int M, const double *mu,
                int64_t nsteps, const double *c, const double *V0,
                const double *S0, double *J, double *dAvs, double *dAsv,
                double *dmu, int64_t stride, int src)
{
    if (nsteps < 0 || M < 0 || kv <= 0 || ks <= 0) return -1;
    if (stride <= 0) {
        stride = (int64_t)ceil(sqrt((double)(nsteps > 0 ? nsteps : 1)));
        if (stride < 1) stride = 1;
    }
    int64_t nseg = nsteps > 0 ? (nsteps + stride - 1) / stride : 0;
    size_t vsz = (size_t)kv * (size_t)M, ssz = (size_t)ks * (size_t)M;
    int kmax = kv > ks ? kv : ks;
    /* checkpoints: state before the first step of each segment */
    double *ckV = (double *)calloc((size_t)(nseg > 0 ? nseg : 1) * vsz + 1, sizeof(double));
    double *ckS = (double *)calloc((size_t)(nseg > 0 ? nseg : 1) * ssz + 1, sizeof(double));
    /* segment buffer: states 0..stride (stride+1 snapshots) */
    double *segV = (double *)calloc((size_t)(stride + 1) * vsz + 1, sizeof(double));
    double *segS = (double *)calloc((size_t)(stride + 1) * ssz + 1, sizeof(double));
    double *R = (double *)calloc((size_t)kmax * (size_t)(M > 0 ? M : 1) + 1, sizeof(double));
    double *V = (double *)calloc(vsz + 1, sizeof(double));
    double *S = (double *)calloc(ssz + 1, sizeof(double));
    double *P = (double *)calloc(vsz + 1, sizeof(double));
    double *Q = (double *)calloc(ssz + 1, sizeof(double));
    double *W = (double *)calloc(vsz + 1, sizeof(double));
    double *y = (double *)calloc((size_t)(M > 0 ? M : 1), sizeof(double));
    int rc = 0;
    if (!ckV || !ckS || !segV || !segS || !R || !V || !S || !P || !Q || !W || !y) { rc = -1; goto done; }

    if (V0) memcpy(V, V0, vsz * sizeof(double));
    if (S0) memcpy(S, S0, ssz * sizeof(double));
    for (int m = 0; m < M; ++m) { J[m] = 0.0; dmu[m] = 0.0; }
    memset(dAvs, 0, sizeof(double) * (size_t)kv * ks);
    memset(dAsv, 0, sizeof(double) * (size_t)ks * kv);

    /* forward sweep: store checkpoints, accumulate J */
    for (int64_t n = 0; n < nsteps; ++n) {
        if (n % stride == 0) {
            memcpy(ckV + (size_t)(n / stride) * vsz, V, vsz * sizeof(double));
            memcpy(ckS + (size_t)(n / stride) * ssz, S, ssz * sizeof(double));
        }
        rank2_step(kv, ks, Avs, Asv, b, dt, M, mu, n, V, S, R, src);
        probe(kv, M, c, V, y);
        for (int m = 0; m < M; ++m) J[m] = J[m] + dt * (y[m] * y[m]);
    }

    /* reverse sweep, one segment at a time from the last */
    for (int64_t g = nseg - 1; g >= 0; --g) {
        int64_t nb = g * stride;
        int64_t ne = nb + stride < nsteps ? nb + stride : nsteps;
        int64_t len = ne - nb;
        memcpy(segV, ckV + (size_t)g * vsz, vsz * sizeof(double));
        memcpy(segS, ckS + (size_t)g * ssz, ssz * sizeof(double));
        memcpy(V, segV, vsz * sizeof(double));
        memcpy(S, segS, ssz * sizeof(double));
        for (int64_t k = 0; k < len; ++k) {
            rank2_step(kv, ks, Avs, Asv, b, dt, M, mu, nb + k, V, S, R, src);
            memcpy(segV + (size_t)(k + 1) * vsz, V, vsz * sizeof(double));
            memcpy(segS + (size_t)(k + 1) * ssz, S, ssz * sizeof(double));
        }
        for (int64_t k = len - 1; k >= 0; --k) {
            int64_t n = nb + k;
            double t = (double)n * dt;
            const double *Vp = segV + (size_t)(k + 1) * vsz; /* V after step n  */
            const double *Sm = segS + (size_t)k * ssz;       /* S before step n */
            /* dAsv += dt * Q * Vp^T  (entry-parallel, sum over m in order) */
            #pragma omp parallel for schedule(static)
            for (int j = 0; j < kv; ++j)
                for (int i = 0; i < ks; ++i) {
                    double acc = 0.0;
                    for (int m = 0; m < M; ++m)
                        acc = acc + Q[i + (int64_t)m * ks] * Vp[j + (int64_t)m * kv];
                    dAsv[i + (int64_t)j * ks] = dAsv[i + (int64_t)j * ks] + dt * acc;
                }
            /* W = P + 2 dt (c^T Vp) c + dt Asv^T Q */
            #pragma omp parallel for schedule(static)
            for (int m = 0; m < M; ++m) {
                double yv = 0.0;
                for (int i = 0; i < kv; ++i) yv = yv + c[i] * Vp[i + (int64_t)m * kv];
                for (int i = 0; i < kv; ++i) {
                    double r = 0.0;
                    for (int j = 0; j < ks; ++j)
                        r = r + Asv[j + (int64_t)i * ks] * Q[j + (int64_t)m * ks];
                    W[i + (int64_t)m * kv] = P[i + (int64_t)m * kv] + 2.0 * dt * yv * c[i] + dt * r;
                }
            }
            /* dAvs += dt * W * Sm^T */
            #pragma omp parallel for schedule(static)
            for (int j = 0; j < ks; ++j)
                for (int i = 0; i < kv; ++i) {
                    double acc = 0.0;
                    for (int m = 0; m < M; ++m)
                        acc = acc + W[i + (int64_t)m * kv] * Sm[j + (int64_t)m * ks];
                    dAvs[i + (int64_t)j * kv] = dAvs[i + (int64_t)j * kv] + dt * acc;
                }
            /* dmu, P <- W, Q <- Q + dt Avs^T W */
            #pragma omp parallel for schedule(static)
            for (int m = 0; m < M; ++m) {
                double bw = 0.0;
                for (int i = 0; i < kv; ++i) bw = bw + b[i] * W[i + (int64_t)m * kv];
                dmu[m] = dmu[m] + dt * bw * src_dmu(src, t, mu[m]);
                for (int i = 0; i < kv; ++i) P[i + (int64_t)m * kv] = W[i + (int64_t)m * kv];
                for (int j = 0; j < ks; ++j) {
                    double r = 0.0;
                    for (int i = 0; i < kv; ++i)
                        r = r + Avs[i + (int64_t)j * kv] * W[i + (int64_t)m * kv];
                    Q[j + (int64_t)m * ks] = Q[j + (int64_t)m * ks] + dt * r;
                }
            }
        }
    }
done:
    free(ckV); free(ckS); free(segV); free(segS); free(R);
    free(V); free(S); free(P); free(Q); free(W); free(y);
    return rc;
}

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- operator rounding for the low-precision runs ------------------------
 * The low-precision operator GEMMs see rounded operators; the "same-input"
 * oracle steps with exactly those rounded values (in FP64).  Both roundings
 * go through FP32 first (the library's input precision), round to nearest
 * with ties to even, and are pinned in the tests against torch's CPU casts. */

#include <float.h>

/* x -> FP32 -> bfloat16 (8-bit mantissa incl. hidden bit), RNE, returned as double */
double orc_round_bf16(double x)
{
    float f = (float)x;
    if (f != f) return (double)f;
    if (f == 0.0f || isinf(f)) return (double)f;
    int e;
    frexpf(f, &e);                 /* f = fr * 2^e, 0.5 <= |fr| < 1 */
    /* spacing of bf16 numbers in [2^(e-1), 2^e) is 2^(e-8); below the normal
     * range (e-1 < -126) the spacing stays at 2^-133 */
    int qexp = (e - 1 < -126 ? -126 : e - 1) - 7;
    double q = ldexp(1.0, qexp);
    double r = nearbyint((double)f / q) * q;   /* exact division by a power of two */
    return r;
}

/* One value -> OCP FP8 E4M3 ("fn": no infinities, max 448), RNE, saturating.
 * Input and output in FP32 value space (the result is exactly representable). */
static float e4m3_rne_sat(float f)
{
    if (f != f) return f;
    float a = fabsf(f);
    if (a > 448.0f) a = 448.0f;
    if (a == 0.0f) return f;       /* keep signed zero */
    int e;
    frexpf(a, &e);                 /* a in [2^(e-1), 2^e) */
    int qexp = (e - 1 < -6 ? -6 : e - 1) - 3;   /* 3 mantissa bits; subnormal quantum 2^-9 */
    double q = ldexp(1.0, qexp);
    double r = nearbyint((double)a / q) * q;
    if (r > 448.0) r = 448.0;
    return (float)(f < 0 ? -r : r);
}

/* Per-tensor scaled FP8 E4M3 quantisation of n values (any layout):
 * x32 = fp32(x), scale = fp32(amax(|x32|) / 448) computed in FP32,
 * q = e4m3(x32 / scale) (FP32 division, RNE, saturate to +-448),
 * out = q * scale evaluated in FP64 (exact).  `amax_in` > 0 overrides the
 * tensor's own amax (to share one scale between two tensors).
 * Returns the scale. */
double orc_quantize_e4m3(int64_t n, const double *x, double *out, double amax_in)
{
    float amax = 0.0f;
    if (amax_in > 0.0) amax = (float)amax_in;
    else
        for (int64_t i = 0; i < n; ++i) {
            float a = fabsf((float)x[i]);
            if (a > amax) amax = a;
        }
    if (amax == 0.0f) {
        for (int64_t i = 0; i < n; ++i) out[i] = 0.0;
        return 1.0;
    }
    float scale = amax / 448.0f;
    for (int64_t i = 0; i < n; ++i) {
        float q = e4m3_rne_sat((float)x[i] / scale);
        out[i] = (double)q * (double)scale;
    }
    return (double)scale;
}

/* ---- full-order model (FOM) ---------------------------------------------
 * The rank-2 FOM of the staggered shear-wave system (Sec. 3, eq. (3.2)):
 *
 *   dV/dt = Av S + f u(t; mu)^T,    dS/dt = As V
 *
 * with sparse Av (Nv x Ns) and As (Ns x Nv) in CSR form (row pointers,
 * column indices, values; the entries of a row in the stored order), f the
 * (sparse) point-source vector and the same leapfrog as the ROM: for
 * n = n0 .. n0+nsteps-1, t_n = n dt,
 *
 *   V[r, m] <- V[r, m] + dt * ((sum_k Av[r, k] S[k, m]) + f[r] u_m(t_n))
 *   S[r, m] <- S[r, m] + dt * (sum_k As[r, k] V[k, m])     (the new V)
 *
 * States are row-major here (element (r, m) at [r*M + m], the layout of the
 * paper's rank-2 FOM runs), sums in the stored entry order. */
static void csr_update(int nrows, const int *ptr, const int *col, const double *val,
                       const double *X, int M, const double *f, const double *u, double dt, double *Y)
{
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < nrows; ++r)
        for (int m = 0; m < M; ++m) {
            double inc = 0.0;
            for (int k = ptr[r]; k < ptr[r + 1]; ++k) inc = inc + val[k] * X[(int64_t)col[k] * M + m];
            if (f) inc = inc + f[r] * u[m];
            Y[(int64_t)r * M + m] = Y[(int64_t)r * M + m] + dt * inc;
        }
}

int orc_fom_run(int nv, int ns, const int *avp, const int *avc, const double *avv,
                const int *asp, const int *asc, const double *asv, const double *f,
                double dt, int M, const double *mu, int64_t n0, int64_t nsteps,
                double *V, double *S, int src)
{
    double *u = (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
    if (!u) return 1;
    for (int64_t k = 0; k < nsteps; ++k) {
        const double t = (double)(n0 + k) * dt;
        for (int m = 0; m < M; ++m) u[m] = src_u(src, t, mu[m]);
        csr_update(nv, avp, avc, avv, S, M, f, u, dt, V);
        csr_update(ns, asp, asc, asv, V, M, NULL, u, dt, S);
    }
    free(u);
    return 0;
}
