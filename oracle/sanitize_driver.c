/*
 * Test infrastructure: a driver that runs every function of the FP64 oracle
 * (rom_oracle.c, compiled into this executable) on small inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer.  It checks a
 * few identities the oracle must satisfy (column-by-column equality of the
 * rank-1 step and the rank-2 run, independence of the adjoint from the
 * checkpoint stride, finite results) and returns nonzero on a mismatch;
 * the sanitizers abort on any out-of-bounds access, use after free, leak
 * or undefined operation.  Edge cases: Kv != Ks, M = 1, nsteps = 0, a
 * stride longer than the run, an empty CSR row.
 */
#include "rom_oracle.c"

#include <stdio.h>

static unsigned long long g_state = 88172645463325252ULL;

/* xorshift64 uniform in [-1, 1): input values only */
static double draw(void) {
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) / 4503599627370496.0 - 1.0;
}

static double *fill(size_t n, double scale) {
    double *x = (double *)malloc(sizeof(double) * (n ? n : 1));
    for (size_t i = 0; i < n; ++i) x[i] = scale * draw();
    return x;
}

static int check_run(int kv, int ks, int M, int64_t nsteps) {
    int bad = 0;
    double *A = fill((size_t)kv * ks, 0.3), *B = fill((size_t)ks * kv, 0.3), *b = fill(kv, 1.0);
    double *c = fill(kv, 1.0), *mu = (double *)malloc(sizeof(double) * M);
    for (int m = 0; m < M; ++m) mu[m] = 0.5 + 0.5 * (draw() + 1.0) / 2.0;
    double *V = (double *)calloc((size_t)kv * M, sizeof(double)), *S = (double *)calloc((size_t)ks * M, sizeof(double));
    double *J = (double *)calloc(M, sizeof(double)), *y = (double *)calloc((size_t)(nsteps > 0 ? nsteps : 1) * M, sizeof(double));
    const double dt = 0.05;
    if (orc_run_rank2(kv, ks, A, B, b, dt, M, mu, 0, nsteps, V, S, c, J, y, 0) != 0) bad |= 1;
    /* rank-1 steps of column M-1 equal the rank-2 column bitwise */
    double *v = (double *)calloc(kv, sizeof(double)), *s = (double *)calloc(ks, sizeof(double));
    for (int64_t n = 0; n < nsteps; ++n) orc_step_rank1(kv, ks, A, B, b, dt, n, mu[M - 1], v, s, 0);
    for (int i = 0; i < kv; ++i) if (v[i] != V[i + (size_t)(M - 1) * kv]) bad |= 2;
    for (int i = 0; i < ks; ++i) if (s[i] != S[i + (size_t)(M - 1) * ks]) bad |= 2;
    double *E = (double *)malloc(sizeof(double) * M);
    orc_energy(kv, ks, A, dt, M, V, S, E);
    for (int m = 0; m < M; ++m) if (!isfinite(E[m]) || !isfinite(J[m])) bad |= 4;
    /* adjoint: stride 1, default and longer than the run give equal results */
    double *dA[3], *dB[3], *dm[3], *Ja[3];
    const int64_t strides[3] = {1, 0, nsteps + 5};
    for (int q = 0; q < 3; ++q) {
        dA[q] = (double *)malloc(sizeof(double) * (size_t)kv * ks);
        dB[q] = (double *)malloc(sizeof(double) * (size_t)ks * kv);
        dm[q] = (double *)malloc(sizeof(double) * M);
        Ja[q] = (double *)malloc(sizeof(double) * M);
        for (int src = 0; src < 2; ++src)
            if (orc_adjoint(kv, ks, A, B, b, dt, M, mu, nsteps, c, V, S, Ja[q], dA[q], dB[q], dm[q], strides[q], src))
                bad |= 8;
    }
    for (int q = 1; q < 3; ++q) {
        for (size_t i = 0; i < (size_t)kv * ks; ++i) if (dA[q][i] != dA[0][i] || dB[q][i] != dB[0][i]) bad |= 16;
        for (int m = 0; m < M; ++m) if (dm[q][m] != dm[0][m] || Ja[q][m] != Ja[0][m]) bad |= 16;
    }
    for (int q = 0; q < 3; ++q) { free(dA[q]); free(dB[q]); free(dm[q]); free(Ja[q]); }
    free(A); free(B); free(b); free(c); free(mu); free(V); free(S); free(J); free(y); free(v); free(s); free(E);
    return bad;
}

static int check_fom(void) {
    /* Av: 3 x 4 with an empty row, As: 4 x 3 */
    const int avp[4] = {0, 2, 2, 5}, avc[5] = {0, 3, 1, 2, 3};
    const int asp[5] = {0, 1, 3, 4, 6}, asc[6] = {2, 0, 1, 2, 0, 1};
    double avv[5], asv[6], f[3] = {0.0, 1.0, 0.0};
    for (int k = 0; k < 5; ++k) avv[k] = draw();
    for (int k = 0; k < 6; ++k) asv[k] = draw();
    const int M = 3;
    double mu[3] = {0.6, 0.8, 1.0}, V[9] = {0}, S[12] = {0};
    if (orc_fom_run(3, 4, avp, avc, avv, asp, asc, asv, f, 0.05, M, mu, 0, 40, V, S, 1)) return 32;
    for (int i = 0; i < 9; ++i) if (!isfinite(V[i])) return 32;
    return 0;
}

static int check_scalars(void) {
    int bad = 0;
    for (int i = 0; i < 200; ++i) {
        const double t = 5.0 * (draw() + 1.0), mu = 0.5 + 0.25 * (draw() + 1.0);
        if (!isfinite(orc_ricker(t, mu) + orc_ricker_dmu(t, mu) + orc_gauss1(t, mu) + orc_gauss1_dmu(t, mu))) bad |= 64;
        const double x = 1e3 * draw();
        if (!isfinite(orc_round_bf16(x))) bad |= 64;
    }
    double x[7] = {0.0, -0.0, 1e-9, -3.5, 448.0, 1e5, 2.0e-3}, out[7];
    if (!(orc_quantize_e4m3(7, x, out, 0.0) > 0.0)) bad |= 128;
    if (!(orc_quantize_e4m3(0, x, out, 1.0) > 0.0)) bad |= 128;
    return bad;
}

int main(void) {
    int bad = 0;
    bad |= check_run(5, 3, 2, 40);
    bad |= check_run(3, 7, 1, 25);
    bad |= check_run(8, 8, 4, 0);
    bad |= check_run(1, 1, 3, 17);
    bad |= check_fom();
    bad |= check_scalars();
    printf("oracle sanitizer driver: %s (code %d, %d threads)\n", bad ? "FAILED" : "ok", bad, orc_num_threads());
    return bad ? 1 : 0;
}
