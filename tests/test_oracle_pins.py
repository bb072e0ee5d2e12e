"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test fixes one part of the computation independently:
  * Ricker wavelet: closed-form special points (peak, zeros, minima) and the
    mu-derivative against finite differences;
  * leapfrog form: the 1x1-block ("2x2 harmonic oscillator") discrete closed
    form, and second-order convergence to the continuous solution;
  * operators + forcing + time sampling together: the SVD-modal closed form
    of any skew instance (independent 2x2 oscillators driven by a discrete
    convolution), also with Kv != Ks;
  * the discrete energy identity of the skew-coupled leapfrog;
  * rank-1 == rank-2 column by column (bitwise), linearity, run splitting,
    time reversibility, and brute force on tiny sizes against a separate
    numpy loop, including non-skew operators;
  * adjoint: central finite differences, checkpoint-stride invariance.
The discrete form being pinned is the leapfrog of Sec. 3.1 (velocity first,
then stress, eq. (3.3)) with forcing sampled at t_n = n dt.
"""
import math

import numpy as np
import pytest

import oracle
import synth

PI = math.pi


# --------------------------------------------------------------------------
# Ricker wavelet (Sec. 3.2 names it; unit-peak form with delay 1.5/mu)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mu", [0.5, 0.73, 1.0])
def test_ricker_special_points(mu):
    t0 = 1.5 / mu
    assert oracle.ricker(t0, mu) == pytest.approx(1.0, abs=1e-15)
    # zeros where (mu t - 1.5) = +-1/(sqrt(2) pi)
    for sgn in (-1, 1):
        tz = (1.5 + sgn / (math.sqrt(2.0) * PI)) / mu
        assert abs(oracle.ricker(tz, mu)) < 1e-14
    # minima -2 e^{-3/2} where (mu t - 1.5) = +-sqrt(1.5)/pi
    for sgn in (-1, 1):
        tm = (1.5 + sgn * math.sqrt(1.5) / PI) / mu
        assert oracle.ricker(tm, mu) == pytest.approx(-2.0 * math.exp(-1.5), rel=1e-13)
        h = 1e-5
        slope = (oracle.ricker(tm + h, mu) - oracle.ricker(tm - h, mu)) / (2 * h)
        assert abs(slope) < 1e-8
    # even symmetry about the peak and decay far from it
    for d in (0.1, 0.37, 1.2):
        assert oracle.ricker(t0 + d, mu) == pytest.approx(oracle.ricker(t0 - d, mu), rel=1e-12, abs=1e-15)
    assert abs(oracle.ricker(t0 + 8.0 / mu, mu)) < 1e-200


@pytest.mark.parametrize("t", [0.0, 0.8, 1.9, 2.5, 3.3, 7.0])
@pytest.mark.parametrize("mu", [0.55, 0.8, 0.97])
def test_ricker_dmu_matches_fd(t, mu):
    h = 1e-6
    fd = (oracle.ricker(t, mu + h) - oracle.ricker(t, mu - h)) / (2 * h)
    an = oracle.ricker_dmu(t, mu)
    assert an == pytest.approx(fd, rel=1e-7, abs=1e-9)


# --------------------------------------------------------------------------
# Leapfrog form: 1x1 blocks (Avs = a, Asv = -a) = discrete harmonic oscillator
# --------------------------------------------------------------------------

def _osc_closed_form(a, dt, n, v0, s0):
    """G^n x0 with G = [[1, a dt], [-a dt, 1 - a^2 dt^2]] (det G = 1) via
    Cayley-Hamilton: G^n = (sin(n th) G - sin((n-1) th) I) / sin th,
    th = 2 asin(a dt / 2)."""
    th = 2.0 * math.asin(a * dt / 2.0)
    G = np.array([[1.0, a * dt], [-a * dt, 1.0 - (a * dt) ** 2]])
    Gn = (math.sin(n * th) * G - math.sin((n - 1) * th) * np.eye(2)) / math.sin(th)
    return Gn @ np.array([v0, s0])


@pytest.mark.parametrize("a,dt,n", [(1.0, 0.1, 2000), (2.3, 0.05, 777), (0.7, 0.5, 1500)])
def test_oscillator_closed_form(a, dt, n):
    Avs = np.array([[a]]); Asv = np.array([[-a]]); b = np.zeros(1)
    out = oracle.run_rank2(Avs, Asv, b, dt, [0.7], n, V=[[1.0]], S=[[0.0]])
    ref = _osc_closed_form(a, dt, n, 1.0, 0.0)
    got = np.array([out["V"][0, 0], out["S"][0, 0]])
    assert np.max(np.abs(got - ref)) < 1e-12


def test_oscillator_second_order_convergence():
    """Staggered reading: v^n ~ v(t_n - dt/2), s^n ~ s(t_n).  With exact
    staggered start values the error at fixed T falls ~4x per halving of dt."""
    a, T = 1.3, 5.0
    errs = []
    for k in range(4):
        dt = 0.1 / 2 ** k
        n = int(round(T / dt))
        v0 = math.cos(-a * dt / 2.0)   # v = cos(a t), s = -sin(a t)
        out = oracle.run_rank2([[a]], [[-a]], [0.0], dt, [0.7], n, V=[[v0]], S=[[0.0]])
        ev = out["V"][0, 0] - math.cos(a * (n * dt - dt / 2.0))
        es = out["S"][0, 0] + math.sin(a * n * dt)
        errs.append(math.hypot(ev, es))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert 3.6 < r < 4.4, (errs, ratios)


# --------------------------------------------------------------------------
# SVD-modal closed form of any skew instance (Asv = -Avs^T), with forcing
# --------------------------------------------------------------------------

def _modal_solution(inst, nsteps, V0=None, S0=None):
    """Exact discrete solution through the SVD Avs = U Sigma W^T.

    alpha = U^T v, beta = W^T s decouple into 2x2 oscillators with step matrix
    G_i = [[1, s dt], [-s dt, 1 - s^2 dt^2]] (s = sigma_i) and kick
    [dt bt_i u_n, -s dt^2 bt_i u_n] (bt = U^T b); modes of alpha beyond the
    rank only accumulate dt bt_i u_n, modes of beta beyond it stay constant.
    x^N = G^N x^0 + sum_n G^(N-1-n) k^n with the closed-form powers
    G^k = P_k G - P_{k-1} I, P_k = sin(k th)/sin(th), th = 2 asin(s dt/2).
    The Ricker values come from the oracle's pinned wavelet."""
    Avs, b, dt, mu = inst["Avs"], inst["b"], inst["dt"], inst["mu"]
    kv, ks = Avs.shape
    M = len(mu)
    U, sig, Wt = np.linalg.svd(Avs)          # U kv x kv, Wt ks x ks
    W = Wt.T
    r = len(sig)
    N = nsteps
    tn = np.arange(N) * dt
    u = np.stack([oracle.ricker(tn, m) for m in mu], axis=1)  # N x M
    bt = U.T @ b                                              # kv
    V0 = np.zeros((kv, M)) if V0 is None else np.asarray(V0)
    S0 = np.zeros((ks, M)) if S0 is None else np.asarray(S0)
    al0 = U.T @ V0
    be0 = W.T @ S0
    alpha = np.zeros((kv, M)); beta = np.zeros((ks, M))
    k = np.arange(-1, N + 1)                                   # P_{-1} .. P_N
    for i in range(r):
        s = sig[i]
        th = 2.0 * math.asin(s * dt / 2.0)
        P = np.sin(k * th) / math.sin(th)                      # P[j] = P_{j-1}
        Pk = lambda kk: P[kk + 1]
        G = np.array([[1.0, s * dt], [-s * dt, 1.0 - (s * dt) ** 2]])
        # homogeneous part
        GN = Pk(N) * G - Pk(N - 1) * np.eye(2)
        x = GN @ np.vstack([al0[i], be0[i]])
        # forced part: sum_n G^(N-1-n) [dt bt u_n ; -s dt^2 bt u_n]
        e = N - 1 - np.arange(N)
        c1 = Pk(e)[:, None]            # coefficient of G
        c0 = Pk(e - 1)[:, None]        # coefficient of I
        k0 = dt * bt[i] * u            # N x M (first component)
        k1 = -s * dt * dt * bt[i] * u  # N x M (second component)
        xa = np.sum(c1 * (G[0, 0] * k0 + G[0, 1] * k1) - c0 * k0, axis=0)
        xb = np.sum(c1 * (G[1, 0] * k0 + G[1, 1] * k1) - c0 * k1, axis=0)
        alpha[i] = x[0] + xa
        beta[i] = x[1] + xb
    for i in range(r, kv):
        alpha[i] = al0[i] + dt * bt[i] * u.sum(axis=0)
    for i in range(r, ks):
        beta[i] = be0[i]
    return U @ alpha, W @ beta


def _relcol(X, R):
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.linalg.norm(R, axis=0)))


@pytest.mark.parametrize("kv,ks,M,N", [(64, 64, 8, 2000), (24, 17, 3, 900), (13, 29, 4, 1100), (5, 5, 2, 300)])
def test_modal_closed_form(kv, ks, M, N):
    inst = synth.make_instance(kv, ks, M, seed=3)
    out = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N)
    Vr, Sr = _modal_solution(inst, N)
    assert _relcol(out["V"], Vr) < 1e-11
    assert _relcol(out["S"], Sr) < 1e-11


def test_modal_closed_form_nonzero_start():
    inst = synth.make_instance(11, 11, 3, seed=9)
    rng = np.random.default_rng(1)
    V0 = rng.standard_normal((11, 3)); S0 = rng.standard_normal((11, 3))
    out = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 400, V=V0, S=S0)
    Vr, Sr = _modal_solution(inst, 400, V0, S0)
    assert _relcol(out["V"], Vr) < 1e-11
    assert _relcol(out["S"], Sr) < 1e-11


# --------------------------------------------------------------------------
# Discrete energy of the skew-coupled leapfrog
# --------------------------------------------------------------------------

def test_energy_identity_per_step():
    """E = |v|^2 + |s|^2 + dt v^T Avs s;  E^{n+1} - E^n = dt (b u_n)^T (v^n + v^{n+1})."""
    inst = synth.make_instance(20, 14, 3, seed=5)
    A, B, b, dt, mu = inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"]
    V = np.zeros((20, 3), order="F"); S = np.zeros((14, 3), order="F")
    E = oracle.energy(A, dt, V, S)
    worst = 0.0
    for n in range(60):
        out = oracle.run_rank2(A, B, b, dt, mu, 1, V=V, S=S, n0=n)
        En = oracle.energy(A, dt, out["V"], out["S"])
        u = np.array([oracle.ricker(n * dt, m) for m in mu])
        rhs = dt * np.einsum("i,im->m", b, V + out["V"]) * u
        scale = max(1.0, float(np.max(np.abs(En))))
        worst = max(worst, float(np.max(np.abs((En - E) - rhs))) / scale)
        V, S, E = out["V"], out["S"], En
    assert worst < 1e-13


def test_energy_conserved_after_source():
    inst = synth.make_instance(64, 64, 8, seed=0)
    A, B, b, dt, mu = inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"]
    first = oracle.run_rank2(A, B, b, dt, mu, 200)          # t = 200 dt >> 1.5/mu + decay
    E1 = oracle.energy(A, dt, first["V"], first["S"])
    second = oracle.run_rank2(A, B, b, dt, mu, 1800, V=first["V"], S=first["S"], n0=200)
    E2 = oracle.energy(A, dt, second["V"], second["S"])
    assert np.all(E1 > 0)
    assert np.max(np.abs(E2 - E1) / E1) < 1e-12
    # boundedness: E >= (1 - dt sigma_max / 2) |x|^2  => states bounded
    x2 = np.sum(second["V"] ** 2, axis=0) + np.sum(second["S"] ** 2, axis=0)
    smax = np.linalg.svd(A, compute_uv=False)[0]
    assert np.all(E2 >= (1 - dt * smax / 2) * x2 * (1 - 1e-12))


# --------------------------------------------------------------------------
# Structural identities
# --------------------------------------------------------------------------

def test_rank1_equals_rank2_columns_bitwise():
    inst = synth.make_instance(23, 31, 5, seed=2, random_asv=True)
    A, B, b, dt, mu = inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"]
    N = 150
    out = oracle.run_rank2(A, B, b, dt, mu, N)
    for m in range(5):
        v = np.zeros(23); s = np.zeros(31)
        for n in range(N):
            v, s = oracle.step_rank1(A, B, b, dt, n, mu[m], v, s)
        assert np.array_equal(v, out["V"][:, m])
        assert np.array_equal(s, out["S"][:, m])


def test_linearity_bitwise():
    inst = synth.make_instance(16, 16, 3, seed=4)
    A, B, b, dt, mu = inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"]
    rng = np.random.default_rng(7)
    V0 = rng.standard_normal((16, 3)); S0 = rng.standard_normal((16, 3))
    o1 = oracle.run_rank2(A, B, b, dt, mu, 300, V=V0, S=S0)
    o2 = oracle.run_rank2(A, B, 2 * b, dt, mu, 300, V=2 * V0, S=2 * S0)
    assert np.array_equal(2 * o1["V"], o2["V"]) and np.array_equal(2 * o1["S"], o2["S"])


def test_run_split_bitwise():
    inst = synth.make_instance(12, 9, 4, seed=6)
    A, B, b, dt, mu = inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"]
    c = inst["c"]
    whole = oracle.run_rank2(A, B, b, dt, mu, 500, c=c)
    p1 = oracle.run_rank2(A, B, b, dt, mu, 173, c=c)
    p2 = oracle.run_rank2(A, B, b, dt, mu, 327, V=p1["V"], S=p1["S"], n0=173, c=c)
    assert np.array_equal(whole["V"], p2["V"]) and np.array_equal(whole["S"], p2["S"])
    # J accumulates in step order; the split sum equals the whole one up to one rounding
    assert np.allclose(p1["J"] + p2["J"], whole["J"], rtol=1e-14, atol=0)


def test_mu_permutation_bitwise():
    inst = synth.make_instance(10, 10, 6, seed=8)
    A, B, b, dt, mu = inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"]
    perm = np.array([3, 0, 5, 1, 4, 2])
    o = oracle.run_rank2(A, B, b, dt, mu, 200)
    op = oracle.run_rank2(A, B, b, dt, mu[perm], 200)
    assert np.array_equal(o["V"][:, perm], op["V"])


def test_time_reversibility():
    """Run forward, then undo each step exactly as the leapfrog allows
    (s^n = s^{n+1} - dt Asv v^{n+1}; v^n = v^{n+1} - dt (Avs s^n + b u_n))."""
    inst = synth.make_instance(18, 18, 2, seed=10)
    A, B, b, dt, mu = inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"]
    rng = np.random.default_rng(3)
    V0 = rng.standard_normal((18, 2)); S0 = rng.standard_normal((18, 2))
    N = 400
    out = oracle.run_rank2(A, B, b, dt, mu, N, V=V0, S=S0)
    V, S = out["V"].copy(), out["S"].copy()
    for n in range(N - 1, -1, -1):
        u = np.array([oracle.ricker(n * dt, m) for m in mu])
        S = S - dt * (B @ V)
        V = V - dt * (A @ S + np.outer(b, u))
    assert _relcol(V, V0) < 1e-12 and _relcol(S, S0) < 1e-12


def _numpy_loop(inst, N, c=None):
    A, B, b, dt, mu = inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"]
    kv, ks = A.shape
    M = len(mu)
    V = np.zeros((kv, M)); S = np.zeros((ks, M)); J = np.zeros(M)
    for n in range(N):
        for m in range(M):
            x = math.pi * (mu[m] * n * dt - 1.5)
            u = (1 - 2 * x * x) * math.exp(-x * x)
            V[:, m] = V[:, m] + dt * (A @ S[:, m] + b * u)
        S = S + dt * (B @ V)
        if c is not None:
            J += dt * (c @ V) ** 2
    return V, S, J


@pytest.mark.parametrize("kv,ks,M", [(1, 1, 1), (2, 3, 2), (3, 2, 3), (5, 5, 1), (5, 2, 3), (1, 5, 2)])
@pytest.mark.parametrize("coupling", ["skew", "weighted", "random"])
def test_bruteforce_tiny(kv, ks, M, coupling):
    inst = synth.make_instance(kv, ks, M, seed=kv * 10 + ks, skew=coupling == "skew",
                               random_asv=coupling == "random")
    c = inst["c"]
    out = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 60, c=c)
    V, S, J = _numpy_loop(inst, 60, c)
    assert np.allclose(out["V"], V, rtol=1e-12, atol=1e-13)
    assert np.allclose(out["S"], S, rtol=1e-12, atol=1e-13)
    assert np.allclose(out["J"], J, rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------------------
# Adjoint
# --------------------------------------------------------------------------

def _J(inst, N, Avs=None, Asv=None, mu=None):
    o = oracle.run_rank2(inst["Avs"] if Avs is None else Avs, inst["Asv"] if Asv is None else Asv,
                         inst["b"], inst["dt"], inst["mu"] if mu is None else mu, N, c=inst["c"])
    return float(np.sum(o["J"])), o["J"]


@pytest.mark.parametrize("kv,ks,M,N,coupling", [(12, 12, 3, 200, "skew"), (9, 14, 2, 150, "weighted"),
                                                (6, 4, 4, 90, "skew"), (7, 5, 2, 60, "random")])
def test_adjoint_vs_central_fd(kv, ks, M, N, coupling):
    inst = synth.make_instance(kv, ks, M, seed=21, skew=coupling == "skew", random_asv=coupling == "random")
    adj = oracle.adjoint(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, inst["c"])
    J0, Jm = _J(inst, N)
    assert np.sum(adj["J"]) == pytest.approx(J0, rel=1e-14)
    h = 1e-6
    rng = np.random.default_rng(5)
    for which in ("Avs", "Asv"):
        for _ in range(2):
            D = rng.standard_normal(inst[which].shape)
            D /= np.linalg.norm(D)
            kw_p = {which: inst[which] + h * D}
            kw_m = {which: inst[which] - h * D}
            fd = (_J(inst, N, **kw_p)[0] - _J(inst, N, **kw_m)[0]) / (2 * h)
            an = float(np.sum(adj["d" + which] * D))
            assert an == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(J0))
        # one single entry
        i, j = 1 % inst[which].shape[0], 2 % inst[which].shape[1]
        E = np.zeros(inst[which].shape); E[i, j] = 1.0
        fd = (_J(inst, N, **{which: inst[which] + h * E})[0] - _J(inst, N, **{which: inst[which] - h * E})[0]) / (2 * h)
        assert adj["d" + which][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(J0))
    # all mu at once: J_m depends on mu_m only, so 2 runs give every partial
    Jp = _J(inst, N, mu=inst["mu"] + h)[1]
    Jmn = _J(inst, N, mu=inst["mu"] - h)[1]
    fd = (Jp - Jmn) / (2 * h)
    assert np.allclose(adj["dmu"], fd, rtol=1e-6, atol=1e-9 * abs(J0))


def test_adjoint_checkpoint_stride_invariance():
    inst = synth.make_instance(10, 10, 3, seed=12)
    args = (inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 97, inst["c"])
    ref = oracle.adjoint(*args, stride=1)
    for stride in (0, 7, 10, 96, 97, 500):
        got = oracle.adjoint(*args, stride=stride)
        for k in ("J", "dAvs", "dAsv", "dmu"):
            assert np.array_equal(ref[k], got[k]), (stride, k)


def test_adjoint_nonzero_start_fd():
    inst = synth.make_instance(7, 7, 2, seed=30)
    rng = np.random.default_rng(2)
    V0 = rng.standard_normal((7, 2)); S0 = rng.standard_normal((7, 2))
    adj = oracle.adjoint(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 80, inst["c"], V0, S0)
    h = 1e-6
    D = rng.standard_normal((7, 7)); D /= np.linalg.norm(D)

    def J(A):
        return float(np.sum(oracle.run_rank2(A, inst["Asv"], inst["b"], inst["dt"], inst["mu"], 80,
                                             V=V0, S=S0, c=inst["c"])["J"]))
    fd = (J(inst["Avs"] + h * D) - J(inst["Avs"] - h * D)) / (2 * h)
    assert float(np.sum(adj["dAvs"] * D)) == pytest.approx(fd, rel=1e-6)


# --------------------------------------------------------------------------
# Operator roundings for the low-precision runs vs torch's CPU casts
# --------------------------------------------------------------------------

def test_round_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.uniform(-30, 30, 4000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e-39, -7.1e-41]])
    ours = oracle.round_bf16(x)
    ref = torch.from_numpy(x).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_state_bf16_oracle_hand_example():
    """Two steps of the rounded-state-operand leapfrog, 1 x 1, worked by hand
    in exact dyadic arithmetic: S0 = 1 + 2^-9 rounds to 1 (BF16 spacing 2^-7
    on [1, 2)), V1 = 1 + 0.25 * 0.5 * 1 = 1.125, S1 = S0 - 0.125 * 1.125 =
    0.861328125 = 220.5 * 2^-8, which rounds (tie, to even) to 0.859375;
    V2 = 1.125 + 0.125 * 0.859375 = 1.232421875 rounds to 1.234375 (157.75 *
    2^-7 -> 158), S2 = S1 - 0.125 * 1.234375 = 0.70703125.  The unrounded
    leapfrog gives V1 = 1.125244140625 instead."""
    out = oracle.run_rank2_state_bf16([[0.5]], [[-0.5]], [0.0], 0.25, [1.0], 2,
                                      V=[[1.0]], S=[[1.0 + 2.0 ** -9]])
    assert out["V"][0, 0] == 1.232421875
    assert out["S"][0, 0] == 0.70703125
    one = oracle.run_rank2_state_bf16([[0.5]], [[-0.5]], [0.0], 0.25, [1.0], 1,
                                      V=[[1.0]], S=[[1.0 + 2.0 ** -9]])
    assert one["V"][0, 0] == 1.125 and one["S"][0, 0] == 0.861328125
    plain = oracle.run_rank2([[0.5]], [[-0.5]], [0.0], 0.25, [1.0], 1, V=[[1.0]], S=[[1.0 + 2.0 ** -9]])
    assert plain["V"][0, 0] == 1.125244140625


def test_state_bf16_oracle_forcing_unrounded():
    """With zero operators the rounding never enters (it acts on product
    operands only), so the model equals the plain leapfrog bitwise: the
    forcing b u(t_n) is added in FP64 at the same step times."""
    rng = np.random.default_rng(5)
    kv, ks, M = 5, 3, 4
    b = rng.standard_normal(kv)
    mu = rng.uniform(0.5, 1.0, M)
    V0, S0 = rng.standard_normal((kv, M)), rng.standard_normal((ks, M))
    for source in ("ricker", "gauss1"):
        a = oracle.run_rank2_state_bf16(np.zeros((kv, ks)), np.zeros((ks, kv)), b, 0.25, mu, 9, V=V0, S=S0,
                                        n0=3, source=source)
        p = oracle.run_rank2(np.zeros((kv, ks)), np.zeros((ks, kv)), b, 0.25, mu, 9, V=V0, S=S0, n0=3,
                             source=source)
        assert np.array_equal(a["V"], p["V"]) and np.array_equal(a["S"], p["S"])


def test_quantize_e4m3_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = rng.standard_normal((37, 41)) / 7.0
    x[3, 4] = 0.0
    deq, scale = oracle.quantize_e4m3(x)
    x32 = torch.from_numpy(x).to(torch.float32)
    sc = (x32.abs().max() / 448.0)
    assert float(sc) == scale
    q = torch.clamp(x32 / sc, -448.0, 448.0).to(torch.float8_e4m3fn).to(torch.float64)
    ref = (q * float(sc)).numpy()
    assert np.array_equal(deq, ref)
    # ties-to-even and subnormals on crafted values (scale 1 via amax = 448)
    y = np.array([448.0, 460.0, 500.0, -1e9, 1.0625, 1.1875, 0.0029296875, 0.001953125, 0.0009765625, 0.00146484375])
    deq2, s2 = oracle.quantize_e4m3(y, amax=448.0)
    assert s2 == 1.0
    ref2 = torch.clamp(torch.from_numpy(y).to(torch.float32), -448, 448).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(deq2, ref2)


# --------------------------------------------------------------------------
# Receivers (seismograms from single basis rows, Sec. 4.5) and ensemble
# statistics (mean and percentile bounds over the ensemble)
# --------------------------------------------------------------------------

def test_receivers_single_row_reproduces_probe_qoi_and_trace():
    """With one receiver row equal to the probe c, the seismogram is the
    probe trace y and dt sum_n y^2 is the probe QoI J of run_rank2."""
    inst = synth.make_instance(24, 20, 5, seed=31, skew=False)
    N = 60
    rc = oracle.receivers(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, inst["c"][None, :])
    r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"], trace=True)
    assert np.allclose(rc["Y"][:, 0, :], r["y"], rtol=1e-13, atol=1e-15 * np.max(np.abs(r["y"])))
    J = inst["dt"] * np.sum(rc["Y"][:, 0, :] ** 2, axis=0)
    assert np.allclose(J, r["J"], rtol=1e-12)
    assert np.array_equal(rc["V"], r["V"]) and np.array_equal(rc["S"], r["S"])


def test_receivers_linear_in_rows_and_offset_run():
    inst = synth.make_instance(16, 16, 3, seed=32)
    rng = np.random.default_rng(1)
    C1, C2 = rng.standard_normal((2, 16)), rng.standard_normal((2, 16))
    N = 40
    y1 = oracle.receivers(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, C1)["Y"]
    y2 = oracle.receivers(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, C2)["Y"]
    y12 = oracle.receivers(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, C1 + 2.0 * C2)["Y"]
    assert np.allclose(y12, y1 + 2.0 * y2, rtol=1e-12, atol=1e-14 * np.max(np.abs(y12)))
    # a run split at step 15 gives the same rows
    a = oracle.receivers(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 15, C1)
    b2 = oracle.receivers(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N - 15, C1, V=a["V"], S=a["S"], n0=15)
    assert np.array_equal(np.concatenate([a["Y"], b2["Y"]]), y1)


def test_ensemble_stats_closed_forms():
    # 1..M: mean (M+1)/2, population variance (M^2-1)/12; nearest rank
    for M in (1, 2, 7, 20, 100, 256, 1000):
        Y = np.random.default_rng(M).permutation(np.arange(1, M + 1, dtype=np.float64))[None, :]
        st = oracle.ensemble_stats(Y)[0]
        assert st[0] == pytest.approx((M + 1) / 2, rel=1e-15)
        assert st[1] == pytest.approx((M * M - 1) / 12, rel=1e-13, abs=1e-15)
        for k, p in enumerate((5, 50, 95)):
            assert st[2 + k] == max(1, math.ceil(p * M / 100))    # the value equals its rank
    # every percentile is one of the samples, and p05 <= p50 <= p95
    Y = np.random.default_rng(0).standard_normal((7, 3, 33))
    st = oracle.ensemble_stats(Y)
    for i in range(7):
        for r in range(3):
            assert all(v in Y[i, r] for v in st[i, r, 2:])
            assert st[i, r, 2] <= st[i, r, 3] <= st[i, r, 4]
    assert oracle.percentile_index(5, 20) == 0 and oracle.percentile_index(50, 20) == 9
    assert oracle.percentile_index(95, 20) == 18 and oracle.percentile_index(95, 1) == 0


# ---- affine operator families (rank-3 direction)

def test_affine_operator_hand_example():
    """Two non-symmetric 2 x 3 terms with integer entries and dyadic
    coefficients: the sum is exact and written out by hand."""
    T = np.array([[[1., 2., 3.], [4., 5., 6.]],
                  [[0., -1., 0.], [2., 0., -8.]]])
    got = oracle.affine_operator(T, [0.5, 0.25])
    want = np.array([[0.5, 0.75, 1.5], [2.5, 2.5, 1.0]])
    assert np.array_equal(got, want)


def test_affine_operator_unit_coefficients_pick_terms():
    syn = synth.make_affine_family(7, 5, 4, 1, 1, seed=2)
    for q in range(4):
        e = np.zeros(4); e[q] = 1.0
        assert np.array_equal(oracle.affine_operator(syn["Avs_terms"], e), syn["Avs_terms"][q])


def test_affine_family_of_multiples_runs_as_scaled_operator():
    """Terms c_q A (scalars c_q): the instance is (sum theta_q c_q) A, so its
    run equals the run of that scaled operator, and sigma_max scales by the
    same factor."""
    inst = synth.make_instance(24, 24, 3, seed=4)
    A, B = inst["Avs"], inst["Asv"]
    cs = np.array([0.5, -0.25, 2.0])
    th = np.array([0.75, 0.5, 0.125])
    f = float(th @ cs)                       # 0.5
    Ai = oracle.affine_operator(np.stack([c * A for c in cs]), th)
    Bi = oracle.affine_operator(np.stack([c * B for c in cs]), th)
    bound = 8 * np.finfo(float).eps * float(np.abs(th) @ np.abs(cs))
    assert np.max(np.abs(Ai - f * A)) <= bound * np.max(np.abs(A))
    assert np.max(np.abs(Bi - f * B)) <= bound * np.max(np.abs(B))
    s = np.linalg.svd(Ai, compute_uv=False)[0] / np.linalg.svd(A, compute_uv=False)[0]
    assert abs(s - f) < 1e-13
    r1 = oracle.run_rank2(Ai, Bi, inst["b"], inst["dt"], inst["mu"], 300)
    r2 = oracle.run_rank2(f * A, f * B, inst["b"], inst["dt"], inst["mu"], 300)
    e = np.max(np.linalg.norm(r1["V"] - r2["V"], axis=0) / np.linalg.norm(r2["V"], axis=0))
    assert e < 1e-12


def test_affine_operator_linear_in_theta():
    syn = synth.make_affine_family(9, 6, 3, 2, 1, seed=8)
    T = syn["Avs_terms"]
    t1, t2 = syn["theta"]
    lhs = oracle.affine_operator(T, 2.0 * t1 - 3.0 * t2)
    rhs = 2.0 * oracle.affine_operator(T, t1) - 3.0 * oracle.affine_operator(T, t2)
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(lhs))


# ---- full-order model, Galerkin projection and POD (offline side)

def test_fom_grid_sizes_match_the_paper():
    """The velocity grids of the FOM scaling runs (256 x 1024 ... 2048 x
    8192) give the total degree-of-freedom counts printed with them
    (Sec. 4.1)."""
    want = {(256, 1024): 785152, (512, 2048): 3143168, (1024, 4096): 12577792, (2048, 8192): 50321408}
    for (nr, nth), n in want.items():
        nv, ns = synth.shear_fom_sizes(nr, nth)
        assert nv + ns == n
    d = synth.make_shear_fom(256, 1024)
    assert d["nv"] + d["ns"] == 785152


def test_fom_operator_structure():
    """About four entries per velocity row and two per stress row (Sec. 3.1):
    interior velocity rows 4, radial-boundary rows 3 (free surface), axis
    rows 0 (v = 0 there); s_rp rows 2 (0 on the axis), s_tp rows 2."""
    nr, nth = 7, 9
    d = synth.make_shear_fom(nr, nth)
    nv = np.diff(d["Av"][0]).reshape(nr, nth)
    assert np.all(nv[:, 0] == 0) and np.all(nv[:, -1] == 0)
    assert np.all(nv[1:-1, 1:-1] == 4) and np.all(nv[0, 1:-1] == 3) and np.all(nv[-1, 1:-1] == 3)
    ns = np.diff(d["As"][0])
    nrp = (nr - 1) * nth
    srp = ns[:nrp].reshape(nr - 1, nth)
    assert np.all(srp[:, 0] == 0) and np.all(srp[:, -1] == 0) and np.all(srp[:, 1:-1] == 2)
    assert np.all(ns[nrp:] == 2)
    assert np.count_nonzero(d["f"]) == 1 and d["f"][d["src"]] == 1.0 / d["rho"]
    assert d["src"] % nth == 1


def _fom_consistency_errors(nr, nth):
    """Max errors of As v and Av s against the continuous right-hand sides of
    eq. (3.1) for smooth fields (v = sin(pi x) sin(2 th), s_rp = sin(pi x)
    sin(th), s_tp = cos(pi x) sin(2 th), x = (r - r_cmb) / L), over interior
    points (two cells away from the radial boundaries)."""
    d = synth.make_shear_fom(nr, nth)
    rc, L = d["r_cmb"], 6371e3 - d["r_cmb"]
    dr, dth, rho, mu = d["dr"], d["dth"], d["rho"], d["rho"] * d["vs"] ** 2
    Av = oracle.csr_dense(d["Av"], d["ns"])
    As = oracle.csr_dense(d["As"], d["nv"])
    k = math.pi / L
    # velocity field on the velocity points
    I, J = np.meshgrid(np.arange(nr), np.arange(nth), indexing="ij")
    r, th = rc + I * dr, J * dth
    v = np.sin(k * (r - rc)) * np.sin(2 * th)
    Sv = As @ v.ravel()
    nrp = (nr - 1) * nth
    Ih, Jh = np.meshgrid(np.arange(nr - 1), np.arange(nth), indexing="ij")
    rh, thh = rc + (Ih + 0.5) * dr, Jh * dth
    want_rp = mu * (k * np.cos(k * (rh - rc)) * np.sin(2 * thh) - np.sin(k * (rh - rc)) * np.sin(2 * thh) / rh)
    It, Jt = np.meshgrid(np.arange(nr), np.arange(nth - 1), indexing="ij")
    rt, tht = rc + It * dr, (Jt + 0.5) * dth
    want_tp = mu * (np.sin(k * (rt - rc)) * 2 * np.cos(2 * tht) / rt
                    - np.cos(tht) / np.sin(tht) * np.sin(k * (rt - rc)) * np.sin(2 * tht) / rt)
    e_rp = np.abs(Sv[:nrp].reshape(nr - 1, nth) - want_rp)[2:-2, 1:-1].max() / np.abs(want_rp).max()
    e_tp = np.abs(Sv[nrp:].reshape(nr, nth - 1) - want_tp)[2:-2, :].max() / np.abs(want_tp).max()
    # stress fields on their points
    srp = np.sin(k * (rh - rc)) * np.sin(thh)
    stp = np.cos(k * (rt - rc)) * np.sin(2 * tht)
    Vs = Av @ np.concatenate([srp.ravel(), stp.ravel()])
    s_rp = lambda rr, tt: np.sin(k * (rr - rc)) * np.sin(tt)
    want_v = (k * np.cos(k * (r - rc)) * np.sin(th) + np.cos(k * (r - rc)) * 2 * np.cos(2 * th) / r
              + (3 * s_rp(r, th) + 2 * np.cos(k * (r - rc)) * np.sin(2 * th) * np.cos(th) / np.sin(np.where(J > 0, th, 1.0))) / r) / rho
    e_v = np.abs(Vs.reshape(nr, nth) - want_v)[2:-2, 1:-1].max() / np.abs(want_v[2:-2, 1:-1]).max()
    return e_rp, e_tp, e_v


def test_fom_operators_second_order_consistent():
    """Halving the grid spacing cuts the truncation error of both operators
    about fourfold (second-order centred differences, Sec. 3.1)."""
    e1 = _fom_consistency_errors(17, 33)
    e2 = _fom_consistency_errors(33, 65)
    ratios = [a / b for a, b in zip(e1, e2)]
    print("FOM consistency errors", e1, e2, "ratios", ratios)
    assert all(3.5 < q < 4.5 for q in ratios), ratios
    assert max(e2) < 1e-2


def test_fom_rank1_columns_equal_rank2_bitwise():
    d = synth.make_shear_fom(6, 10)
    mu = synth.fom_periods(4, seed=3)
    r2 = oracle.fom_run(d["Av"], d["As"], d["f"], d["dt"], mu, 300)
    for m in (0, 3):
        r1 = oracle.fom_run(d["Av"], d["As"], d["f"], d["dt"], mu[m:m + 1], 300)
        assert np.array_equal(r1["V"][:, 0], r2["V"][:, m]) and np.array_equal(r1["S"][:, 0], r2["S"][:, m])


def test_full_basis_rom_reproduces_fom():
    """With orthonormal bases spanning the whole velocity and stress spaces,
    the Galerkin ROM is the FOM in rotated coordinates: Phi_v V_rom equals
    V_fom up to rounding.  This ties the FOM stepper, the projection and the
    ROM oracle (separate code) together."""
    d = synth.make_shear_fom(5, 7)
    rng = np.random.default_rng(1)
    Pv, _ = np.linalg.qr(rng.standard_normal((d["nv"], d["nv"])))
    Ps, _ = np.linalg.qr(rng.standard_normal((d["ns"], d["ns"])))
    Avs, Asv, b = oracle.project(d["Av"], d["As"], d["f"], Pv, Ps)
    mu = synth.fom_periods(3, seed=2)
    N = 200
    rom = oracle.run_rank2(Avs, Asv, b, d["dt"], mu, N)
    fom = oracle.fom_run(d["Av"], d["As"], d["f"], d["dt"], mu, N)
    ev = np.linalg.norm(Pv @ rom["V"] - fom["V"]) / np.linalg.norm(fom["V"])
    es = np.linalg.norm(Ps @ rom["S"] - fom["S"]) / np.linalg.norm(fom["S"])
    print("full-basis ROM vs FOM: %.2e %.2e" % (ev, es))
    assert ev < 1e-10 and es < 1e-10


def test_projection_onto_coordinate_basis_is_submatrix():
    d = synth.make_shear_fom(6, 9)
    Av = oracle.csr_dense(d["Av"], d["ns"])
    As = oracle.csr_dense(d["As"], d["nv"])
    iv = np.array([3, 10, 11, 25, 40])
    is_ = np.array([0, 7, 30, 31, 50, 60, 70])
    Pv = np.eye(d["nv"])[:, iv]
    Ps = np.eye(d["ns"])[:, is_]
    Avs, Asv, b = oracle.project(d["Av"], d["As"], d["f"], Pv, Ps)
    assert np.array_equal(Avs, Av[np.ix_(iv, is_)]) and np.array_equal(Asv, As[np.ix_(is_, iv)])
    assert np.array_equal(b, d["f"][iv])


def test_pod_recovers_a_constructed_spectrum():
    """X = U diag(s) W^T with known orthonormal U, W: POD returns s and the
    leading columns of U (up to sign); the energy criterion keeps the
    smallest k whose energy fraction reaches 1 - tol."""
    rng = np.random.default_rng(4)
    N, ns = 400, 30
    U, _ = np.linalg.qr(rng.standard_normal((N, ns)))
    W, _ = np.linalg.qr(rng.standard_normal((ns, ns)))
    s = 10.0 ** (-np.arange(ns, dtype=float) / 2.0)    # energies 10^-i
    X = U @ np.diag(s) @ W.T
    Phi, sig, k = oracle.pod(X, tol=3e-6)
    assert np.allclose(sig, s, rtol=1e-9, atol=1e-14 * s[0])
    # energy left out after k modes: sum_{i>=k} 10^-i / sum_i 10^-i = 10^-k
    # (to 1e-30), which first falls to 3e-6 at k = 6
    assert k == 6
    G = Phi.T @ U[:, :k]
    assert np.allclose(np.abs(np.diag(G)), 1.0, atol=1e-10)
    # energies 16 and 9 of 25: one mode holds 0.64
    assert oracle.pod_rank([4.0, 3.0], 0.36) == 1 and oracle.pod_rank([4.0, 3.0], 0.35) == 2


# ---- the second source signal: first derivative of a Gaussian

@pytest.mark.parametrize("mu", [1.0 / 60.0, 0.7])
def test_gauss1_shape(mu):
    """Unit peak at x = -1/sqrt(2) (t = (3 - 1/(sqrt(2) pi)) / mu), zero at the
    delay 3/mu, odd about it, and proportional to the time derivative of the
    Gaussian exp(-(pi (mu t - 3))^2) (central differences of that bump)."""
    t0 = 3.0 / mu
    tp = (3.0 - 1.0 / (math.sqrt(2.0) * math.pi)) / mu
    assert abs(float(oracle.gauss1(tp, mu)) - 1.0) < 1e-14
    assert abs(float(oracle.gauss1(t0, mu))) < 1e-13       # t0 = 3 / mu rounds
    ts = np.linspace(0.0, 2 * t0, 801)
    u = oracle.gauss1(ts, mu)
    assert np.max(np.abs(u)) <= 1.0 + 1e-14
    assert np.allclose(oracle.gauss1(t0 + (ts - t0), mu), -oracle.gauss1(t0 - (ts - t0), mu), atol=1e-13)
    h = 1e-4 / mu
    bump = lambda t: np.exp(-(math.pi * (mu * t - 3.0)) ** 2)
    d = (bump(ts + h) - bump(ts - h)) / (2 * h)
    scale = math.sqrt(2.0 * math.e) / (2.0 * math.pi * mu)
    assert np.max(np.abs(u - scale * d)) < 1e-7


@pytest.mark.parametrize("t,mu", [(100.0, 1.0 / 65.0), (3.0, 0.9), (5.0, 0.55)])
def test_gauss1_dmu_matches_fd(t, mu):
    h = 1e-6 * mu
    fd = (float(oracle.gauss1(t, mu + h)) - float(oracle.gauss1(t, mu - h))) / (2 * h)
    assert abs(float(oracle.gauss1_dmu(t, mu)) - fd) <= 1e-6 * max(1.0, abs(fd))


def test_source_kind_reaches_the_step():
    """With zero operators the leapfrog only accumulates the forcing:
    V_N = dt sum_n b u(t_n), S stays 0 -- for each source kind."""
    kv, ks, M, N, dt = 3, 2, 4, 300, 0.01
    b = np.array([1.0, -2.0, 0.5])
    mu = np.array([0.6, 0.7, 0.8, 0.95])
    Z1, Z2 = np.zeros((kv, ks), order="F"), np.zeros((ks, kv), order="F")
    for src, fn in (("ricker", oracle.ricker), ("gauss1", oracle.gauss1)):
        r = oracle.run_rank2(Z1, Z2, b, dt, mu, N, source=src)
        t = np.arange(N) * dt
        want = dt * np.outer(b, [np.sum(fn(t, m)) for m in mu])
        assert np.allclose(r["V"], want, rtol=1e-12, atol=1e-15) and not np.any(r["S"])
    a = oracle.run_rank2(Z1, Z2, b, dt, mu, N, source="ricker")["V"]
    g = oracle.run_rank2(Z1, Z2, b, dt, mu, N, source="gauss1")["V"]
    assert np.max(np.abs(a - g)) > 1e-3


# ---- adjoint by complex step: directional derivatives exact to rounding

def _complex_J(Avs, Asv, b, dt, mu, N, c, ricker):
    """The probe QoI of the leapfrog, written out again in complex arithmetic
    (numpy, separate from the oracle's C): J = sum_m sum_n dt (c^T V_m)^2."""
    kv, ks = Avs.shape
    M = len(mu)
    V = np.zeros((kv, M), dtype=complex)
    S = np.zeros((ks, M), dtype=complex)
    J = 0.0 + 0.0j
    for n in range(N):
        u = ricker(n * dt, mu)
        V = V + dt * (Avs @ S + np.outer(b, u))
        S = S + dt * (Asv @ V)
        y = c @ V
        J = J + dt * np.sum(y * y)
    return J


def _ricker_c(t, mu):
    a = (np.pi * (mu * t - 1.5)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


@pytest.mark.parametrize("kv,ks,M,N", [(5, 4, 3, 60), (7, 7, 2, 120)])
def test_adjoint_complex_step(kv, ks, M, N):
    """Complex-step directional derivatives (h = 1e-30, no cancellation) of
    the QoI along random directions of Avs, Asv and mu equal the oracle
    adjoint's inner products to 1e-10: a pin of the adjoint far tighter than
    finite differences (the dot-product test of the tangent and the
    adjoint)."""
    inst = synth.make_instance(kv, ks, M, seed=kv + N, skew=False)
    A, B, b, dt, mu, c = inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], inst["c"]
    adj = oracle.adjoint(A, B, b, dt, mu, N, c)
    h = 1e-30
    rng = np.random.default_rng(3)
    J0 = _complex_J(A, B, b, dt, mu, N, c, _ricker_c).real
    assert abs(J0 - np.sum(adj["J"])) <= 1e-12 * abs(J0)
    for _ in range(2):
        DA = rng.standard_normal(A.shape)
        DB = rng.standard_normal(B.shape)
        Dm = rng.standard_normal(M)
        d = _complex_J(A + 1j * h * DA, B + 1j * h * DB, b, dt, mu + 1j * h * Dm, N, c, _ricker_c).imag / h
        an = float(np.sum(adj["dAvs"] * DA) + np.sum(adj["dAsv"] * DB) + np.sum(adj["dmu"] * Dm))
        assert abs(an - d) <= 1e-10 * max(abs(d), 1e-300), (an, d)
