"""GPU discrete adjoint against the FP64 oracle adjoint and finite differences.

Bar: norm-wise relative error <= 1e-4 for dJ/dAvs, dJ/dAsv and dJ/dmu
(FP32 states and operators; the oracle integrates the same FP32-rounded
inputs in FP64).  Finite differences: central, h = 1e-6, of the FP64 oracle
forward run.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _gpu_adjoint(inst, M_cols, nsteps, stride=0, V0=None, S0=None):
    from paper_2009_11742_amd import Rom
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"][M_cols], dtype=torch.float64, device="cuda")
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    v0 = None if V0 is None else torch.tensor(np.ascontiguousarray(V0.T), dtype=torch.float32, device="cuda")
    s0 = None if S0 is None else torch.tensor(np.ascontiguousarray(S0.T), dtype=torch.float32, device="cuda")
    out = rom.adjoint(mu, nsteps, c, V0=v0, S0=s0, stride=stride)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    rom.close()
    return res


def _oracle_adjoint(inst, M_cols, nsteps, V0=None, S0=None):
    return oracle.adjoint(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][M_cols], nsteps,
                          inst["c"], V0=V0, S0=S0)


@pytest.mark.parametrize("kv,ks,M,N,skew,stride", [(40, 40, 6, 300, True, 0), (70, 45, 5, 240, False, 7),
                                                   (64, 64, 4, 500, True, 1), (17, 90, 3, 200, False, 200)])
def test_adjoint_matches_oracle(kv, ks, M, N, skew, stride):
    inst = synth.round_to(synth.make_instance(kv, ks, M, seed=kv * 3 + ks, skew=skew), "f32")
    cols = np.arange(M)
    g = _gpu_adjoint(inst, cols, N, stride=stride)
    r = _oracle_adjoint(inst, cols, N)
    errs = {k: _rel(g[k], r[k]) for k in ("J", "dAvs", "dAsv", "dmu")}
    print("adjoint", (kv, ks, M, N, stride), {k: "%.2e" % v for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL, (k, v)


def test_adjoint_nonzero_start():
    inst = synth.round_to(synth.make_instance(32, 48, 4, seed=5, skew=False), "f32")
    rng = np.random.default_rng(0)
    V0 = rng.standard_normal((32, 4)).astype(np.float32).astype(np.float64)
    S0 = rng.standard_normal((48, 4)).astype(np.float32).astype(np.float64)
    cols = np.arange(4)
    g = _gpu_adjoint(inst, cols, 150, V0=V0, S0=S0)
    r = _oracle_adjoint(inst, cols, 150, V0=V0, S0=S0)
    for k in ("J", "dAvs", "dAsv", "dmu"):
        assert _rel(g[k], r[k]) <= TOL, k


def test_adjoint_vs_finite_differences():
    """Directional derivatives of the FP64 oracle QoI (central, h = 1e-6)."""
    inst = synth.round_to(synth.make_instance(48, 48, 3, seed=9), "f32")
    cols = np.arange(3)
    N = 400
    g = _gpu_adjoint(inst, cols, N)
    rng = np.random.default_rng(4)
    h = 1e-6

    def Jsum(**kw):
        args = dict(Avs=inst["Avs"], Asv=inst["Asv"], mu=inst["mu"])
        args.update(kw)
        return float(np.sum(oracle.run_rank2(args["Avs"], args["Asv"], inst["b"], inst["dt"], args["mu"], N,
                                             c=inst["c"])["J"]))
    for name in ("Avs", "Asv"):
        D = rng.standard_normal(inst[name].shape)
        D /= np.linalg.norm(D)
        fd = (Jsum(**{name: inst[name] + h * D}) - Jsum(**{name: inst[name] - h * D})) / (2 * h)
        an = float(np.sum(g["d" + name] * D))
        assert abs(an - fd) <= TOL * max(abs(fd), 1e-3 * float(np.linalg.norm(g["d" + name]))), (name, an, fd)
    Jp = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"] + h, N, c=inst["c"])["J"]
    Jm = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"] - h, N, c=inst["c"])["J"]
    fd = (Jp - Jm) / (2 * h)
    assert _rel(g["dmu"], fd) <= TOL


def test_adjoint_full_workload_properties():
    """K = 512, M = 256, 5000 steps (the differentiation workload): dmu of
    sampled columns equals a run over those columns alone (columns are
    independent), the operator gradients are additive over disjoint column
    sets, and a K = 512 oracle check on 4 columns over 1000 steps."""
    inst = synth.round_to(synth.make_instance(512, 512, 256, seed=0), "f32")
    N = 5000
    full = _gpu_adjoint(inst, np.arange(256), N)
    assert all(np.all(np.isfinite(v)) for v in full.values())
    cols = np.array([0, 1, 2, 3, 100, 255])
    sub = _gpu_adjoint(inst, cols, N)
    assert _rel(sub["dmu"], full["dmu"][cols]) <= 1e-12
    assert _rel(sub["J"], full["J"][cols]) <= 1e-12
    lo = _gpu_adjoint(inst, np.arange(128), N)
    hi = _gpu_adjoint(inst, np.arange(128, 256), N)
    assert _rel(lo["dAvs"] + hi["dAvs"], full["dAvs"]) <= 1e-6
    assert _rel(lo["dAsv"] + hi["dAsv"], full["dAsv"]) <= 1e-6
    c4 = np.arange(4)
    g = _gpu_adjoint(inst, c4, 1000)
    r = _oracle_adjoint(inst, c4, 1000)
    for k in ("J", "dAvs", "dAsv", "dmu"):
        assert _rel(g[k], r[k]) <= TOL, k


def test_autograd_function():
    from paper_2009_11742_amd import RomQoI
    inst = synth.round_to(synth.make_instance(24, 24, 3, seed=2), "f32")
    Avs = torch.tensor(inst["Avs"], dtype=torch.float64, requires_grad=True)
    Asv = torch.tensor(inst["Asv"], dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda", requires_grad=True)
    J = RomQoI.apply(Avs, Asv, mu, inst["b"], inst["c"], inst["dt"], 200)
    (3.0 * J).backward()
    r = oracle.adjoint(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 200, inst["c"])
    assert abs(float(J) - np.sum(r["J"])) <= TOL * np.sum(r["J"])
    assert _rel(Avs.grad.numpy(), 3.0 * r["dAvs"]) <= TOL
    assert _rel(Asv.grad.numpy(), 3.0 * r["dAsv"]) <= TOL
    assert _rel(mu.grad.cpu().numpy(), 3.0 * r["dmu"]) <= TOL


# ---- checkpoint-free adjoint: states rebuilt by stepping the leapfrog back

@pytest.mark.parametrize("kv,ks,M,N,skew", [(40, 40, 6, 300, True), (70, 45, 5, 240, False),
                                            (64, 64, 4, 500, True), (17, 90, 3, 200, False)])
def test_time_reversal_adjoint_matches_oracle(kv, ks, M, N, skew):
    inst = synth.round_to(synth.make_instance(kv, ks, M, seed=kv * 3 + ks, skew=skew), "f32")
    cols = np.arange(M)
    g = _gpu_adjoint(inst, cols, N, stride=-1)
    c = _gpu_adjoint(inst, cols, N)
    r = _oracle_adjoint(inst, cols, N)
    errs = {k: _rel(g[k], r[k]) for k in ("J", "dAvs", "dAsv", "dmu")}
    vs_ck = {k: _rel(g[k], c[k]) for k in ("J", "dAvs", "dAsv", "dmu")}
    print("reversal adjoint", (kv, ks, M, N), {k: "%.2e" % v for k, v in errs.items()},
          "vs checkpoints", {k: "%.2e" % v for k, v in vs_ck.items()})
    # one forward launch instead of one per checkpoint segment: the state is
    # rounded to FP32 at fewer boundaries, so J agrees to FP32 level only
    assert _rel(g["J"], c["J"]) <= 1e-6
    for k, v in errs.items():
        assert v <= TOL, (k, v)


def test_time_reversal_adjoint_full_workload():
    """K = 512, M = 256, 5000 steps: the reversal gradients against the
    checkpointed ones (the rebuilt states drift by the accumulated
    rounding of the forward and backward sweeps, which stays far below the
    gradient bar), and an oracle check on 4 columns."""
    inst = synth.round_to(synth.make_instance(512, 512, 256, seed=0), "f32")
    N = 5000
    rv = _gpu_adjoint(inst, np.arange(256), N, stride=-1)
    ck = _gpu_adjoint(inst, np.arange(256), N)
    d = {k: _rel(rv[k], ck[k]) for k in ("J", "dAvs", "dAsv", "dmu")}
    print("reversal vs checkpointed adjoint, K=512 M=256 N=5000:", {k: "%.2e" % v for k, v in d.items()})
    assert all(v <= TOL for v in d.values()), d
    c4 = np.arange(4)
    g = _gpu_adjoint(inst, c4, 1000, stride=-1)
    r = _oracle_adjoint(inst, c4, 1000)
    for k in ("J", "dAvs", "dAsv", "dmu"):
        assert _rel(g[k], r[k]) <= TOL, k
