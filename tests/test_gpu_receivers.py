"""Seismograms at R receivers and ensemble statistics (rom_run_receivers)
against the FP64 oracle (oracle.receivers / oracle.ensemble_stats).

Bars: Y within 1e-5 of the oracle relative to max |Y| (FP32 states); mean
and variance within 1e-5 (relative to the spread); percentiles bitwise equal
to the nearest-rank selection applied to the GPU's own Y (the selection is
exact) and within the Y bar of the oracle's.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _run(inst, N, C, cols=None, n0=0):
    from paper_2009_11742_amd import Rom
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu_np = inst["mu"] if cols is None else inst["mu"][cols]
    M = len(mu_np)
    mu = torch.tensor(mu_np, dtype=torch.float64, device="cuda")
    V, S = rom.zeros(M)
    Ct = torch.tensor(np.ascontiguousarray(C), dtype=torch.float32, device="cuda")
    out = rom.run_receivers(mu, V, S, N, Ct, n0=n0)
    torch.cuda.synchronize()
    res = {"Y": out["Y"].cpu().numpy(), "stats": out["stats"].cpu().numpy(),
           "V": V.cpu().numpy().astype(np.float64).T}
    rom.close()
    return res


def _check_stats_self(g):
    """GPU statistics equal the definitions applied to the GPU's own Y."""
    mine = oracle.ensemble_stats(g["Y"])
    assert np.array_equal(g["stats"][..., 2:], mine[..., 2:])           # exact order statistics
    assert np.allclose(g["stats"][..., 0], mine[..., 0], rtol=1e-12, atol=1e-15 * np.max(np.abs(g["Y"])))
    assert np.allclose(g["stats"][..., 1], mine[..., 1], rtol=1e-10, atol=1e-15 * np.max(g["Y"] ** 2))


@pytest.mark.parametrize("kv,ks,M,R,N", [(96, 80, 37, 5, 300), (64, 64, 1, 3, 200), (130, 70, 64, 16, 150)])
def test_receivers_match_oracle(kv, ks, M, R, N):
    inst = synth.round_to(synth.make_instance(kv, ks, M, seed=kv + 7 * M, skew=(kv == ks)), "f32")
    C = np.asarray(np.random.default_rng(kv).standard_normal((R, kv)), dtype=np.float32).astype(np.float64)
    g = _run(inst, N, C)
    ref = oracle.receivers(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, C)
    ys = np.max(np.abs(ref["Y"]))
    e = float(np.max(np.abs(g["Y"] - ref["Y"])) / ys)
    st = oracle.ensemble_stats(ref["Y"])
    spread = np.sqrt(np.max(st[..., 1])) + 1e-300
    em = float(np.max(np.abs(g["stats"][..., 0] - st[..., 0])) / ys)
    ev = float(np.max(np.abs(np.sqrt(g["stats"][..., 1]) - np.sqrt(st[..., 1]))) / max(spread, 1e-30 * ys))
    ep = float(np.max(np.abs(g["stats"][..., 2:] - st[..., 2:])) / ys)
    print("receivers kv=%d ks=%d M=%d R=%d N=%d: Y %.2e mean %.2e std %.2e pct %.2e" % (kv, ks, M, R, N, e, em, ev, ep))
    assert e <= 1e-5 and em <= 1e-5 and ep <= 1e-5
    if M > 1:
        assert ev <= 1e-5
    _check_stats_self(g)


def test_receivers_two_chunks_and_probe_consistency():
    """5000 steps at K = 64 span two chunks (4096 + 904 steps); the first
    receiver row equal to the probe c reproduces the probe trace of a
    plain run, and the final state matches the oracle."""
    from paper_2009_11742_amd import Rom
    K, M, N = 64, 16, 5000
    inst = synth.round_to(synth.make_instance(K, K, M, seed=41), "f32")
    rng = np.random.default_rng(2)
    C = np.stack([inst["c"], np.asarray(rng.standard_normal(K), dtype=np.float32).astype(np.float64)])
    g = _run(inst, N, C)
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule="columns")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(M)
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    J = torch.zeros(M, dtype=torch.float64, device="cuda")
    y = torch.zeros((N, M), dtype=torch.float64, device="cuda")
    rom.run_rank2(mu, V, S, N, c=c, J=J, y=y)
    torch.cuda.synchronize()
    yp = y.cpu().numpy()
    # the receiver run rounds its state at the chunk boundary (step 4096) and
    # reads FP32-rounded trace states; the plain run keeps the two-term state
    # throughout, so the two agree to the FP32 bar, not bitwise
    assert np.max(np.abs(g["Y"][:, 0, :] - yp)) <= 1e-5 * np.max(np.abs(yp))
    rom.close()
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"], trace=True)
    assert np.max(np.abs(g["Y"][:, 0, :] - ref["y"])) <= 1e-5 * np.max(np.abs(ref["y"]))
    nr = np.linalg.norm(ref["V"], axis=0)
    assert np.max(np.linalg.norm(g["V"] - ref["V"], axis=0) / nr) <= 1e-5
    _check_stats_self(g)


def test_receivers_bench_size_sampled():
    """K = 256, M = 256, R = 16, 1500 steps: statistics equal their
    definitions on the GPU's Y, and three sampled columns match the oracle."""
    K, M, R, N = 256, 256, 16, 1500
    inst = synth.round_to(synth.make_instance(K, K, M, seed=0), "f32")
    C = np.asarray(np.random.default_rng(3).standard_normal((R, K)), dtype=np.float32).astype(np.float64)
    g = _run(inst, N, C)
    _check_stats_self(g)
    cols = np.array([0, 128, 255])
    ref = oracle.receivers(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][cols], N, C)
    e = float(np.max(np.abs(g["Y"][:, :, cols] - ref["Y"])) / np.max(np.abs(ref["Y"])))
    print("receivers K=M=256 R=16 N=1500 sampled: Y %.2e" % e)
    assert e <= 1e-5


def test_receivers_argument_errors():
    from paper_2009_11742_amd import Rom, RomError
    from paper_2009_11742_amd import _lib
    inst = synth.round_to(synth.make_instance(32, 32, 200, seed=5), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(200)
    for R, code in ((65, _lib.ROM_E_ARG), (50, _lib.ROM_E_UNSUPPORTED)):      # 50 x 200 > 8192
        C = torch.zeros((R, 32), dtype=torch.float32, device="cuda")
        with pytest.raises(RomError) as ei:
            rom.run_receivers(mu, V, S, 10, C)
        assert ei.value.status == code
    assert torch.count_nonzero(V) == 0
    rom.close()
