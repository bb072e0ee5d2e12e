"""Operator-resident schedule (skew FP32 pairs, Kv, Ks <= 256): one sample
per workgroup with all of Avs in its registers, used for both half-steps
(Asv V = -Avs^T V).

Parity against the FP64 oracle on the same FP32-rounded inputs at the FP32
bar (1e-5, per-sample relative l2 error of the final states; the probe QoI
J and trace y relative): square and rectangular (Kv != Ks) skew pairs over
every tile shape (padded Kv in {64, 128, 192, 256}, Ks in {64, ..., 256}),
ragged sizes and M; the rank-2 bench workload (K = 256, M = 256, 10^4 steps)
on sampled columns.  Structural checks: a permutation of the samples
permutes the results bitwise, a run split in two equals the whole run to a
rounding of the state, graph replays equal the eager run bitwise, a
non-skew pair asked for this schedule falls back to column blocks.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
BAR = 1e-5


def _relcol(X, R):
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.linalg.norm(R, axis=0)))


def _run(inst, N, cols=None, schedule="resident", trace=True, n_split=None):
    from paper_2009_11742_amd import Rom
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule=schedule)
    mu_np = inst["mu"] if cols is None else inst["mu"][cols]
    M = len(mu_np)
    mu = torch.tensor(mu_np, dtype=torch.float64, device="cuda")
    V, S = rom.zeros(M)
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    J = torch.zeros(M, dtype=torch.float64, device="cuda")
    y = torch.zeros((N, M), dtype=torch.float64, device="cuda") if trace else None
    if n_split is None:
        rom.run_rank2(mu, V, S, N, c=c, J=J, y=y)
    else:
        rom.run_rank2(mu, V, S, n_split, c=c, J=J)
        rom.run_rank2(mu, V, S, N - n_split, n0=n_split, c=c, J=J)
    torch.cuda.synchronize()
    sched = rom.last_schedule
    rom.close()
    return {"V": V.cpu().numpy().astype(np.float64).T, "S": S.cpu().numpy().astype(np.float64).T,
            "J": J.cpu().numpy(), "y": None if y is None else y.cpu().numpy(), "sched": sched}


@pytest.mark.parametrize("kv,ks,M,N", [(256, 256, 40, 1500), (200, 120, 9, 800), (64, 64, 5, 600),
                                       (128, 256, 7, 700), (192, 192, 13, 700), (100, 60, 3, 500),
                                       (256, 64, 6, 600), (33, 250, 4, 400)])
def test_resident_parity(kv, ks, M, N):
    inst = synth.round_to(synth.make_instance(kv, ks, M, seed=kv + 7 * ks + M), "f32")
    g = _run(inst, N)
    assert g["sched"] == "resident"
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"],
                           trace=True)
    ev, es = _relcol(g["V"], ref["V"]), _relcol(g["S"], ref["S"])
    ej = float(np.max(np.abs(g["J"] - ref["J"]) / ref["J"]))
    ey = float(np.max(np.linalg.norm(g["y"] - ref["y"], axis=0) / np.linalg.norm(ref["y"], axis=0)))
    print("resident K=(%d,%d) M=%d N=%d: V %.2e S %.2e J %.2e y %.2e" % (kv, ks, M, N, ev, es, ej, ey))
    assert max(ev, es, ej, ey) <= BAR


def test_resident_bench_workload_sampled():
    """K = 256, M = 256, 10^4 steps, all samples stepped, 8 checked."""
    inst = synth.round_to(synth.make_instance(256, 256, 256, seed=0), "f32")
    N = 10000
    g = _run(inst, N, trace=False)
    assert g["sched"] == "resident"
    cols = np.array([0, 1, 63, 64, 127, 128, 200, 255])
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][cols], N, c=inst["c"])
    ev, es = _relcol(g["V"][:, cols], ref["V"]), _relcol(g["S"][:, cols], ref["S"])
    ej = float(np.max(np.abs(g["J"][cols] - ref["J"]) / ref["J"]))
    print("resident bench workload: V %.2e S %.2e J %.2e" % (ev, es, ej))
    assert max(ev, es, ej) <= BAR


def test_resident_permutation_and_split():
    inst = synth.round_to(synth.make_instance(256, 256, 24, seed=5), "f32")
    N = 900
    base = _run(inst, N, trace=False)
    perm = np.random.default_rng(1).permutation(24)
    pinst = dict(inst, mu=inst["mu"][perm])
    pg = _run(pinst, N, trace=False)
    for k in ("V", "S"):
        assert np.array_equal(pg[k], base[k][:, perm])
    assert np.array_equal(pg["J"], base["J"][perm])
    sp = _run(inst, N, trace=False, n_split=333)
    # the split run rounds the (hi, lo) state to FP32 once more
    assert _relcol(sp["V"], base["V"]) <= 1e-6 and _relcol(sp["S"], base["S"]) <= 1e-6


def test_resident_graph_replay_bitwise():
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(256, 256, 16, seed=8), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule="resident")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    V, S = rom.zeros(16)
    J = torch.zeros(16, dtype=torch.float64, device="cuda")
    rom.run_rank2(mu, V, S, 300, c=c, J=J)
    torch.cuda.synchronize()
    eager = [t.clone() for t in (V, S, J)]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rom.run_rank2(mu, V, S, 300, c=c, J=J, stream=s)
    for _ in range(3):
        V.zero_(); S.zero_(); J.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((V, S, J), eager):
            assert torch.equal(a, b)
    rom.close()


def test_resident_flag_on_non_skew_pair_falls_back():
    inst = synth.round_to(synth.make_instance(128, 128, 5, seed=9, skew=False), "f32")
    g = _run(inst, 200, trace=False)
    assert g["sched"] == "columns"
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 200, c=inst["c"])
    assert _relcol(g["V"], ref["V"]) <= BAR
