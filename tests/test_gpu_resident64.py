"""Operator-resident schedule with FP64 states (skew pairs with Kv, Ks <=
128; other pairs with Kv_pad Ks_pad <= 8192): one sample per workgroup with
its operators in registers in FP64 (Avs alone for a skew pair, used for both
half-steps as Asv V = -Avs^T V; Avs and Asv^T otherwise), states held
redundantly in registers.

Parity against the FP64 oracle at the FP64 bar (1e-12, per-sample relative
l2 error of the final states; the probe QoI J and trace y relative): the
plain-method workload (K = 64, M = 8, 2000 steps) and every tile shape
(padded Kv, Ks in {64, 128}, square and rectangular), ragged sizes, one
sample; non-skew pairs (weighted transposes and an independent random Asv)
at the three tiles they take.  Structural checks: agreement with the
vector-ALU column blocks (ROM_SCHED_COLUMNS), a permutation of the samples
permutes the results bitwise, a run split in two (the second part with
n0 > 0) equals the whole run bitwise in V and S, graph replays equal the
eager run bitwise, pairs above the size limits keep the column blocks, and
BF16 operators with FP64 states (skew after rounding) agree with the column
blocks on the same rounded operators.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
BAR64 = 1e-12


def _relcol(X, R):
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.linalg.norm(R, axis=0)))


def _run(inst, N, mu_np=None, schedule="auto", trace=True, n_split=None, ops=None):
    """Run on FP64 states; returns states (K x M), J, y and the schedule."""
    from paper_2009_11742_amd import Rom
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f64", ops=ops, schedule=schedule)
    mu_np = inst["mu"] if mu_np is None else mu_np
    M = len(mu_np)
    mu = torch.tensor(mu_np, dtype=torch.float64, device="cuda")
    V, S = rom.zeros(M)
    c = torch.tensor(inst["c"], dtype=torch.float64, device="cuda")
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
    return {"V": V.cpu().numpy().T, "S": S.cpu().numpy().T, "J": J.cpu().numpy(),
            "y": None if y is None else y.cpu().numpy(), "sched": sched}


def _errors(g, ref):
    ev, es = _relcol(g["V"], ref["V"]), _relcol(g["S"], ref["S"])
    ej = float(np.max(np.abs(g["J"] - ref["J"]) / ref["J"]))
    ey = 0.0
    if g["y"] is not None:
        ey = float(np.max(np.linalg.norm(g["y"] - ref["y"], axis=0) / np.linalg.norm(ref["y"], axis=0)))
    return ev, es, ej, ey


# (64, 64, 8, 2000): the plain-method workload; the others cover the four
# tiles (4x4, 4x8, 8x4, 8x8 entries per thread), padding rows and columns,
# a single sample and tiny sizes.
@pytest.mark.parametrize("kv,ks,M,N", [(64, 64, 8, 2000), (128, 128, 9, 700), (100, 60, 3, 500),
                                       (40, 128, 5, 400), (128, 64, 4, 500), (64, 64, 1, 300), (5, 3, 2, 300)])
def test_resident64_parity(kv, ks, M, N):
    inst = synth.make_instance(kv, ks, M, seed=kv + 3 * ks + M)
    g = _run(inst, N)
    assert g["sched"] == "resident"
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"],
                           trace=True)
    e = _errors(g, ref)
    print("resident f64 K=(%d,%d) M=%d N=%d: V %.2e S %.2e J %.2e y %.2e" % ((kv, ks, M, N) + e))
    assert max(e) <= BAR64


# non-skew pairs: weighted transposes (the form of staggered finite-difference
# operators) and an independent random Asv, at the (64, 64), (128, 64) and
# (64, 128) tiles
@pytest.mark.parametrize("kv,ks,M,N,kind", [(64, 64, 8, 1500, "weighted"), (100, 60, 3, 500, "weighted"),
                                            (40, 128, 5, 400, "weighted"), (60, 50, 4, 60, "random")])
def test_resident64_non_skew_parity(kv, ks, M, N, kind):
    inst = synth.make_instance(kv, ks, M, seed=kv + ks + 5 * M, skew=False, random_asv=(kind == "random"))
    g = _run(inst, N)
    assert g["sched"] == "resident"
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"],
                           trace=True)
    e = _errors(g, ref)
    print("resident f64 %s K=(%d,%d) M=%d N=%d: V %.2e S %.2e J %.2e y %.2e" % ((kind, kv, ks, M, N) + e))
    assert max(e) <= BAR64


@pytest.mark.parametrize("skew", [True, False])
def test_resident64_agrees_with_vector_alu_columns(skew):
    inst = synth.make_instance(96, 60, 12, seed=21, skew=skew)
    a = _run(inst, 800)
    b = _run(inst, 800, schedule="columns")
    assert a["sched"] == "resident" and b["sched"] is None
    for key in ("V", "S"):
        d = np.linalg.norm(a[key] - b[key], axis=0) / np.linalg.norm(b[key], axis=0)
        assert float(np.max(d)) <= 1e-13, key
    assert float(np.max(np.abs(a["J"] - b["J"]) / b["J"])) <= 1e-13


def test_resident64_permutation_and_split():
    """A permutation of the samples permutes V, S, J and y bitwise; a run
    split at step 77 (the second part with n0 = 77, inside a forcing window)
    equals the whole run bitwise in V and S (the FP64 state carries no
    compensation term); J only changes its summation order."""
    inst = synth.make_instance(64, 64, 11, seed=31)
    N = 400
    whole = _run(inst, N)
    perm = np.random.default_rng(2).permutation(11)
    p = _run(inst, N, mu_np=inst["mu"][perm])
    for key in ("V", "S"):
        assert np.array_equal(p[key], whole[key][:, perm]), key
    assert np.array_equal(p["J"], whole["J"][perm]) and np.array_equal(p["y"], whole["y"][:, perm])
    split = _run(inst, N, trace=False, n_split=77)
    for key in ("V", "S"):
        assert np.array_equal(split[key], whole[key]), key
    assert float(np.max(np.abs(split["J"] - whole["J"]) / whole["J"])) <= 1e-14


def test_resident64_graph_replay_bitwise():
    from paper_2009_11742_amd import Rom
    inst = synth.make_instance(128, 128, 6, seed=41)
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f64")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    c = torch.tensor(inst["c"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(6)
    J = torch.zeros(6, dtype=torch.float64, device="cuda")
    rom.run_rank2(mu, V, S, 250, c=c, J=J)
    torch.cuda.synchronize()
    assert rom.last_schedule == "resident"
    eager = [t.clone() for t in (V, S, J)]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rom.run_rank2(mu, V, S, 250, c=c, J=J, stream=s)
    for _ in range(3):
        V.zero_(); S.zero_(); J.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((V, S, J), eager):
            assert torch.equal(a, b)
    rom.close()


@pytest.mark.parametrize("kv,ks,skew", [(128, 128, False), (70, 100, False), (130, 130, True), (64, 129, True)])
def test_resident64_not_applicable_keeps_the_column_blocks(kv, ks, skew):
    inst = synth.make_instance(kv, ks, 4, seed=51, skew=skew)
    g = _run(inst, 300, trace=False)
    assert g["sched"] is None
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 300, c=inst["c"])
    assert max(_relcol(g["V"], ref["V"]), _relcol(g["S"], ref["S"])) <= BAR64


def test_resident64_bf16_operators_agree_with_the_column_blocks():
    """BF16 rounding keeps a skew pair skew (round(-x) = -round(x)), so FP64
    states on BF16 operators take the resident kernel; it runs the same
    dequantised operators as the column blocks."""
    inst = synth.make_instance(64, 64, 7, seed=61)
    a = _run(inst, 600, ops="bf16")
    b = _run(inst, 600, ops="bf16", schedule="columns")
    assert a["sched"] == "resident" and b["sched"] is None
    for key in ("V", "S"):
        d = np.linalg.norm(a[key] - b[key], axis=0) / np.linalg.norm(b[key], axis=0)
        assert float(np.max(d)) <= 1e-13, key
