"""Panel schedule (FP32 operators and states, any Kv, Ks): one tiled
matrix-product launch per half-step, nothing resident between them; the
schedule FP32 runs take above the column blocks' LDS limit (Kv_pad + Ks_pad
> 4096), up to the K = 4096 of the paper's ROM scaling study (Sec. 4.2);
with few tiles the products are split over k ranges and summed by a
second launch.

Parity against the FP64 oracle on the same FP32-rounded inputs at the FP32
bar (1e-5, per-sample relative l2 error of the final states; J and the
probe trace y relative): pinned at small, ragged and rectangular sizes
(full oracle), and taken automatically at K = 2304, K = 4096 and a
rectangular Kv != Ks pair above the limit (sampled columns).  Structural
checks: a permutation of the samples permutes the results bitwise, a run
split in two equals the whole run to a rounding of the state, graph replays
equal the eager run bitwise, and a first run under capture is refused.

FP64 states take the same schedule on the FP64 matrix cores (from
Kv_pad + Ks_pad >= 768, or pinned): parity against the FP64 oracle at the
FP64 bar (1e-12), pinned and automatic, split and unsplit, and agreement
with the vector-ALU column blocks.
"""
BAR64 = 1e-12
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
BAR = 1e-5


def _relcol(X, R):
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.linalg.norm(R, axis=0)))


def _run(inst, N, mu_np=None, schedule="panel", trace=True, n_split=None, state="f32"):
    from paper_2009_11742_amd import Rom
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state=state, schedule=schedule)
    mu_np = inst["mu"] if mu_np is None else mu_np
    M = len(mu_np)
    mu = torch.tensor(mu_np, dtype=torch.float64, device="cuda")
    V, S = rom.zeros(M)
    c = torch.tensor(inst["c"], dtype=torch.float32 if state == "f32" else torch.float64, device="cuda")
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


def _errors(g, ref, cols=slice(None)):
    ev, es = _relcol(g["V"][:, cols], ref["V"]), _relcol(g["S"][:, cols], ref["S"])
    ej = float(np.max(np.abs(g["J"][cols] - ref["J"]) / ref["J"]))
    ey = 0.0
    if g["y"] is not None and "y" in ref:
        gy = g["y"][:, cols]
        ey = float(np.max(np.linalg.norm(gy - ref["y"], axis=0) / np.linalg.norm(ref["y"], axis=0)))
    return ev, es, ej, ey


# (256, 256): two row tiles, ragged samples; (200, 330) weighted (not skew)
# pair with Kv != Ks; (64, 64, 5): one tile, mostly padding; (130, 70, 3):
# rows just past one tile.
@pytest.mark.parametrize("kv,ks,M,N,skew", [(256, 256, 100, 400, True), (200, 330, 70, 300, False),
                                            (64, 64, 5, 500, True), (130, 70, 3, 300, False)])
def test_panel_parity_pinned(kv, ks, M, N, skew):
    inst = synth.round_to(synth.make_instance(kv, ks, M, seed=kv + 3 * ks + M, skew=skew), "f32")
    g = _run(inst, N)
    assert g["sched"] == "panel"
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"],
                           trace=True)
    e = _errors(g, ref)
    print("panel K=(%d,%d) M=%d N=%d: V %.2e S %.2e J %.2e y %.2e" % ((kv, ks, M, N) + e))
    assert max(e) <= BAR


@pytest.mark.parametrize("kv,ks,M,N,skew,cols", [
    (2304, 2304, 96, 150, True, [0, 1, 31, 32, 63, 64, 90, 95]),
    (2200, 2000, 33, 100, False, [0, 7, 16, 31, 32]),
    (4096, 4096, 64, 20, True, [0, 21, 42, 63]),
    (2176, 2048, 1000, 30, False, [0, 333, 640, 999]),
])
def test_panel_large_k_sampled(kv, ks, M, N, skew, cols):
    """Above the column blocks' limit the run takes the panel schedule
    without being asked; all samples are stepped, `cols` checked.  With
    few tiles the products are split over k ranges and a second launch
    sums the partials and updates: 8 ways at K = 2304, M = 96, at
    2200 x 2000, M = 33 and at K = 4096, M = 64; at 2176 x 2048, M = 1000
    the velocity half-step (272 tiles) 4 ways while the stress half-step
    (256 tiles) runs whole."""
    inst = synth.round_to(synth.make_instance(kv, ks, M, seed=kv + ks, skew=skew), "f32")
    g = _run(inst, N, schedule="auto")
    assert g["sched"] == "panel"
    cols = np.array(cols)
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][cols], N, c=inst["c"],
                           trace=True)
    e = _errors(g, ref, cols)
    print("panel K=(%d,%d) M=%d N=%d sampled: V %.2e S %.2e J %.2e y %.2e" % ((kv, ks, M, N) + e))
    assert max(e) <= BAR
    assert np.all(np.isfinite(g["V"])) and np.all(np.isfinite(g["S"]))


def test_panel_permutation_and_split():
    inst = synth.round_to(synth.make_instance(300, 300, 70, seed=11), "f32")
    N = 300
    whole = _run(inst, N)
    perm = np.random.default_rng(3).permutation(70)
    p = _run(inst, N, mu_np=inst["mu"][perm])
    for key in ("V", "S"):
        assert np.array_equal(p[key], whole[key][:, perm]), key
    assert np.array_equal(p["J"], whole["J"][perm]) and np.array_equal(p["y"], whole["y"][:, perm])
    split = _run(inst, N, trace=False, n_split=137)
    for key in ("V", "S"):
        d = np.linalg.norm(split[key] - whole[key], axis=0) / np.linalg.norm(whole[key], axis=0)
        assert float(np.max(d)) <= 1e-6, key
    assert float(np.max(np.abs(split["J"] - whole["J"]) / whole["J"])) <= 1e-6


def test_panel_graph_replay_bitwise_and_first_run_not_captured():
    from paper_2009_11742_amd import Rom, _lib
    inst = synth.round_to(synth.make_instance(192, 160, 40, seed=12, skew=False), "f32")
    M, N = 40, 60
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule="panel")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    V, S = rom.zeros(M)
    J = torch.zeros(M, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    # no workspace yet: the captured run is refused before anything is enqueued
    with pytest.raises(_lib.RomError) as ei:
        with torch.cuda.graph(g, stream=s):
            rom.run_rank2(mu, V, S, N, c=c, J=J)
    assert ei.value.status == _lib.ROM_E_UNSUPPORTED
    torch.cuda.synchronize()
    # eager reference, which also allocates the workspace
    V0 = torch.tensor(np.asarray(inst["b"][:, None] * 1e-3 * np.ones((1, M)), dtype=np.float32).T.copy(),
                      device="cuda")
    V.copy_(V0); S.zero_(); J.zero_()
    rom.run_rank2(mu, V, S, N, c=c, J=J)
    torch.cuda.synchronize()
    ref = [V.clone(), S.clone(), J.clone()]
    g = torch.cuda.CUDAGraph()
    V.copy_(V0); S.zero_(); J.zero_()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        rom.run_rank2(mu, V, S, N, c=c, J=J)
    for rep in range(3):
        V.copy_(V0); S.zero_(); J.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((V, S, J), ref):
            assert torch.equal(a, b), rep
        # eager work between replays
        rom.run_rank2(mu, V, S, 3, c=c, J=J)
        torch.cuda.synchronize()
    rom.close()


@pytest.mark.parametrize("kv,ks,M,N,skew", [(256, 256, 100, 400, True), (200, 330, 70, 300, False),
                                            (130, 70, 3, 300, False)])
def test_panel_f64_parity_pinned(kv, ks, M, N, skew):
    inst = synth.make_instance(kv, ks, M, seed=kv + 5 * ks + M, skew=skew)
    g = _run(inst, N, state="f64")
    assert g["sched"] == "panel"
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"],
                           trace=True)
    e = _errors(g, ref)
    print("panel f64 K=(%d,%d) M=%d N=%d: V %.2e S %.2e J %.2e y %.2e" % ((kv, ks, M, N) + e))
    assert max(e) <= BAR64


@pytest.mark.parametrize("kv,ks,M,N,cols", [(512, 512, 300, 200, [0, 150, 299]),
                                            (2304, 2304, 96, 60, [0, 33, 95])])
def test_panel_f64_auto_sampled(kv, ks, M, N, cols):
    """FP64 runs from Kv_pad + Ks_pad = 768 take the panel schedule
    unasked (K = 2304, M = 96: 8 k-range splits)."""
    inst = synth.make_instance(kv, ks, M, seed=kv + M)
    g = _run(inst, N, schedule="auto", state="f64")
    assert g["sched"] == "panel"
    cols = np.array(cols)
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][cols], N, c=inst["c"],
                           trace=True)
    e = _errors(g, ref, cols)
    print("panel f64 K=(%d,%d) M=%d N=%d sampled: V %.2e S %.2e J %.2e y %.2e" % ((kv, ks, M, N) + e))
    assert max(e) <= BAR64


def test_panel_f64_agrees_with_vector_alu_columns():
    inst = synth.make_instance(384, 384, 40, seed=9)
    a = _run(inst, 300, state="f64", schedule="panel")
    b = _run(inst, 300, state="f64", schedule="columns")
    assert a["sched"] == "panel" and b["sched"] is None
    for key in ("V", "S"):
        d = np.linalg.norm(a[key] - b[key], axis=0) / np.linalg.norm(b[key], axis=0)
        assert float(np.max(d)) <= 1e-13, key
    assert float(np.max(np.abs(a["J"] - b["J"]) / b["J"])) <= 1e-13


def test_panel_f64_permutation_split_and_offset():
    """FP64 panel runs: a sample permutation permutes the results bitwise;
    a run split at step 91 (the second part with n0 = 91) equals the whole
    run to FP64 rounding (the FP64 state carries no compensation term, so
    only the order of the J sums differs)."""
    inst = synth.make_instance(600, 600, 70, seed=13)        # Kv_pad + Ks_pad = 1280: automatic, 2 splits
    N = 200
    whole = _run(inst, N, state="f64", schedule="auto")
    assert whole["sched"] == "panel"
    perm = np.random.default_rng(4).permutation(70)
    p = _run(inst, N, mu_np=inst["mu"][perm], state="f64", schedule="auto")
    for key in ("V", "S"):
        assert np.array_equal(p[key], whole[key][:, perm]), key
    assert np.array_equal(p["J"], whole["J"][perm]) and np.array_equal(p["y"], whole["y"][:, perm])
    split = _run(inst, N, trace=False, n_split=91, state="f64", schedule="auto")
    for key in ("V", "S"):
        assert np.array_equal(split[key], whole[key]), key
    assert float(np.max(np.abs(split["J"] - whole["J"]) / whole["J"])) <= 1e-14


def test_panel_f64_capture_before_and_after_the_workspace():
    """An FP64 run that would take the panel schedule, captured into a graph
    before any panel run of the context, stays on the vector-ALU column
    blocks (it cannot allocate under capture), bitwise equal to an eager
    run pinned there; after an eager panel run the captured run takes the
    panel schedule, bitwise equal to its eager run."""
    from paper_2009_11742_amd import Rom
    inst = synth.make_instance(400, 400, 12, seed=14)
    M, N = 12, 50
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()

    def eager(schedule):
        rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f64", schedule=schedule)
        V, S = rom.zeros(M)
        V.fill_(1e-3)
        rom.run_rank2(mu, V, S, N)
        torch.cuda.synchronize()
        out = (V.clone(), S.clone(), rom.last_schedule)
        rom.close()
        return out

    ref_cols, ref_panel = eager("columns"), eager("auto")
    assert ref_cols[2] is None and ref_panel[2] == "panel"
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f64")
    V, S = rom.zeros(M)
    for want, ref in ((None, ref_cols), ("panel", ref_panel)):
        g = torch.cuda.CUDAGraph()
        V.fill_(1e-3); S.zero_()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            rom.run_rank2(mu, V, S, N)
        assert rom.last_schedule == want
        for rep in range(2):
            V.fill_(1e-3); S.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(V, ref[0]) and torch.equal(S, ref[1]), (want, rep)
        if want is None:
            V.fill_(1e-3); S.zero_()
            rom.run_rank2(mu, V, S, N)          # eager: sets the panel workspace up
            torch.cuda.synchronize()
            assert rom.last_schedule == "panel"
    rom.close()
