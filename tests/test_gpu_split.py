"""Row-split schedule of the FP32-state rank-2 run (FP32, BF16 and FP8
operators): operator rows split over the workgroups of a sample group (64
samples with BF16 / FP8 operators; with FP32 the narrowest of 16, 32 and 64
that fits the chip), exchanged every half-step.

BF16 / FP8: parity against the same-input FP64 oracle (the operators exactly
as the products use them), with the bar of the column-block low-precision
kernel: each state value enters the products as a BF16 (hi, lo) pair
(~2^-17 relative), which random-walks to ~1e-4 over a few thousand steps;
the bar is lowp_bars.pair_bar(N) = 6e-6 sqrt(N), three times that walk.
FP32: the FP32 bar, 1e-5.  Every run is followed by rom_check (no barrier
timed out).
"""
import concurrent.futures as cf

import numpy as np
import pytest

import lowp_bars
import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
bar_of = lowp_bars.pair_bar


def _relcol(X, R):
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.linalg.norm(R, axis=0)))


def _run(inst, ops, N, schedule, probe=True, trace=False, n_split=None):
    from paper_2009_11742_amd import Rom
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", ops=ops, schedule=schedule)
    M = len(inst["mu"])
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(M)
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda") if probe else None
    J = torch.zeros(M, dtype=torch.float64, device="cuda") if probe else None
    y = torch.zeros((N, M), dtype=torch.float64, device="cuda") if trace else None
    if n_split is None:
        rom.run_rank2(mu, V, S, N, c=c, J=J, y=y)
    else:
        rom.run_rank2(mu, V, S, n_split, c=c, J=J)
        rom.run_rank2(mu, V, S, N - n_split, n0=n_split, c=c, J=J)
    rom.check()
    A, B, _ = rom.operators()
    out = {"V": V.cpu().numpy().astype(np.float64).T, "S": S.cpu().numpy().astype(np.float64).T,
           "J": J.cpu().numpy() if probe else None, "y": y.cpu().numpy() if trace else None, "A": A, "B": B,
           "schedule": rom.last_schedule}
    rom.close()
    return out


# (256, 100): 16-sample groups whose exchange reads (32 KB per half-step)
# fit in a CU's L1 -- the case that caught exchange lines served stale from
# the L1 when the barrier's invalidate did not reach it.
# K = 100, 330, 740: padded K 128, 384, 768 (one, three and six k-blocks of 32
# terms per wave; 6 and 12 workgroups per group, so 2 to 8 CUs of each XCD
# idle), with zero rows padding the operators.
@pytest.mark.parametrize("ops", ["bf16", "fp8"])
@pytest.mark.parametrize("K,M,N", [(256, 100, 1500), (512, 64, 800), (256, 200, 600),
                                   (100, 40, 900), (330, 90, 700), (740, 70, 500)])
def test_rowsplit_same_input_parity(ops, K, M, N):
    inst = synth.round_to(synth.make_instance(K, K, M, seed=K + M), "f32")
    g = _run(inst, ops, N, "rowsplit", trace=True)
    assert g["schedule"] == "rowsplit"
    ref = oracle.run_rank2(g["A"], g["B"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"], trace=True)
    e = max(_relcol(g["V"], ref["V"]), _relcol(g["S"], ref["S"]))
    eJ = float(np.max(np.abs(g["J"] - ref["J"]) / ref["J"]))
    ey = float(np.max(np.abs(g["y"] - ref["y"])) / np.max(np.abs(ref["y"])))
    print("rowsplit %s K=%d M=%d N=%d: state %.2e  J %.2e  y %.2e" % (ops, K, M, N, e, eJ, ey))
    assert e <= bar_of(N) and eJ <= bar_of(N) and ey <= bar_of(N)
    assert np.all(np.isfinite(g["V"])) and np.all(np.isfinite(g["S"]))


@pytest.mark.parametrize("ops", ["bf16", "fp8"])
def test_rowsplit_agrees_with_column_block(ops):
    """Both schedules integrate the same rounded model: each within the bar
    of the same-input oracle and of each other."""
    inst = synth.round_to(synth.make_instance(256, 256, 70, seed=11), "f32")
    N = 1000
    a = _run(inst, ops, N, "rowsplit")
    b = _run(inst, ops, N, "columns")
    assert np.array_equal(a["A"], b["A"]) and np.array_equal(a["B"], b["B"])
    ref = oracle.run_rank2(a["A"], a["B"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"])
    for g in (a, b):
        assert max(_relcol(g["V"], ref["V"]), _relcol(g["S"], ref["S"])) <= bar_of(N)
    assert _relcol(a["V"], b["V"]) <= 2 * bar_of(N)


def test_rowsplit_run_split_and_offset():
    """Two runs (n0 = 0 and n0 = 400) equal one run of 1000 steps up to the
    state rounding at the boundary."""
    inst = synth.round_to(synth.make_instance(256, 256, 64, seed=5), "f32")
    N = 1000
    one = _run(inst, "bf16", N, "rowsplit")
    two = _run(inst, "bf16", N, "rowsplit", n_split=400)
    ref = oracle.run_rank2(one["A"], one["B"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"])
    assert _relcol(two["V"], one["V"]) <= 1e-4
    assert max(_relcol(two["V"], ref["V"]), _relcol(two["S"], ref["S"])) <= bar_of(N)
    assert float(np.max(np.abs(two["J"] - ref["J"]) / ref["J"])) <= bar_of(N)


def test_rowsplit_k1024_m1024_sampled():
    """K = M = 1024 (the precision workload's shape), 600 steps, BF16 and
    FP8: three sampled columns against the same-input oracle."""
    inst = synth.round_to(synth.make_instance(1024, 1024, 1024, seed=0), "f32")
    N = 600
    cols = np.array([0, 517, 1023])
    for ops in ("bf16", "fp8"):
        g = _run(inst, ops, N, "rowsplit")

        def ref(ci):
            return oracle.run_rank2(g["A"], g["B"], inst["b"], inst["dt"], inst["mu"][ci:ci + 1], N, c=inst["c"])
        with cf.ThreadPoolExecutor(max_workers=3) as ex:
            refs = list(ex.map(ref, cols))
        e = max(max(_relcol(g["V"][:, ci:ci + 1], r["V"]), _relcol(g["S"][:, ci:ci + 1], r["S"]))
                for ci, r in zip(cols, refs))
        eJ = max(abs(g["J"][ci] - r["J"][0]) / r["J"][0] for ci, r in zip(cols, refs))
        print("rowsplit %s K=M=1024 N=%d sampled: state %.2e J %.2e" % (ops, N, e, eJ))
        assert e <= bar_of(N) and eJ <= bar_of(N)


# ---- FP32 operators (row-split FP32 kernel): the FP32 bar, 1e-5
F32_BAR = 1e-5


@pytest.mark.parametrize("K,M,N", [(256, 100, 2000), (512, 130, 1000)])
def test_rowsplit_f32_parity(K, M, N):
    inst = synth.round_to(synth.make_instance(K, K, M, seed=2 * K + M), "f32")
    g = _run(inst, "f32", N, "rowsplit", trace=True)
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"], trace=True)
    e = max(_relcol(g["V"], ref["V"]), _relcol(g["S"], ref["S"]))
    eJ = float(np.max(np.abs(g["J"] - ref["J"]) / ref["J"]))
    ey = float(np.max(np.abs(g["y"] - ref["y"])) / np.max(np.abs(ref["y"])))
    print("rowsplit f32 K=%d M=%d N=%d: state %.2e  J %.2e  y %.2e" % (K, M, N, e, eJ, ey))
    assert e <= F32_BAR and eJ <= F32_BAR and ey <= F32_BAR


# Any padded K that is a multiple of 64 from 128 to 2048 (the k-group count
# of the FP32 kernel taken at run time; a group's K / 64 workgroups on one
# XCD, so 8 floor(32 / (K / 64)) groups per launch): ragged K, R that does
# not divide 32, and the largest K (one group per XCD).  Sampled columns
# against the oracle where it would take long.
@pytest.mark.parametrize("K,M,N,cols", [(128, 50, 800, None), (320, 70, 600, None), (700, 33, 500, None),
                                        (1216, 20, 300, (0, 19)), (2048, 70, 300, (0, 69))])
def test_rowsplit_f32_any_k_parity(K, M, N, cols):
    inst = synth.round_to(synth.make_instance(K, K, M, seed=3 * K + M), "f32")
    g = _run(inst, "f32", N, "rowsplit", trace=True)
    sel = np.arange(M) if cols is None else np.array(cols)
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][sel], N, c=inst["c"],
                           trace=True)
    e = max(_relcol(g["V"][:, sel], ref["V"]), _relcol(g["S"][:, sel], ref["S"]))
    eJ = float(np.max(np.abs(g["J"][sel] - ref["J"]) / ref["J"]))
    ey = float(np.max(np.abs(g["y"][:, sel] - ref["y"])) / np.max(np.abs(ref["y"])))
    print("rowsplit f32 K=%d M=%d N=%d: state %.2e  J %.2e  y %.2e" % (K, M, N, e, eJ, ey))
    assert e <= F32_BAR and eJ <= F32_BAR and ey <= F32_BAR


def test_rowsplit_f32_any_k_schedule_and_limits():
    """The autotuner may pick row-split at any eligible K; beyond one launch
    (K = 2048: 8 groups of 64, so M > 512) or above K = 2048 the run takes
    column blocks."""
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(2048, 2048, 600, seed=4), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule="rowsplit")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(600)
    rom.run_rank2(mu, V, S, 3)
    rom.check()
    assert rom.last_schedule == "columns"
    V, S = rom.zeros(512)
    rom.run_rank2(mu[:512], V, S, 3)
    rom.check()
    assert rom.last_schedule == "rowsplit"
    rom.close()


@pytest.mark.parametrize("ops,K,Ms", [("f32", 256, (1000, 2000, 4000)), ("f32", 512, (500, 1000, 2000)),
                                      ("f32", 1024, (250, 500, 1000)), ("f32", 320, (700, 1500, 3000)),
                                      ("bf16", 512, (500, 1000, 2000)), ("bf16", 1024, (250, 500, 1000))])
def test_rowsplit_group_width_bitwise(ops, K, Ms):
    """Row-split runs take the narrowest column group (16, 32 or 64
    samples) whose groups all fit in one launch (8 floor(32 / (K / 64)));
    the Ms here select the three widths in turn.  A column's state arithmetic does
    not depend on the width, so the shared samples (a prefix of the same mu)
    agree bitwise in V and S; the probe's FP64 row sum is spread over 4 NCB
    rows per thread and a shuffle tree over 16 / NCB threads, and so is the
    sum of the row-tile partials, so J and the trace agree to FP64
    reassociation (1e-14)."""
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(K, K, max(Ms), seed=K + 5), "f32")
    N = 120
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", ops=ops, schedule="rowsplit")
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    outs = []
    for M in Ms:
        mu = torch.tensor(inst["mu"][:M], dtype=torch.float64, device="cuda")
        V, S = rom.zeros(M)
        J = torch.zeros(M, dtype=torch.float64, device="cuda")
        y = torch.zeros((N, M), dtype=torch.float64, device="cuda")
        rom.run_rank2(mu, V, S, N, c=c, J=J, y=y)
        rom.check()
        assert rom.last_schedule == "rowsplit"
        outs.append((V.cpu().numpy(), S.cpu().numpy(), J.cpu().numpy(), y.cpu().numpy()))
    m0 = Ms[0]
    for V, S, J, y in outs[1:]:
        assert np.array_equal(V[:m0], outs[0][0]) and np.array_equal(S[:m0], outs[0][1])
        assert np.allclose(J[:m0], outs[0][2], rtol=1e-14, atol=0)
        assert np.max(np.abs(y[:, :m0] - outs[0][3])) <= 1e-14 * np.max(np.abs(outs[0][3]))
    cols = np.array([0, m0 // 2, m0 - 1])
    A, B, _ = rom.operators()
    rom.close()
    bar = F32_BAR if ops == "f32" else bar_of(N)
    for ci in cols:
        r = oracle.run_rank2(A, B, inst["b"], inst["dt"], inst["mu"][ci:ci + 1], N, c=inst["c"])
        g = outs[0]
        assert _relcol(g[0][ci:ci + 1].astype(np.float64).T, r["V"]) <= bar
        assert abs(g[2][ci] - r["J"][0]) <= bar * r["J"][0]


def test_rowsplit_f32_k1024_m1024_sampled():
    inst = synth.round_to(synth.make_instance(1024, 1024, 1024, seed=0), "f32")
    N = 600
    cols = np.array([0, 333, 1023])
    g = _run(inst, "f32", N, "auto")

    def ref(ci):
        return oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][ci:ci + 1], N, c=inst["c"])
    with cf.ThreadPoolExecutor(max_workers=3) as ex:
        refs = list(ex.map(ref, cols))
    e = max(max(_relcol(g["V"][:, ci:ci + 1], r["V"]), _relcol(g["S"][:, ci:ci + 1], r["S"]))
            for ci, r in zip(cols, refs))
    eJ = max(abs(g["J"][ci] - r["J"][0]) / r["J"][0] for ci, r in zip(cols, refs))
    print("rowsplit f32 K=M=1024 N=%d sampled: state %.2e J %.2e" % (N, e, eJ))
    assert e <= F32_BAR and eJ <= F32_BAR


@pytest.mark.parametrize("K,M,ops", [(1024, 1024, "f32"), (256, 256, "f32"), (512, 512, "bf16"), (2048, 1024, "f32")])
def test_schedule_autotuner(K, M, ops):
    """Without a schedule flag the first run of a shape times every schedule
    that applies and keeps the fastest (or takes the table's entry); the run
    uses it and is correct."""
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(K, K, M, seed=7), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", ops=ops)
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(M)
    N = 200
    rom.run_rank2(mu, V, S, N)
    rom.check()
    t = rom.schedule_times(M)
    chosen = rom.last_schedule
    print("autotuner K=%d M=%d %s: %s -> %s" % (K, M, ops, t, chosen))
    timed = {k: v for k, v in t.items() if v is not None}
    assert chosen == min(timed, key=timed.get)
    if K <= 1024:                  # the 8-column blocks' states fit in LDS
        assert (t["columns8"] is None) == (ops != "f32")
    if (K, M) == (2048, 1024):
        # beyond one row-split launch: column blocks against the panel
        # schedule, both timed
        assert t["rowsplit"] is None and t["panel"] is not None and t["columns"] is not None
    A, B, _ = rom.operators()
    col = M // 3
    r = oracle.run_rank2(A, B, inst["b"], inst["dt"], inst["mu"][col:col + 1], N)
    bar = F32_BAR if ops == "f32" else bar_of(N)
    assert _relcol(V.cpu().numpy().astype(np.float64).T[:, col:col + 1], r["V"]) <= bar
    rom.close()


def test_online_tuning_and_table_entries_steer_the_schedule():
    """An empty table is filled by the first run of a shape; an entry put in
    the table decides the schedule of later runs of that shape."""
    from paper_2009_11742_amd import Rom, tuning
    saved = tuning.entries()
    try:
        tuning.clear()
        K, M, N = 256, 100, 300
        inst = synth.round_to(synth.make_instance(K, K, M, seed=3), "f32")
        rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
        mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
        V, S = rom.zeros(M)
        rom.run_rank2(mu, V, S, N)
        rom.check()
        e = [d for d in tuning.entries() if d["m_pad"] == 128]
        # every schedule timed but the panel one, not weighed below Kv_pad + Ks_pad = 2048
        assert len(e) == 1 and all(u > 0 for u in e[0]["us"][:4]) and e[0]["us"][4] < 0, e
        ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N)
        outs = {}
        for sched in ("rowsplit", "columns8", "columns"):
            tuning.put(K, K, 128, "f32", sched, e[0]["us"])
            V, S = rom.zeros(M)
            rom.run_rank2(mu, V, S, N)
            rom.check()
            assert rom.last_schedule == sched
            outs[sched] = V.clone()
            assert _relcol(V.cpu().numpy().astype(np.float64).T, ref["V"]) <= F32_BAR
        assert torch.equal(outs["columns"], outs["columns8"])
        rom.close()
    finally:
        tuning.clear()
        for d in saved:
            tuning.put(d["kv_pad"], d["ks_pad"], d["m_pad"], d["op"], d["schedule"], d["us"])
