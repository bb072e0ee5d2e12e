"""Grouped runs with a row-split part: square FP32 instances with a padded
K that is a multiple of 64 in [128, 2048], each split into 64-sample groups
whose operator rows are spread over K / 64 workgroups of one XCD; groups of
different K share cooperative launches (8 XCDs x 32 workgroups), and the
instances below the plan's K threshold run in one column-block launch
after them.

Each instance of such a run must equal its own rank-2 run on the schedule
it ran on bitwise (same per-column arithmetic), and the FP64 oracle to the
FP32 bar (1e-5).  Every run is followed by the plan's barrier check.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _relcol(X, R):
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.linalg.norm(R, axis=0)))


def _setup(specs, schedule):
    """specs: (K, M, operator seed, mu seed); instances of one operator seed
    share operators but get their own contexts and samples."""
    from paper_2009_11742_amd import Rom
    ops, insts, roms, mus, Vs, Ss = {}, [], [], [], [], []
    for K, M, oseed, mseed in specs:
        if (K, oseed) not in ops:
            ops[(K, oseed)] = synth.round_to(synth.make_instance(K, K, 1, seed=oseed), "f32")
        base = ops[(K, oseed)]
        inst = dict(base)
        inst["mu"] = np.random.default_rng(mseed).uniform(0.5, 1.0, M)
        rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule=schedule)
        V, S = rom.zeros(M)
        insts.append(inst); roms.append(rom); Vs.append(V); Ss.append(S)
        mus.append(torch.tensor(inst["mu"], dtype=torch.float64, device="cuda"))
    return insts, roms, mus, Vs, Ss


def _standalone(inst, mu, nsteps, schedule):
    from paper_2009_11742_amd import Rom
    r = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule=schedule)
    V, S = r.zeros(int(mu.numel()))
    r.run_rank2(mu, V, S, nsteps)
    r.check()
    torch.cuda.synchronize()
    r.close()
    return V, S


def _close(roms, plan=None):
    if plan is not None:
        plan.close()
    for r in roms:
        r.close()


def test_split_plan_ragged_matches_standalone_and_oracle():
    """K = 256, ragged M (1 .. 130: 8 groups, one launch), forced row-split."""
    from paper_2009_11742_amd import GroupPlan
    specs = [(256, 64, 1, 10), (256, 100, 2, 11), (256, 1, 1, 12), (256, 130, 3, 13), (256, 30, 2, 14)]
    insts, roms, mus, Vs, Ss = _setup(specs, "rowsplit")
    N = 900
    plan = GroupPlan(roms, mus, Vs, Ss)
    assert plan.schedule == "rowsplit"
    plan.run(N)
    plan.check()
    torch.cuda.synchronize()
    for inst, mu, V, S in zip(insts, mus, Vs, Ss):
        V1, S1 = _standalone(inst, mu, N, "rowsplit")
        assert torch.equal(V, V1) and torch.equal(S, S1)
        r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N)
        e = max(_relcol(V.cpu().numpy().astype(np.float64).T, r["V"]),
                _relcol(S.cpu().numpy().astype(np.float64).T, r["S"]))
        print("split plan M=%d: err %.2e" % (len(inst["mu"]), e))
        assert e <= TOL
    # continuing runs (n0 offsets) equal one run up to the state rounding at the boundary
    for V, S in zip(Vs, Ss):
        V.zero_(); S.zero_()
    plan.run(400)
    plan.run(N - 400, n0=400)
    plan.check()
    torch.cuda.synchronize()
    for inst, V in zip(insts, Vs):
        r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N)
        assert _relcol(V.cpu().numpy().astype(np.float64).T, r["V"]) <= TOL
    _close(roms, plan)


def test_split_plan_several_launches():
    """K = 512 (32 groups per launch): 30 instances of 1 .. 100 samples over
    three operators, 41 groups, so two launches; every instance bitwise
    equal to its standalone row-split run, sampled columns against the
    oracle."""
    from paper_2009_11742_amd import run_grouped
    rng = np.random.default_rng(5)
    Ms = [int(m) for m in rng.integers(1, 101, 30)]
    specs = [(512, M, 20 + i % 3, 100 + i) for i, M in enumerate(Ms)]
    assert sum((M + 63) // 64 for M in Ms) > 32
    insts, roms, mus, Vs, Ss = _setup(specs, "rowsplit")
    N = 500
    run_grouped(roms, mus, Vs, Ss, N)
    torch.cuda.synchronize()
    for inst, mu, V, S in zip(insts, mus, Vs, Ss):
        V1, S1 = _standalone(inst, mu, N, "rowsplit")
        assert torch.equal(V, V1) and torch.equal(S, S1)
    picks = [0, 7, 15, 29]

    def check(i):
        inst = insts[i]
        col = len(inst["mu"]) - 1
        r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][col:col + 1], N)
        Vg = Vs[i].cpu().numpy().astype(np.float64).T[:, col:col + 1]
        Sg = Ss[i].cpu().numpy().astype(np.float64).T[:, col:col + 1]
        return max(_relcol(Vg, r["V"]), _relcol(Sg, r["S"]))

    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        errs = list(ex.map(check, picks))
    print("split plan, two launches: sampled errors", ["%.2e" % e for e in errs])
    assert max(errs) <= TOL
    _close(roms)


def test_auto_plan_is_timed_and_correct():
    """Unpinned contexts: the plan times both forms, keeps the faster, and
    its run equals the standalone runs of that schedule bitwise."""
    from paper_2009_11742_amd import GroupPlan
    specs = [(512, 64, 30 + i % 2, 200 + i) for i in range(12)]
    insts, roms, mus, Vs, Ss = _setup(specs, "auto")
    plan = GroupPlan(roms, mus, Vs, Ss)
    t = plan.times
    print("auto plan: %s, times %s" % (plan.schedule, t))
    assert t["columns"] is not None and t["rowsplit"] is not None
    assert plan.schedule == ("rowsplit" if t["rowsplit"] < t["columns"] else "columns")
    N = 300
    plan.run(N)
    plan.check()
    torch.cuda.synchronize()
    sched = plan.schedule
    for inst, mu, V, S in zip(insts, mus, Vs, Ss):
        V1, S1 = _standalone(inst, mu, N, sched)
        assert torch.equal(V, V1) and torch.equal(S, S1)
    # the decision is remembered: a second plan of the same shape does not time
    plan2 = GroupPlan(roms, mus, Vs, Ss)
    assert plan2.schedule == sched
    assert plan2.times == {"columns": None, "rowsplit": None}
    plan2.close()
    _close(roms, plan)


def test_columns_pin_keeps_column_plan():
    from paper_2009_11742_amd import GroupPlan
    specs = [(256, 64, 40, 300), (256, 64, 41, 301)]
    insts, roms, mus, Vs, Ss = _setup(specs, "columns")
    plan = GroupPlan(roms, mus, Vs, Ss)
    assert plan.schedule == "columns"
    _close(roms, plan)


def test_split_plan_graph_capture_uses_column_form():
    """A row-split plan captured into a graph records its column-block form:
    every replay equals the standalone column-block runs bitwise."""
    from paper_2009_11742_amd import GroupPlan
    specs = [(256, 70, 50, 400), (256, 20, 51, 401)]
    insts, roms, mus, Vs, Ss = _setup(specs, "rowsplit")
    plan = GroupPlan(roms, mus, Vs, Ss)
    assert plan.schedule == "rowsplit"
    N = 300
    ref = [_standalone(inst, mu, N, "columns") for inst, mu in zip(insts, mus)]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    for V, S in zip(Vs, Ss):
        V.zero_(); S.zero_()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        plan.run(N, stream=s)
    for rep in range(3):
        for V, S in zip(Vs, Ss):
            V.zero_(); S.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (V, S), (Vr, Sr) in zip(zip(Vs, Ss), ref):
            assert torch.equal(V, Vr) and torch.equal(S, Sr), rep
    del g
    _close(roms, plan)


def test_mixed_k_split_plan_matches_standalone():
    """Forced row-split over instances of seven padded K (128 .. 2048,
    ragged Kv = 700) and ragged M: groups of different K side by side in
    one launch, 18 groups of K = 704 (16 per launch) forcing a second
    launch that the smaller groups fill.  Every instance bitwise equal to
    its standalone row-split run; sampled columns against the oracle."""
    from paper_2009_11742_amd import GroupPlan
    specs = ([(700, 128, 60, 500 + i) for i in range(9)] + [(320, 64, 61, 520 + i) for i in range(6)] +
             [(128, 200, 62, 540), (128, 7, 62, 541), (448, 90, 63, 542), (2048, 64, 64, 543),
              (1024, 100, 65, 544), (192, 1, 66, 545)])
    insts, roms, mus, Vs, Ss = _setup(specs, "rowsplit")
    plan = GroupPlan(roms, mus, Vs, Ss)
    assert plan.schedule == "rowsplit" and plan.split_k == 128
    N = 300
    plan.run(N)
    plan.check()
    torch.cuda.synchronize()
    for inst, mu, V, S in zip(insts, mus, Vs, Ss):
        V1, S1 = _standalone(inst, mu, N, "rowsplit")
        assert torch.equal(V, V1) and torch.equal(S, S1), inst["Avs"].shape
    picks = [0, 9, 15, 16, 17, 18, 19, 20]

    def check(i):
        inst = insts[i]
        col = len(inst["mu"]) - 1
        r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][col:col + 1], N)
        Vg = Vs[i].cpu().numpy().astype(np.float64).T[:, col:col + 1]
        Sg = Ss[i].cpu().numpy().astype(np.float64).T[:, col:col + 1]
        return max(_relcol(Vg, r["V"]), _relcol(Sg, r["S"]))

    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        errs = list(ex.map(check, picks))
    print("mixed-K split plan: sampled errors", ["%.2e" % e for e in errs])
    assert max(errs) <= TOL
    _close(roms, plan)


def test_mixed_plan_auto_threshold():
    """Unpinned contexts of several K: the plan times column blocks alone
    and each K threshold, keeps the fastest; instances at or above the
    threshold equal their standalone row-split runs bitwise, the others
    their standalone column-block runs; a context pinned to column blocks
    stays there."""
    from paper_2009_11742_amd import GroupPlan, Rom
    specs = [(128, 40, 70, 600), (320, 100, 71, 601), (704, 130, 72, 602), (768, 64, 73, 603),
             (512, 300, 74, 604), (192, 17, 75, 605)]
    insts, roms, mus, Vs, Ss = _setup(specs, "auto")
    pinned = insts[5]
    roms[5].close()
    roms[5] = Rom(pinned["Avs"], pinned["Asv"], pinned["b"], pinned["dt"], state="f32", schedule="columns")
    plan = GroupPlan(roms, mus, Vs, Ss)
    t, k = plan.times, plan.split_k
    print("mixed auto plan: %s, split_k %d, times %s" % (plan.schedule, k, t))
    assert t["columns"] is not None
    assert (k > 0) == (plan.schedule == "rowsplit")
    if t["rowsplit"] is not None and t["rowsplit"] < t["columns"]:
        assert k > 0
    N = 300
    plan.run(N)
    plan.check()
    torch.cuda.synchronize()
    for i, (inst, mu, V, S) in enumerate(zip(insts, mus, Vs, Ss)):
        kp = -(-inst["Avs"].shape[0] // 64) * 64
        sched = "rowsplit" if (k > 0 and kp >= k and i != 5) else "columns"
        V1, S1 = _standalone(inst, mu, N, sched)
        assert torch.equal(V, V1) and torch.equal(S, S1), (i, sched)
    _close(roms, plan)
