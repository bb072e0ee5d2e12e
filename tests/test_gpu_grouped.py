"""Grouped runs: many ROM instances of uneven sizes in one launch.

Each instance of a grouped run must equal its own rank-2 run bitwise (same
per-column arithmetic) on the schedule it ran on, and the FP64 oracle to
the FP32 bar (1e-5).  With unpinned contexts a plan may put the square
instances from a padded-K threshold up (GroupPlan.split_k) on row-split
launches and the rest on column blocks; a graph-captured run takes column
blocks for all.
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


def _setup(specs):
    from paper_2009_11742_amd import Rom
    insts, roms, mus, Vs, Ss = [], [], [], [], []
    for kv, ks, M, seed in specs:
        inst = synth.round_to(synth.make_instance(kv, ks, M, seed=seed, skew=(kv == ks)), "f32")
        rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
        V, S = rom.zeros(M)
        insts.append(inst); roms.append(rom); Vs.append(V); Ss.append(S)
        mus.append(torch.tensor(inst["mu"], dtype=torch.float64, device="cuda"))
    return insts, roms, mus, Vs, Ss


def _standalone(inst, mu, nsteps, schedule="columns"):
    """The instance's own rank-2 run on `schedule` (4-column blocks by
    default; a fresh context from the same inputs packs the same
    operators)."""
    from paper_2009_11742_amd import Rom
    r = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule=schedule)
    V, S = r.zeros(int(mu.numel()))
    r.run_rank2(mu, V, S, nsteps)
    r.check()
    torch.cuda.synchronize()
    r.close()
    return V, S


def _schedule_in_plan(inst, split_k):
    """Schedule an unpinned instance ran on in a plan with threshold split_k."""
    kv, ks = inst["Avs"].shape
    kp = -(-kv // 64) * 64
    return "rowsplit" if split_k > 0 and kv == ks and kp >= split_k else "columns"


SMALL = [(64, 64, 5, 1), (128, 96, 17, 2), (256, 256, 9, 3), (33, 70, 3, 4), (192, 192, 40, 5)]


def test_grouped_small_matches_standalone_and_oracle():
    from paper_2009_11742_amd import GroupPlan
    insts, roms, mus, Vs, Ss = _setup(SMALL)
    N = 1200
    plan = GroupPlan(roms, mus, Vs, Ss)
    plan.run(N)
    plan.check()
    torch.cuda.synchronize()
    k = plan.split_k
    plan.close()
    for inst, rom, mu, V, S in zip(insts, roms, mus, Vs, Ss):
        V1, S1 = _standalone(inst, mu, N, _schedule_in_plan(inst, k))
        assert torch.equal(V, V1) and torch.equal(S, S1)
        r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N)
        assert _relcol(V.cpu().numpy().astype(np.float64).T, r["V"]) <= TOL
        assert _relcol(S.cpu().numpy().astype(np.float64).T, r["S"]) <= TOL


def test_grouped_plan_graph_capture_replays():
    from paper_2009_11742_amd import GroupPlan
    insts, roms, mus, Vs, Ss = _setup(SMALL[:3])
    N = 300
    plan = GroupPlan(roms, mus, Vs, Ss)
    # a captured run takes column blocks for every instance
    ref = [_standalone(inst, mu, N) for inst, mu in zip(insts, mus)]
    g = torch.cuda.CUDAGraph()
    for V, S in zip(Vs, Ss):
        V.zero_(); S.zero_()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.run(N)
    for rep in range(3):
        for V, S in zip(Vs, Ss):
            V.zero_(); S.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (V, S), (Vr, Sr) in zip(zip(Vs, Ss), ref):
            assert torch.equal(V, Vr) and torch.equal(S, Sr), rep
    # a plan run continues from the current state (n0 offset)
    for V, S in zip(Vs, Ss):
        V.zero_(); S.zero_()
    plan.run(100)
    plan.run(200, n0=100)
    torch.cuda.synchronize()
    for (V, S), (Vr, Sr), inst in zip(zip(Vs, Ss), ref, insts):
        r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N)
        assert _relcol(V.cpu().numpy().astype(np.float64).T, r["V"]) <= TOL
    plan.close()


def test_grouped_full_workload():
    """64 instances, K uniform in {128, ..., 768}, M log-uniform in [16, 512],
    4000 steps, on the plan the library picks (timed threshold): every
    instance bitwise equal to its standalone run on the schedule it ran on;
    sampled columns of 8 instances within 1e-5 of the oracle."""
    from paper_2009_11742_amd import GroupPlan
    draws = synth.grouped_draws(64, base_seed=0)
    specs = [(K, K, M, seed) for K, M, seed in draws]
    insts, roms, mus, Vs, Ss = _setup(specs)
    N = 4000
    plan = GroupPlan(roms, mus, Vs, Ss)
    k = plan.split_k
    print("grouped full workload: split_k %d, times %s" % (k, plan.times))
    plan.run(N)
    plan.check()
    torch.cuda.synchronize()
    plan.close()
    for inst, mu, V, S in zip(insts, mus, Vs, Ss):
        V1, S1 = _standalone(inst, mu, N, _schedule_in_plan(inst, k))
        assert torch.equal(V, V1) and torch.equal(S, S1)
    picks = np.linspace(0, 63, 8).round().astype(int)

    def check(i):
        inst = insts[i]
        col = len(inst["mu"]) // 2
        r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][col:col + 1], N)
        Vg = Vs[i].cpu().numpy().astype(np.float64).T[:, col:col + 1]
        Sg = Ss[i].cpu().numpy().astype(np.float64).T[:, col:col + 1]
        return max(_relcol(Vg, r["V"]), _relcol(Sg, r["S"]))

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        errs = list(ex.map(check, picks))
    print("grouped sampled errors", ["%.2e" % e for e in errs])
    assert max(errs) <= TOL


@pytest.mark.parametrize("tile_small,tile_big", [("columns", "columns8"), ("columns8", "columns")])
def test_grouped_tiles_from_table(tile_small, tile_big):
    """The grouped plan takes each instance's tile from the table's
    per-workgroup entries: forcing 8-column tiles on one K bucket and 4 on
    the other, every instance still equals its standalone run bitwise."""
    from paper_2009_11742_amd import run_grouped, tuning
    saved = tuning.entries()
    try:
        tuning.clear()
        # us = (4-column, -, 8-column) per-workgroup step times; 8 wins when t8 < 2 t4
        fast8, slow8 = [10.0, -1.0, 12.0], [10.0, -1.0, 30.0]
        tuning.put(128, 128, 0, "f32", tile_small, fast8 if tile_small == "columns8" else slow8)
        tuning.put(320, 320, 0, "f32", tile_big, fast8 if tile_big == "columns8" else slow8)
        # Kv != Ks: never on row-split, so the plan is all column blocks
        specs = [(128, 120, 37, 11), (300, 290, 21, 12), (128, 124, 8, 13), (300, 296, 5, 14)]
        insts, roms, mus, Vs, Ss = _setup(specs)
        N = 600
        run_grouped(roms, mus, Vs, Ss, N)
        torch.cuda.synchronize()
        for inst, mu, V, S in zip(insts, mus, Vs, Ss):
            V1, S1 = _standalone(inst, mu, N)
            assert torch.equal(V, V1) and torch.equal(S, S1)
            r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N)
            assert _relcol(V.cpu().numpy().astype(np.float64).T, r["V"]) <= TOL
    finally:
        tuning.clear()
        for d in saved:
            tuning.put(d["kv_pad"], d["ks_pad"], d["m_pad"], d["op"], d["schedule"], d["us"])
