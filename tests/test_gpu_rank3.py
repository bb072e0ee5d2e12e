"""Affine operator families (rank-3 direction): operators assembled on the
device from their affine terms, run together in one grouped launch.

* The assembled operators equal the oracle's FP64 sum (same order) rounded
  as rom_create rounds host operators, bitwise (the build does not contract).
* Each instance of a grouped rank-3 run equals, bitwise, the standalone run
  of a context created from the host-assembled operators, and is within the
  FP32 bar (1e-5) of the FP64 oracle on the same operators.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _terms(kv, ks, Q, seed, skew):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((Q, kv, ks)) / np.sqrt(ks)
    if skew:
        B = -np.transpose(A, (0, 2, 1)).copy()
    else:
        w = rng.uniform(0.5, 1.5, size=ks)
        B = -(w[None, :, None] * np.transpose(A, (0, 2, 1)))
    b = rng.standard_normal(kv)
    return A, B, b


def _assemble(T, theta):
    return oracle.affine_operator(T, theta)


def _relcol(X, R):
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.linalg.norm(R, axis=0)))


@pytest.mark.parametrize("kv,ks,Q,skew", [(128, 128, 3, True), (96, 80, 4, False)])
def test_affine_instance_operators_exact(kv, ks, Q, skew):
    from paper_2009_11742_amd import AffineFamily
    A, B, b = _terms(kv, ks, Q, seed=kv + Q, skew=skew)
    fam = AffineFamily(A, B, b, 0.1, state="f32")
    rng = np.random.default_rng(5)
    for _ in range(3):
        th = rng.uniform(0.2, 0.8, Q)
        rom = fam.instance(th)
        Ag, Bg, _ = rom.operators()
        assert np.array_equal(Ag, _assemble(A, th).astype(np.float32).astype(np.float64))
        assert np.array_equal(Bg, _assemble(B, th).astype(np.float32).astype(np.float64))
        rom.close()
    fam.close()


def test_rank3_grouped_run_matches_standalone_and_oracle():
    from paper_2009_11742_amd import AffineFamily, GroupPlan, Rom
    kv = ks = 128
    Q = 3
    A, B, b = _terms(kv, ks, Q, seed=3, skew=True)
    b32 = b.astype(np.float32).astype(np.float64)
    fam = AffineFamily(A, B, b32, 0.1, state="f32")
    rng = np.random.default_rng(11)
    Ms = [3, 17, 8, 40, 1, 12]
    N = 700
    roms, mus, Vs, Ss, ths, dts = [], [], [], [], [], []
    for p, M in enumerate(Ms):
        th = rng.uniform(0.2, 0.8, Q)
        Ah = _assemble(A, th)
        dt = float(np.float32(0.5 / np.linalg.norm(Ah, 2)))
        rom = fam.instance(th, dt=dt)
        roms.append(rom); ths.append(th); dts.append(dt)
        mus.append(torch.tensor(rng.uniform(0.5, 1.0, M), dtype=torch.float64, device="cuda"))
        V, S = rom.zeros(M)
        Vs.append(V); Ss.append(S)
    plan = GroupPlan(roms, mus, Vs, Ss)
    plan.run(N)
    plan.check()
    torch.cuda.synchronize()
    sched = plan.schedule          # one K: all instances on one schedule
    plan.close()
    for p, M in enumerate(Ms):
        Ah = _assemble(A, ths[p]); Bh = _assemble(B, ths[p])
        ref_rom = Rom(Ah, Bh, b32, dts[p], state="f32", schedule=sched)
        V1, S1 = ref_rom.zeros(M)
        ref_rom.run_rank2(mus[p], V1, S1, N)
        ref_rom.check()
        torch.cuda.synchronize()
        assert torch.equal(Vs[p], V1) and torch.equal(Ss[p], S1), p
        Ag, Bg, _ = roms[p].operators()
        r = oracle.run_rank2(Ag, Bg, b32, dts[p], mus[p].cpu().numpy(), N)
        e = max(_relcol(Vs[p].cpu().numpy().astype(np.float64).T, r["V"]),
                _relcol(Ss[p].cpu().numpy().astype(np.float64).T, r["S"]))
        print("rank-3 instance %d (M=%d): err %.2e" % (p, M, e))
        assert e <= 1e-5
        ref_rom.close()
    for r_ in roms:
        r_.close()
    fam.close()


def test_affine_skew_check():
    from paper_2009_11742_amd import AffineFamily, RomError
    from paper_2009_11742_amd import _lib
    A, B, b = _terms(64, 64, 2, seed=9, skew=True)
    fam = AffineFamily(A, B, b, 0.05, state="f32", skew_check=True)
    th = np.array([0.5, 0.7])
    smax = np.linalg.norm(_assemble(A, th), 2)
    rom = fam.instance(th, dt=1.0 / smax)          # dt sigma = 1: fine
    rom.close()
    with pytest.raises(RomError) as ei:
        fam.instance(th, dt=2.01 / smax)
    assert ei.value.status == _lib.ROM_E_UNSTABLE
    fam.close()


def test_rank3_rowsplit_plan_matches_standalone():
    """Instances of a K = 256 family pinned to the row-split schedule run as
    one row-split grouped plan, each bitwise equal to its own row-split
    run; one sampled column per instance against the oracle."""
    from paper_2009_11742_amd import AffineFamily, GroupPlan
    fam_in = synth.make_affine_family(256, 256, 3, 5, 64, seed=4)
    b32 = fam_in["b"].astype(np.float32).astype(np.float64)
    fam = AffineFamily(fam_in["Avs_terms"], fam_in["Asv_terms"], b32, 0.1, state="f32", schedule="rowsplit")
    roms, mus, Vs, Ss, dts = [], [], [], [], []
    for th, mu in zip(fam_in["theta"], fam_in["mu"]):
        dt = float(np.float32(0.5 / float(np.abs(th) @ fam_in["smax"])))
        r = fam.instance(th, dt=dt)
        V, S = r.zeros(len(mu))
        roms.append(r); dts.append(dt); Vs.append(V); Ss.append(S)
        mus.append(torch.tensor(mu, dtype=torch.float64, device="cuda"))
    plan = GroupPlan(roms, mus, Vs, Ss)
    assert plan.schedule == "rowsplit"
    N = 600
    plan.run(N)
    plan.check()
    torch.cuda.synchronize()
    for p, r in enumerate(roms):
        V1, S1 = r.zeros(64)
        r.run_rank2(mus[p], V1, S1, N)
        r.check()
        assert r.last_schedule == "rowsplit"
        torch.cuda.synchronize()
        assert torch.equal(Vs[p], V1) and torch.equal(Ss[p], S1), p
        Ag, Bg, _ = r.operators()
        col = 17 * p % 64
        ref = oracle.run_rank2(Ag, Bg, b32, dts[p], fam_in["mu"][p][col:col + 1], N)
        e = _relcol(Vs[p].cpu().numpy().astype(np.float64).T[:, col:col + 1], ref["V"])
        assert e <= 1e-5, (p, e)
    plan.close()
    for r in roms:
        r.close()
    fam.close()


def test_rank3_full_workload_sampled():
    """The rank-3 measurement workload as bench.py runs it: Q = 4 terms,
    K = 512, 64 parameter points x 64 samples, 2000 steps, on the plan the
    timing picks; four instances bitwise equal to their own runs of that
    schedule, one sampled column each within 1e-5 of the oracle."""
    import concurrent.futures as cf
    from paper_2009_11742_amd import AffineFamily, GroupPlan
    K, Q, P, M, N = 512, 4, 64, 64, 2000
    fam_in = synth.make_affine_family(K, K, Q, P, M, seed=0)
    b32 = fam_in["b"].astype(np.float32).astype(np.float64)
    fam = AffineFamily(fam_in["Avs_terms"], fam_in["Asv_terms"], b32, 0.1, state="f32")
    dts = [float(np.float32(0.5 / float(np.abs(th) @ fam_in["smax"]))) for th in fam_in["theta"]]
    roms = [fam.instance(th, dt=d) for th, d in zip(fam_in["theta"], dts)]
    mus = [torch.tensor(m, dtype=torch.float64, device="cuda") for m in fam_in["mu"]]
    Vs, Ss = zip(*[r.zeros(M) for r in roms])
    plan = GroupPlan(roms, mus, list(Vs), list(Ss))
    plan.run(N)
    plan.check()
    torch.cuda.synchronize()
    sched = plan.schedule
    picks = [0, 21, 42, 63]
    for p in picks:
        from paper_2009_11742_amd import Rom
        Ag, Bg, _ = roms[p].operators()
        ref = Rom(Ag, Bg, b32, dts[p], state="f32", schedule=sched)
        V1, S1 = ref.zeros(M)
        ref.run_rank2(mus[p], V1, S1, N)
        ref.check()
        torch.cuda.synchronize()
        assert torch.equal(Vs[p], V1) and torch.equal(Ss[p], S1), p
        ref.close()

    def check(p):
        Ag, Bg, _ = roms[p].operators()
        col = (13 * p) % M
        r = oracle.run_rank2(Ag, Bg, b32, dts[p], fam_in["mu"][p][col:col + 1], N)
        return max(_relcol(Vs[p].cpu().numpy().astype(np.float64).T[:, col:col + 1], r["V"]),
                   _relcol(Ss[p].cpu().numpy().astype(np.float64).T[:, col:col + 1], r["S"]))
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        errs = list(ex.map(check, picks))
    print("rank-3 full workload (%s plan): sampled errors %s" % (sched, ["%.2e" % e for e in errs]))
    assert max(errs) <= 1e-5
    plan.close()
    for r in roms:
        r.close()
    fam.close()
