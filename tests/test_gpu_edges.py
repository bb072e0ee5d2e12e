"""Edge cases of the GPU path: the largest LDS-resident FP32 state
(Kv_pad + Ks_pad = 4096), the first size past it (the panel schedule with
FP32 operators, ROM_E_UNSUPPORTED with BF16 ones), the
8-column flag where 8 samples' state does not fit (falls back to 4), a
single sample on every FP32 schedule, a one-step adjoint and a stride >= N
adjoint, and a grouped run of one instance with one sample.  Bars as
elsewhere: 1e-5 (FP32 states), 1e-4 (adjoint gradients)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _relcol(X, R):
    nr = np.linalg.norm(R, axis=0)
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.where(nr > 0, nr, 1.0)))


def _run(inst, N, schedule="auto", probe=True):
    from paper_2009_11742_amd import Rom
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule=schedule)
    M = len(inst["mu"])
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(M)
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda") if probe else None
    J = torch.zeros(M, dtype=torch.float64, device="cuda") if probe else None
    rom.run_rank2(mu, V, S, N, c=c, J=J)
    rom.check()
    out = {"V": V.cpu().numpy().astype(np.float64).T, "S": S.cpu().numpy().astype(np.float64).T,
           "J": J.cpu().numpy() if probe else None, "schedule": rom.last_schedule}
    rom.close()
    return out


@pytest.mark.parametrize("kv,ks,M", [(2048, 2048, 5), (3000, 1000, 3)])
def test_largest_lds_resident_state(kv, ks, M):
    inst = synth.round_to(synth.make_instance(kv, ks, M, seed=kv + ks, skew=(kv == ks)), "f32")
    N = 20
    g = _run(inst, N)
    r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"])
    e = max(_relcol(g["V"], r["V"]), _relcol(g["S"], r["S"]))
    print("largest state kv=%d ks=%d M=%d: err %.2e schedule %s" % (kv, ks, M, e, g["schedule"]))
    assert e <= 1e-5
    assert np.max(np.abs(g["J"] - r["J"]) / r["J"]) <= 1e-5


def test_past_the_lds_limit_takes_the_panel_schedule():
    """FP32 runs past the column blocks' LDS limit (Kv_pad + Ks_pad > 4096)
    run on the panel schedule; BF16 operators there are refused before
    anything is written."""
    from paper_2009_11742_amd import Rom, RomError
    from paper_2009_11742_amd import _lib
    inst = synth.round_to(synth.make_instance(2049, 2048, 2, seed=1, skew=False), "f32")
    N = 5
    g = _run(inst, N, schedule="auto")
    assert g["schedule"] == "panel"
    r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"])
    assert max(_relcol(g["V"], r["V"]), _relcol(g["S"], r["S"])) <= 1e-5
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", ops="bf16")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(2)
    with pytest.raises(RomError) as ei:
        rom.run_rank2(mu, V, S, N)
    assert ei.value.status == _lib.ROM_E_UNSUPPORTED
    assert torch.count_nonzero(V) == 0 and torch.count_nonzero(S) == 0     # nothing written
    rom.close()


def test_columns8_flag_falls_back_where_8_samples_do_not_fit():
    inst = synth.round_to(synth.make_instance(1536, 1536, 9, seed=3), "f32")
    N = 30
    g = _run(inst, N, schedule="columns8")
    assert g["schedule"] == "columns"
    r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"])
    assert max(_relcol(g["V"], r["V"]), _relcol(g["S"], r["S"])) <= 1e-5


@pytest.mark.parametrize("schedule", ["columns", "columns8", "rowsplit"])
def test_single_sample_every_schedule(schedule):
    inst = synth.round_to(synth.make_instance(256, 256, 1, seed=4), "f32")
    N = 800
    g = _run(inst, N, schedule=schedule)
    assert g["schedule"] == schedule
    r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"])
    assert max(_relcol(g["V"], r["V"]), _relcol(g["S"], r["S"])) <= 1e-5
    assert abs(g["J"][0] - r["J"][0]) / r["J"][0] <= 1e-5


@pytest.mark.parametrize("N,stride", [(1, 0), (37, 37), (37, 1000)])
def test_adjoint_short_and_single_segment(N, stride):
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(48, 40, 3, seed=9, skew=False), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    out = rom.adjoint(mu, N, c, stride=stride)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    rom.close()
    r = oracle.adjoint(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, inst["c"])
    for k in ("J", "dAvs", "dAsv", "dmu"):
        nr = float(np.linalg.norm(r[k]))
        if nr == 0.0:
            # one step from rest: S^0 = 0 and q starts at 0, so the operator
            # gradients are exactly zero
            assert float(np.linalg.norm(g[k])) == 0.0, k
            continue
        e = float(np.linalg.norm(g[k] - r[k])) / nr
        assert e <= 1e-4, (k, e)


def test_grouped_single_instance_single_sample():
    from paper_2009_11742_amd import Rom, run_grouped
    inst = synth.round_to(synth.make_instance(96, 160, 1, seed=12, skew=False), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(1)
    run_grouped([rom], [mu], [V], [S], 900)
    torch.cuda.synchronize()
    r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 900)
    assert _relcol(V.cpu().numpy().astype(np.float64).T, r["V"]) <= 1e-5
    assert _relcol(S.cpu().numpy().astype(np.float64).T, r["S"]) <= 1e-5
    rom.close()


def test_zero_steps_change_nothing():
    """nsteps = 0 is a valid no-op on every entry point that steps."""
    from paper_2009_11742_amd import Fom, GroupPlan, Rom
    inst = synth.round_to(synth.make_instance(64, 64, 3, seed=2), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(3)
    V.fill_(1.0); S.fill_(2.0)
    rom.run_rank2(mu, V, S, 0)
    plan = GroupPlan([rom], [mu], [V], [S])
    plan.run(0)
    d = synth.make_shear_fom(5, 6)
    F = Fom(d["Av"], d["As"], d["f"], d["dt"])
    Vf, Sf = F.zeros(2)
    Vf.fill_(3.0)
    F.run(mu[:2], Vf, Sf, 0)
    torch.cuda.synchronize()
    assert torch.all(V == 1.0) and torch.all(S == 2.0) and torch.all(Vf == 3.0) and torch.all(Sf == 0.0)
    plan.close(); rom.close(); F.close()


def test_pod_rank_one_and_square_snapshots():
    """A rank-one snapshot matrix keeps exactly one mode (the normalised
    common direction) whatever the tolerance; a square full-rank one (n = ns)
    keeps all modes when asked, orthonormal."""
    from paper_2009_11742_amd import pod
    rng = np.random.default_rng(1)
    u = rng.standard_normal(500)
    X = np.outer(u, rng.standard_normal(12))
    Phi, sig, k = pod(torch.tensor(X, device="cuda"), tol=0.0, kmax=12)
    assert k == 1
    p = Phi.cpu().numpy()[:, 0]
    assert abs(abs(p @ u) / np.linalg.norm(u) - 1.0) < 1e-13
    assert abs(sig[0] - np.linalg.norm(X, 2)) <= 1e-13 * sig[0]
    Y = rng.standard_normal((40, 40))
    Phi, sig, k = pod(torch.tensor(Y, device="cuda"))
    P = Phi.cpu().numpy()
    assert k == 40 and np.max(np.abs(P.T @ P - np.eye(40))) < 1e-12
    assert np.max(np.abs(sig - np.linalg.svd(Y, compute_uv=False)) / sig) < 1e-11


def test_fom_csr_with_empty_rows_and_one_dof():
    """CSR operators with empty rows (the axis rows of the grid) and a 1 x 1
    system: the FOM run equals the oracle."""
    from paper_2009_11742_amd import Fom
    ptr = np.array([0, 0, 2, 2], dtype=np.int32)        # rows 0 and 2 empty
    col = np.array([0, 1], dtype=np.int32)
    Av = (ptr, col, np.array([0.5, -1.0]))
    As = (np.array([0, 1, 2], dtype=np.int32), np.array([1, 1], dtype=np.int32), np.array([2.0, -0.25]))
    f = np.array([0.0, 1.0, 0.5])
    mu = np.array([0.6, 0.9])
    for Avx, Asx, ff, nv, ns in ((Av, As, f, 3, 2),
                                 ((np.array([0, 1], np.int32), np.array([0], np.int32), np.array([-1.0])),
                                  (np.array([0, 1], np.int32), np.array([0], np.int32), np.array([1.0])),
                                  np.array([1.0]), 1, 1)):
        F = Fom(Avx, Asx, ff, 0.05)
        V = torch.zeros((nv, 2), dtype=torch.float64, device="cuda")
        S = torch.zeros((ns, 2), dtype=torch.float64, device="cuda")
        F.run(torch.tensor(mu, device="cuda"), V, S, 300)
        torch.cuda.synchronize()
        r = oracle.fom_run(Avx, Asx, ff, 0.05, mu, 300)
        assert np.max(np.abs(V.cpu().numpy() - r["V"])) <= 1e-12 * max(1.0, np.abs(r["V"]).max())
        assert np.max(np.abs(S.cpu().numpy() - r["S"])) <= 1e-12 * max(1.0, np.abs(r["S"]).max())
        F.close()


def _guarded(shape, dtype, pad=320, fill=0.0):
    """A tensor of `shape` inside a larger buffer whose `pad` elements on each
    side hold a sentinel: writes past the tensor's ends show up there."""
    n = int(np.prod(shape))
    buf = torch.full((n + 2 * pad,), 7777.0, dtype=dtype, device="cuda")
    t = buf[pad:pad + n].view(*shape)
    t.fill_(fill)
    return buf, t


def _canaries_intact(buf, n, pad=320):
    torch.cuda.synchronize()
    return bool(torch.all(buf[:pad] == 7777.0)) and bool(torch.all(buf[pad + n:] == 7777.0))


@pytest.mark.parametrize("kv,ks,M,state,ops,schedule", [
    (70, 45, 13, "f32", "f32", "columns"), (70, 45, 13, "f32", "f32", "columns8"),
    (256, 256, 70, "f32", "f32", "rowsplit"), (256, 256, 70, "f32", "bf16", "rowsplit"),
    (70, 45, 13, "f32", "bf16", "columns"), (33, 50, 5, "f64", "f64", "auto"),
    (100, 100, 5, "f64", "f64", "auto")])
def test_no_writes_outside_the_outputs(kv, ks, M, state, ops, schedule):
    """Canary-padded states, QoI and trace buffers on ragged K and M: every
    kernel path writes only inside the arrays it is given."""
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(kv, ks, M, seed=kv + M, skew=(kv == ks)), state)
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state=state, ops=ops, schedule=schedule)
    dt = torch.float32 if state == "f32" else torch.float64
    N = 50
    bV, V = _guarded((M, kv), dt)
    bS, S = _guarded((M, ks), dt)
    bJ, J = _guarded((M,), torch.float64)
    by, y = _guarded((N, M), torch.float64)
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    c = torch.tensor(inst["c"], dtype=dt, device="cuda")
    rom.run_rank2(mu, V, S, N, c=c, J=J, y=y)
    rom.check()
    for b, t in ((bV, V), (bS, S), (bJ, J), (by, y)):
        assert _canaries_intact(b, t.numel())
    assert torch.all(torch.isfinite(V)) and float(V.abs().max()) > 0
    rom.close()


def test_no_writes_outside_the_outputs_adjoint_grouped_receivers_fom():
    from paper_2009_11742_amd import Fom, GroupPlan, Rom, pod
    inst = synth.round_to(synth.make_instance(70, 45, 6, seed=4, skew=False), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    out = rom.adjoint(mu, 40, c)                      # outputs allocated by the binding: compare with a guarded run
    bV, V = _guarded((6, 70), torch.float32)
    bS, S = _guarded((6, 45), torch.float32)
    plan = GroupPlan([rom], [mu], [V], [S])
    plan.run(60)
    assert _canaries_intact(bV, V.numel()) and _canaries_intact(bS, S.numel())
    bY, Y = _guarded((30, 3, 6), torch.float64)
    bst, st = _guarded((30, 3, 5), torch.float64)
    C3 = torch.tensor(np.random.default_rng(1).standard_normal((3, 70)), dtype=torch.float32, device="cuda")
    from paper_2009_11742_amd import _lib
    from paper_2009_11742_amd.rom import _ptr, _stream_handle
    V.zero_(); S.zero_()
    _lib.check(_lib.load().rom_run_receivers(rom.handle, 6, _ptr(mu), 0, 30, _ptr(V), _ptr(S), 3, _ptr(C3),
                                             _ptr(Y), _ptr(st), _stream_handle(None)))
    assert _canaries_intact(bY, Y.numel()) and _canaries_intact(bst, st.numel())
    assert all(torch.all(torch.isfinite(v)) for v in out.values())
    plan.close(); rom.close()
    d = synth.make_shear_fom(9, 13)
    F = Fom(d["Av"], d["As"], d["f"], d["dt"])
    bFV, FV = _guarded((d["nv"], 3), torch.float64)
    bFS, FS = _guarded((d["ns"], 3), torch.float64)
    F.run(mu[:3], FV, FS, 80)
    assert _canaries_intact(bFV, FV.numel()) and _canaries_intact(bFS, FS.numel())
    X = torch.tensor(np.random.default_rng(2).standard_normal((d["nv"], 20)), device="cuda")
    Phi, _, k = pod(X, kmax=7)
    Pv = Phi.contiguous()
    Ps = torch.tensor(np.linalg.qr(np.random.default_rng(3).standard_normal((d["ns"], 5)))[0], device="cuda")
    bA, A = _guarded((5, 7), torch.float64)          # Kv x Ks column-major = (Ks, Kv) row-major
    bB, B = _guarded((7, 5), torch.float64)
    bb, bvec = _guarded((7,), torch.float64)
    _lib.check(_lib.load().rom_fom_project(F._h, 7, 5, _ptr(Pv), _ptr(Ps), _ptr(A), _ptr(B), _ptr(bvec),
                                           _stream_handle(None)))
    assert _canaries_intact(bA, A.numel()) and _canaries_intact(bB, B.numel()) and _canaries_intact(bb, 7)
    F.close()


@pytest.mark.parametrize("state", ["f32", "f64"])
def test_check_finite_reports_blown_up_states(state):
    """rom_check_finite passes a healthy run, and flags a state that holds a
    NaN and a run whose unstable pair (independent random Asv, long
    horizon) overflowed."""
    from paper_2009_11742_amd import Rom, RomError, _lib
    inst = synth.round_to(synth.make_instance(40, 40, 4, seed=1), state)
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state=state)
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(4)
    rom.run_rank2(mu, V, S, 200)
    rom.check_finite(V, S)
    S[2, 7] = float("nan")
    with pytest.raises(RomError) as ei:
        rom.check_finite(V, S)
    assert ei.value.status == _lib.ROM_E_NONFINITE
    rom.close()
    bad = synth.round_to(synth.make_instance(40, 40, 4, seed=2, random_asv=True), state)
    rom = Rom(bad["Avs"], bad["Asv"], bad["b"], 4.0 * bad["dt"], state=state)
    V, S = rom.zeros(4)
    rom.run_rank2(mu, V, S, 20000)
    torch.cuda.synchronize()
    assert not bool(torch.all(torch.isfinite(V)))        # the pair did blow up
    with pytest.raises(RomError) as ei:
        rom.check_finite(V, S)
    assert ei.value.status == _lib.ROM_E_NONFINITE
    rom.close()
