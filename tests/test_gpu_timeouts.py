"""Row-split time-outs reach the caller on every entry point that runs the
row-split kernels.

The condition is forced from the host (rom_debug_force_timeout): the first
group barrier of each row-split launch then waits for one arrival more than
the group has, with a short poll budget, so it runs out, records
ROM_E_TIMEOUT and releases every later wait; the kernel still ends normally
(its results are garbage).  Each case checks that the failure is reported,
that the report clears the condition, and that a normal run afterwards is
correct again.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2009_11742_amd import _lib

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture
def forced():
    lib = _lib.load()
    lib.rom_debug_force_timeout(1)
    try:
        yield
    finally:
        lib.rom_debug_force_timeout(0)


def _relcol(X, R):
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.linalg.norm(R, axis=0)))


def _rom(inst, schedule="rowsplit"):
    from paper_2009_11742_amd import Rom
    return Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule=schedule)


def _timed_out(fn):
    with pytest.raises(_lib.RomError) as ei:
        fn()
    assert ei.value.status == _lib.ROM_E_TIMEOUT, str(ei.value)


def test_rank2_run_reports_timeout_and_recovers():
    inst = synth.round_to(synth.make_instance(256, 256, 48, seed=1), "f32")
    rom = _rom(inst)
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    lib = _lib.load()
    lib.rom_debug_force_timeout(1)
    try:
        V, S = rom.zeros(48)
        rom.run_rank2(mu, V, S, 50)
        assert rom.last_schedule == "rowsplit"
        _timed_out(rom.check)
    finally:
        lib.rom_debug_force_timeout(0)
    rom.check()                         # the report cleared the condition
    V, S = rom.zeros(48)
    rom.run_rank2(mu, V, S, 200)
    rom.check()
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 200)
    assert _relcol(V.cpu().numpy().astype(np.float64).T, ref["V"]) <= 1e-5
    rom.close()


def test_adjoint_reports_forward_sweep_timeout(forced):
    inst = synth.round_to(synth.make_instance(256, 256, 8, seed=2), "f32")
    rom = _rom(inst)
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    for stride in (0, -1):
        _timed_out(lambda: rom.adjoint(mu, 40, c, stride=stride))
    rom.check()                         # rom_adjoint cleared what it reported
    rom.close()


def test_autograd_function_raises_on_timeout(forced):
    from paper_2009_11742_amd import RomQoI, tuning
    # K = 512, M = 64 runs row-split by the shipped tuning table, so the
    # function's context (no schedule flag) takes it without tuning
    if not any(e["kv_pad"] == 512 and e["m_pad"] == 64 and e["op"] == "f32" and e["schedule"] == "rowsplit"
               for e in tuning.entries()):
        pytest.skip("tuning table does not route K = 512, M = 64 to the row-split kernels")
    inst = synth.round_to(synth.make_instance(512, 512, 64, seed=3), "f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda", requires_grad=True)
    Avs = torch.tensor(inst["Avs"], dtype=torch.float64, requires_grad=True)
    Asv = torch.tensor(inst["Asv"], dtype=torch.float64)
    _timed_out(lambda: RomQoI.apply(Avs, Asv, mu, inst["b"], inst["c"], inst["dt"], 30))
    # forward only (no input needs a gradient): the plain run, checked too
    _timed_out(lambda: RomQoI.apply(Avs.detach(), Asv, mu.detach(), inst["b"], inst["c"], inst["dt"], 30))


def test_autograd_forward_only_matches_oracle():
    from paper_2009_11742_amd import RomQoI
    inst = synth.round_to(synth.make_instance(40, 40, 3, seed=4), "f32")
    J = RomQoI.apply(torch.tensor(inst["Avs"]), torch.tensor(inst["Asv"]),
                     torch.tensor(inst["mu"], device="cuda"), inst["b"], inst["c"], inst["dt"], 150)
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 150, c=inst["c"])
    assert abs(float(J) - float(np.sum(ref["J"]))) <= 1e-5 * float(np.sum(ref["J"]))


def test_tuner_marks_timed_out_rowsplit_not_applicable(forced):
    from paper_2009_11742_amd import tuning
    saved = tuning.entries()
    try:
        tuning.clear()
        inst = synth.round_to(synth.make_instance(512, 512, 100, seed=5), "f32")
        rom = _rom(inst, schedule="auto")
        mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
        V, S = rom.zeros(100)
        rom.run_rank2(mu, V, S, 20)     # tunes this shape first
        times = rom.schedule_times(100)
        assert times["rowsplit"] is None and rom.last_schedule != "rowsplit", times
        rom.check()                     # the tuner's time-out is not the run's
        rom.close()
    finally:
        tuning.clear()
        for e in saved:
            tuning.put(e["kv_pad"], e["ks_pad"], e["m_pad"], e["op"], e["schedule"], e["us"])


def test_grouped_rowsplit_plan_reports_timeout():
    from paper_2009_11742_amd import GroupPlan, Rom, run_grouped
    insts = [synth.round_to(synth.make_instance(256, 256, M, seed=10 + i), "f32") for i, M in enumerate((30, 70))]
    roms = [Rom(d["Avs"], d["Asv"], d["b"], d["dt"], state="f32", schedule="rowsplit") for d in insts]
    mus = [torch.tensor(d["mu"], dtype=torch.float64, device="cuda") for d in insts]
    states = [r.zeros(len(d["mu"])) for r, d in zip(roms, insts)]
    Vs, Ss = [s[0] for s in states], [s[1] for s in states]
    lib = _lib.load()
    lib.rom_debug_force_timeout(1)
    try:
        _timed_out(lambda: run_grouped(roms, mus, Vs, Ss, 30))
        plan = GroupPlan(roms, mus, Vs, Ss)
        assert plan.schedule == "rowsplit"
        plan.run(30)
        _timed_out(plan.check)
    finally:
        lib.rom_debug_force_timeout(0)
    plan.check()
    for V, S in zip(Vs, Ss):
        V.zero_(); S.zero_()
    plan.run(100)
    plan.check()
    for V, d in zip(Vs, insts):
        ref = oracle.run_rank2(d["Avs"], d["Asv"], d["b"], d["dt"], d["mu"], 100)
        assert _relcol(V.cpu().numpy().astype(np.float64).T, ref["V"]) <= 1e-5
    plan.close()
    for r in roms:
        r.close()
