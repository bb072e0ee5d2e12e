"""rom_run_rank2_noalloc (the allocation-free rank-2 run) against
rom_run_rank2 on the row-split schedule: the same kernels with the scratch in
the library's static per-GPU array instead of the context's workspace, so
the results must be bitwise equal.  Two calls in a row on different
contexts, the second with a smaller input (fewer samples, smaller K, other
operator type), so the second runs over what the first left in the array.
Called through the C ABI (ctypes), not the Python wrapper.
"""
import ctypes as C

import numpy as np
import pytest

import synth
from paper_2009_11742_amd import _lib

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _both(inst, ops, nsteps, n0=0):
    from paper_2009_11742_amd import Rom
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", ops=ops, schedule="rowsplit")
    M = len(inst["mu"])
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    lib = _lib.load()
    out = {}
    for name in ("reference", "noalloc"):
        V, S = rom.zeros(M)
        J = torch.zeros(M, dtype=torch.float64, device="cuda")
        y = torch.zeros((nsteps, M), dtype=torch.float64, device="cuda")
        fn = lib.rom_run_rank2 if name == "reference" else lib.rom_run_rank2_noalloc
        _lib.check(fn(rom.handle, M, _ptr(mu), n0, nsteps, _ptr(V), _ptr(S), _ptr(c), _ptr(J), _ptr(y), st))
        rom.check()
        assert rom.last_schedule == "rowsplit"
        out[name] = [t.cpu().numpy() for t in (V, S, J, y)]
    rom.close()
    return out


def test_noalloc_equals_rowsplit_run_twice_second_smaller():
    big = synth.round_to(synth.make_instance(512, 512, 200, seed=21), "f32")
    small = synth.round_to(synth.make_instance(256, 256, 40, seed=22), "f32")
    odd = synth.round_to(synth.make_instance(330, 330, 30, seed=24), "f32")      # padded K 384, run-time K
    for inst, ops, N, n0 in ((big, "f32", 300, 0), (small, "bf16", 200, 7), (odd, "f32", 150, 2)):
        out = _both(inst, ops, N, n0=n0)
        for a, b, name in zip(out["reference"], out["noalloc"], ("V", "S", "J", "y")):
            assert np.array_equal(a, b), (ops, name, float(np.max(np.abs(a - b))))
        assert np.all(np.isfinite(out["noalloc"][0]))


def test_noalloc_rejects_what_rowsplit_cannot_run():
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(320, 256, 8, seed=23, skew=False), "f32")   # Kv != Ks
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(8)
    with pytest.raises(_lib.RomError) as ei:
        rom.run_rank2_noalloc(mu, V, S, 10)
    assert ei.value.status == _lib.ROM_E_UNSUPPORTED
    assert float(V.abs().max()) == 0.0          # nothing was enqueued
    rom.close()
