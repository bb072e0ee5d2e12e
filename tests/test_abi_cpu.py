"""Host-side checks of the C ABI (no GPU needed).

* the built library exports every function include/rom.h declares;
* argument validation happens before any device work, so the error codes of
  rom_create / rom_run_rank2 / rom_step_rank1 are checked here on the CPU.
"""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import synth
from paper_2009_11742_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rom.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rom_[a-z0-9_]+)\s*\(", src)))


def test_header_lists_entry_points():
    names = _declared()
    for n in ("rom_create", "rom_step_rank1", "rom_run_rank2", "rom_adjoint", "rom_destroy"):
        assert n in names
    assert sorted(_lib.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (rom_[a-z0-9_]+)$", out, flags=re.M))
    for name in _declared():
        assert name in exported, name
        assert hasattr(lib, name)
    assert lib.rom_version().startswith(b"rank2rom")


def _create(cfg, A, B, b):
    lib = _lib.load()
    pd = C.POINTER(C.c_double)
    ctx = C.c_void_p(12345)
    st = lib.rom_create(C.byref(cfg) if cfg is not None else None,
                        None if A is None else A.ctypes.data_as(pd),
                        None if B is None else B.ctypes.data_as(pd),
                        None if b is None else b.ctypes.data_as(pd), None, C.byref(ctx))
    return st, ctx


def _inst(k=8):
    inst = synth.make_instance(k, k, 2, seed=1)
    return (np.asfortranarray(inst["Avs"]), np.asfortranarray(inst["Asv"]), inst["b"].copy(), inst["dt"])


def test_create_rejects_bad_arguments():
    A, B, b, dt = _inst()
    cfg = _lib.RomConfig(8, 8, dt, _lib.ROM_F32, _lib.ROM_F32, 0)
    assert _create(None, A, B, b)[0] == _lib.ROM_E_ARG
    assert _create(cfg, None, B, b)[0] == _lib.ROM_E_ARG
    assert _create(cfg, A, B, None)[0] == _lib.ROM_E_ARG
    st, ctx = _create(_lib.RomConfig(0, 8, dt, _lib.ROM_F32, _lib.ROM_F32, 0), A, B, b)
    assert st == _lib.ROM_E_ARG and not ctx.value          # out is cleared on failure
    assert _create(_lib.RomConfig(8, 8, 0.0, _lib.ROM_F32, _lib.ROM_F32, 0), A, B, b)[0] == _lib.ROM_E_ARG
    assert _create(_lib.RomConfig(8, 8, float("nan"), _lib.ROM_F32, _lib.ROM_F32, 0), A, B, b)[0] == _lib.ROM_E_ARG
    assert _create(_lib.RomConfig(8, 8, dt, _lib.ROM_F32, _lib.ROM_BF16, 0), A, B, b)[0] == _lib.ROM_E_ARG
    assert _create(_lib.RomConfig(8, 8, dt, _lib.ROM_F32, _lib.ROM_F32, 0x100), A, B, b)[0] == _lib.ROM_E_ARG
    two = _lib.ROM_SCHED_PANEL | _lib.ROM_SCHED_COLUMNS                   # at most one schedule flag
    assert _create(_lib.RomConfig(8, 8, dt, _lib.ROM_F32, _lib.ROM_F32, two), A, B, b)[0] == _lib.ROM_E_ARG
    assert "rom_create" in _lib.load().rom_last_error().decode()


def test_create_rejects_nonfinite_inputs():
    A, B, b, dt = _inst()
    cfg = _lib.RomConfig(8, 8, dt, _lib.ROM_F32, _lib.ROM_F32, 0)
    A2 = A.copy(); A2[3, 4] = np.nan
    assert _create(cfg, A2, B, b)[0] == _lib.ROM_E_NONFINITE
    b2 = b.copy(); b2[0] = np.inf
    assert _create(cfg, A, B, b2)[0] == _lib.ROM_E_NONFINITE


def test_create_skew_stability_check():
    """dt * sigma_max(Avs) >= 2 makes the leapfrog energy indefinite."""
    A, B, b, dt = _inst()
    smax = np.linalg.svd(A, compute_uv=False)[0]
    bad = 2.0 / smax * 1.001
    cfg = _lib.RomConfig(8, 8, bad, _lib.ROM_F32, _lib.ROM_F32, _lib.ROM_SKEW_CHECK)
    assert _create(cfg, A, B, b)[0] == _lib.ROM_E_UNSTABLE
    assert "sigma_max" in _lib.load().rom_last_error().decode()


def test_run_rejects_bad_arguments():
    lib = _lib.load()
    d = C.c_void_p(0x1000)
    assert lib.rom_run_rank2(None, 4, d, 0, 10, d, d, None, None, None, None) == _lib.ROM_E_ARG
    # a non-null but never-dereferenced handle is enough to reach the per-argument checks
    fake = C.c_void_p(0x10)
    assert lib.rom_run_rank2(fake, 0, d, 0, 10, d, d, None, None, None, None) == _lib.ROM_E_ARG
    assert lib.rom_run_rank2(fake, 4, None, 0, 10, d, d, None, None, None, None) == _lib.ROM_E_ARG
    assert lib.rom_run_rank2(fake, 4, d, -1, 10, d, d, None, None, None, None) == _lib.ROM_E_ARG
    assert lib.rom_run_rank2(fake, 4, d, 0, -5, d, d, None, None, None, None) == _lib.ROM_E_ARG
    assert lib.rom_run_rank2(fake, 4, d, 0, 10, d, d, None, d, None, None) == _lib.ROM_E_ARG  # J w/o c
    assert lib.rom_step_rank1(None, d, d, 0, 0.7, None) == _lib.ROM_E_ARG
    assert lib.rom_step_rank1(fake, None, d, 0, 0.7, None) == _lib.ROM_E_ARG
    assert lib.rom_step_rank1(fake, d, d, -1, 0.7, None) == _lib.ROM_E_ARG
    assert lib.rom_step_rank1(fake, d, d, 0, float("inf"), None) == _lib.ROM_E_NONFINITE
    assert lib.rom_destroy(None) == _lib.ROM_OK


def test_create_rejects_two_schedule_flags():
    A, B, b, dt = _inst()
    for f in (_lib.ROM_SCHED_COLUMNS | _lib.ROM_SCHED_COLUMNS8, _lib.ROM_SCHED_ROWSPLIT | _lib.ROM_SCHED_COLUMNS8,
              _lib.ROM_SCHED_COLUMNS | _lib.ROM_SCHED_ROWSPLIT):
        cfg = _lib.RomConfig(8, 8, dt, _lib.ROM_F32, _lib.ROM_F32, f)
        assert _create(cfg, A, B, b)[0] == _lib.ROM_E_ARG
    assert "ROM_SCHED" in _lib.load().rom_last_error().decode()


def test_create_rejects_state_bf16_without_lowp_operators():
    """The single BF16 state operand exists only for BF16 / FP8 operators
    with FP32 states; other pairs are refused before any device work."""
    A, B, b, dt = _inst()
    for op, st in ((_lib.ROM_F32, _lib.ROM_F32), (_lib.ROM_F64, _lib.ROM_F64), (_lib.ROM_BF16, _lib.ROM_F64),
                   (_lib.ROM_F8E4M3, _lib.ROM_F64)):
        cfg = _lib.RomConfig(8, 8, dt, op, st, _lib.ROM_STATE_BF16)
        assert _create(cfg, A, B, b)[0] == _lib.ROM_E_ARG
        assert "ROM_STATE_BF16" in _lib.load().rom_last_error().decode()
    cfg = _lib.RomConfig(8, 8, dt, _lib.ROM_BF16, _lib.ROM_F32, 256)    # unknown bit
    assert _create(cfg, A, B, b)[0] == _lib.ROM_E_ARG


def test_tune_table_put_get_clear_and_file_round_trip(tmp_path):
    """The tuning table is host state: entries round-trip through put / get
    (key order) and through the text format; bad entries are refused."""
    from paper_2009_11742_amd import tuning
    lib = _lib.load()
    saved = tuning.entries()
    try:
        tuning.clear()
        assert lib.rom_tune_count() == 0
        tuning.put(512, 512, 1024, "f32", "columns", [17.4, 27.2, -1.0, -1.0])
        tuning.put(256, 256, 256, "f32", "columns8", [4.9, 18.5, 4.1, 1.3])
        tuning.put(1024, 1024, 1024, "bf16", "rowsplit", [60.0, 11.0, -1.0, -1.0])
        tuning.put(768, 768, 0, "f32", "columns8", [40.0, -1.0, 45.0])       # last time missing: -1
        tuning.put(256, 256, 256, "f32", "resident", [4.9, 18.5, 5.5, 1.2])  # replaces
        e = tuning.entries()
        assert [(d["kv_pad"], d["m_pad"]) for d in e] == [(256, 256), (512, 1024), (768, 0), (1024, 1024)]
        assert e[0]["schedule"] == "resident" and e[0]["us"] == pytest.approx([4.9, 18.5, 5.5, 1.2, -1.0])
        assert e[2]["us"] == pytest.approx([40.0, -1.0, 45.0, -1.0, -1.0])
        assert e[3]["op"] == "bf16" and e[3]["schedule"] == "rowsplit"
        bad = [(100, 256, 64, "f32", "columns"), (256, 256, 65, "f32", "columns"),
               (256, 256, 0, "f32", "rowsplit"), (256, 256, 0, "f32", "resident"), (256, 256, 0, "f32", "panel"),
               (0, 256, 64, "f32", "columns")]
        for kv, ks, m, op, sc in bad:
            with pytest.raises(_lib.RomError):
                tuning.put(kv, ks, m, op, sc, [1.0, 1.0, 1.0, 1.0])
        ent = _lib.RomTuneEntry(256, 256, 64, _lib.ROM_F32, _lib.ROM_NSCHEDULES)
        assert lib.rom_tune_put(ent) == _lib.ROM_E_ARG
        assert lib.rom_tune_get(99, _lib.RomTuneEntry()) == _lib.ROM_E_ARG
        p = tmp_path / "table.txt"
        tuning.save(str(p), header="test table")
        text = p.read_text()
        assert text.startswith("# test table") and "512 512 1024 f32 columns 17.400 27.200 -1.000 -1.000" in text
        tuning.clear()
        assert tuning.load(str(p)) == 4
        assert tuning.entries() == e
        # lines of the earlier formats (no resident or panel time) still load
        p.write_text("256 256 64 f32 columns 1.0 2.0 3.0\n512 512 64 f32 rowsplit 4.0 2.0 5.0 -1.0\n")
        tuning.clear()
        assert tuning.load(str(p)) == 2
        assert tuning.entries()[0]["us"] == pytest.approx([1.0, 2.0, 3.0, -1.0, -1.0])
        assert tuning.entries()[1]["us"] == pytest.approx([4.0, 2.0, 5.0, -1.0, -1.0])
        tuning.put(2048, 2048, 1024, "f32", "panel", [286.0, -1.0, 400.0, -1.0, 198.0])
        assert tuning.entries()[-1]["schedule"] == "panel"
        p.write_text("256 256 64 f32 columns 1.0\n")
        with pytest.raises(ValueError):
            tuning.load(str(p))
    finally:
        tuning.clear()
        for d in saved:
            tuning.put(d["kv_pad"], d["ks_pad"], d["m_pad"], d["op"], d["schedule"], d["us"])


def test_shipped_tune_table_is_well_formed():
    """The shipped table parses, and each entry's schedule is the fastest of
    its measured times (the autotuner's rule), grouped tile entries by
    per-sample throughput."""
    from paper_2009_11742_amd import tuning
    if not os.path.exists(tuning.DEFAULT_TABLE):
        pytest.skip("no shipped tuning table")
    saved = tuning.entries()
    try:
        tuning.clear()
        n = tuning.load(tuning.DEFAULT_TABLE)
        assert n >= 1
        for d in tuning.entries():
            us = d["us"]
            if d["m_pad"] == 0:
                want = "columns8" if 0 <= us[2] < 2 * us[0] else "columns"
            else:
                ok = [(u, name) for u, name in zip(us, tuning.SCHEDULES) if u >= 0]
                want = min(ok)[1]
            assert d["schedule"] == want, d
    finally:
        tuning.clear()
        for d in saved:
            tuning.put(d["kv_pad"], d["ks_pad"], d["m_pad"], d["op"], d["schedule"], d["us"])


def test_receivers_rejects_bad_arguments():
    lib = _lib.load()
    d = C.c_void_p(0x1000)
    fake = C.c_void_p(0x10)
    E = _lib.ROM_E_ARG
    assert lib.rom_run_receivers(None, 4, d, 0, 10, d, d, 2, d, d, d, None) == E
    assert lib.rom_run_receivers(fake, 0, d, 0, 10, d, d, 2, d, d, d, None) == E          # M
    assert lib.rom_run_receivers(fake, 1025, d, 0, 10, d, d, 2, d, d, d, None) == E       # M > 1024
    assert lib.rom_run_receivers(fake, 4, d, 0, 10, d, d, 0, d, d, d, None) == E          # R
    assert lib.rom_run_receivers(fake, 4, d, 0, 10, d, d, 65, d, d, d, None) == E         # R > 64
    assert lib.rom_run_receivers(fake, 4, d, 0, 10, d, d, 2, None, d, d, None) == E       # C
    assert lib.rom_run_receivers(fake, 4, None, 0, 10, d, d, 2, d, d, d, None) == E       # mu
    assert lib.rom_run_receivers(fake, 4, d, -1, 10, d, d, 2, d, d, d, None) == E         # n0
    assert "rom_run_receivers" in lib.rom_last_error().decode()


def test_affine_rejects_bad_arguments():
    lib = _lib.load()
    A, B, b, dt = _inst()
    pd = C.POINTER(C.c_double)
    AA = np.concatenate([A.ravel(order="F")] * 2)
    BB = np.concatenate([B.ravel(order="F")] * 2)
    out = C.c_void_p(123)
    cfg = _lib.RomConfig(8, 8, dt, _lib.ROM_F32, _lib.ROM_F32, 0)
    E = _lib.ROM_E_ARG
    assert lib.rom_affine_create(None, 2, AA.ctypes.data_as(pd), BB.ctypes.data_as(pd), b.ctypes.data_as(pd), None, C.byref(out)) == E
    assert not out.value
    for Q in (0, 17):
        assert lib.rom_affine_create(C.byref(cfg), Q, AA.ctypes.data_as(pd), BB.ctypes.data_as(pd), b.ctypes.data_as(pd), None, C.byref(out)) == E
    bad = _lib.RomConfig(8, 8, -1.0, _lib.ROM_F32, _lib.ROM_F32, 0)
    assert lib.rom_affine_create(C.byref(bad), 2, AA.ctypes.data_as(pd), BB.ctypes.data_as(pd), b.ctypes.data_as(pd), None, C.byref(out)) == E
    AA2 = AA.copy(); AA2[5] = np.nan
    assert lib.rom_affine_create(C.byref(cfg), 2, AA2.ctypes.data_as(pd), BB.ctypes.data_as(pd), b.ctypes.data_as(pd), None, C.byref(out)) == _lib.ROM_E_NONFINITE
    th = np.ones(2)
    assert lib.rom_affine_instance(None, th.ctypes.data_as(pd), 0.0, None, C.byref(out)) == E
    assert lib.rom_affine_destroy(None) == _lib.ROM_OK


def test_fom_and_pod_reject_bad_arguments():
    lib = _lib.load()
    pi = C.POINTER(C.c_int32)
    pd = C.POINTER(C.c_double)
    out = C.c_void_p(7)
    ptr = np.array([0, 1, 2], dtype=np.int32)
    col = np.array([0, 1], dtype=np.int32)
    val = np.array([1.0, 2.0])
    f = np.zeros(2)
    E = _lib.ROM_E_ARG

    def create(nv, ns, ap, ac, av, sp, sc, sv, ff, dt, flags=0):
        return lib.rom_fom_create(nv, ns, ap.ctypes.data_as(pi), ac.ctypes.data_as(pi), av.ctypes.data_as(pd),
                                  sp.ctypes.data_as(pi), sc.ctypes.data_as(pi), sv.ctypes.data_as(pd),
                                  ff.ctypes.data_as(pd), dt, flags, None, C.byref(out))
    assert create(0, 2, ptr, col, val, ptr, col, val, f, 0.1) == E and not out.value
    assert create(2, 2, ptr, col, val, ptr, col, val, f, 0.0) == E
    bad = np.array([0, 2, 1], dtype=np.int32)                 # decreasing row pointer
    assert create(2, 2, bad, col, val, ptr, col, val, f, 0.1) == E
    badc = np.array([0, 5], dtype=np.int32)                   # column out of range
    assert create(2, 2, ptr, badc, val, ptr, col, val, f, 0.1) == E
    assert create(2, 2, ptr, col, val, ptr, col, val, f, 0.1, flags=32) == E        # unknown flag
    nanv = np.array([1.0, np.nan])
    assert create(2, 2, ptr, col, nanv, ptr, col, val, f, 0.1) == _lib.ROM_E_NONFINITE
    assert lib.rom_fom_run(None, 1, None, 0, 1, None, None, None) == E
    assert lib.rom_fom_project(None, 1, 1, None, None, None, None, None, None) == E
    assert lib.rom_fom_destroy(None) == _lib.ROM_OK
    k = C.c_int32(5)
    sig = np.zeros(4)
    assert lib.rom_pod(10, 4, None, 0.0, 2, None, sig.ctypes.data_as(pd), C.byref(k), None) == E and k.value == 0
    X = C.c_void_p(16)   # never dereferenced: the arguments are rejected first
    assert lib.rom_pod(3, 4, X, 0.0, 2, X, sig.ctypes.data_as(pd), C.byref(k), None) == E      # n < ns
    assert lib.rom_pod(10, 4, X, 0.0, 5, X, sig.ctypes.data_as(pd), C.byref(k), None) == E     # kmax > ns
    assert lib.rom_pod(10, 4, X, 1.0, 2, X, sig.ctypes.data_as(pd), C.byref(k), None) == E     # tol >= 1


def test_check_finite_rejects_bad_arguments():
    lib = _lib.load()
    E = _lib.ROM_E_ARG
    assert lib.rom_check_finite(None, 4, None, None, None) == E
