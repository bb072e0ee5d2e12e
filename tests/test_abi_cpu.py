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
    assert _create(_lib.RomConfig(8, 8, dt, _lib.ROM_F32, _lib.ROM_F32, 0x80), A, B, b)[0] == _lib.ROM_E_ARG
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
