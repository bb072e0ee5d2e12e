"""ctypes loader for ``librom.so`` (the HIP library).  Argument marshalling only.

The library is built in-tree by :mod:`paper_2009_11742_amd.build`.  Loading
fails loudly when it is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
# ROM_LIB overrides the library file (the sanitizer build of the host layer
# is loaded this way by its CPU test)
LIB_PATH = os.environ.get("ROM_LIB") or os.path.join(HERE, "librom.so")

ROM_OK, ROM_E_ARG, ROM_E_NOMEM, ROM_E_DEVICE, ROM_E_UNSTABLE, ROM_E_UNSUPPORTED, \
    ROM_E_NONFINITE, ROM_E_TIMEOUT = range(8)
STATUS_NAMES = ["ROM_OK", "ROM_E_ARG", "ROM_E_NOMEM", "ROM_E_DEVICE", "ROM_E_UNSTABLE",
                "ROM_E_UNSUPPORTED", "ROM_E_NONFINITE", "ROM_E_TIMEOUT"]
ROM_F64, ROM_F32, ROM_BF16, ROM_F8E4M3 = range(4)
ROM_SKEW_CHECK = 1
ROM_SCHED_COLUMNS = 2
ROM_SCHED_ROWSPLIT = 4
ROM_SCHED_COLUMNS8 = 8
ROM_SOURCE_GAUSS1 = 16
ROM_STATE_BF16 = 32
ROM_SCHED_RESIDENT = 64
ROM_SCHED_PANEL = 128
ROM_SCHEDULE_COLUMNS4, ROM_SCHEDULE_ROWSPLIT, ROM_SCHEDULE_COLUMNS8, ROM_SCHEDULE_RESIDENT, ROM_SCHEDULE_PANEL = range(5)
ROM_NSCHEDULES = 5

# Every symbol include/rom.h declares.
EXPORTS = ["rom_create", "rom_destroy", "rom_step_rank1", "rom_run_rank1", "rom_run_rank1_batch", "rom_run_rank2", "rom_run_rank2_noalloc",
           "rom_adjoint", "rom_run_grouped", "rom_group_create", "rom_group_run", "rom_group_destroy",
           "rom_group_schedule", "rom_group_times", "rom_group_split_k", "rom_group_check",
           "rom_get_operators", "rom_energy", "rom_check", "rom_debug_force_timeout", "rom_debug_pack_groups", "rom_check_finite", "rom_last_schedule", "rom_schedule_times",
           "rom_tune_count", "rom_tune_get", "rom_tune_put", "rom_tune_clear", "rom_run_receivers",
           "rom_affine_create", "rom_affine_instance", "rom_affine_destroy",
           "rom_fom_create", "rom_fom_run", "rom_fom_project", "rom_fom_destroy", "rom_pod",
           "rom_last_error", "rom_version"]


class RomConfig(C.Structure):
    _fields_ = [("kv", C.c_int32), ("ks", C.c_int32), ("dt", C.c_double),
                ("op_type", C.c_int), ("state_type", C.c_int), ("flags", C.c_uint32)]


class RomTuneEntry(C.Structure):
    _fields_ = [("kv_pad", C.c_int32), ("ks_pad", C.c_int32), ("m_pad", C.c_int32),
                ("op_type", C.c_int), ("schedule", C.c_int32), ("us", C.c_double * ROM_NSCHEDULES)]


class RomError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__("%s: %s" % (name, msg))


_lock = threading.Lock()
_lib = None

_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_d = C.c_double
_pd = C.POINTER(C.c_double)


def load():
    """Load librom.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librom.so is not built (run paper_2009_11742_amd.build.build() "
                               "or __graft_entry__.build()); there is no fallback path")
        lib = C.CDLL(LIB_PATH)
        lib.rom_create.restype = C.c_int
        lib.rom_create.argtypes = [C.POINTER(RomConfig), _pd, _pd, _pd, _vp, C.POINTER(_vp)]
        lib.rom_destroy.restype = C.c_int
        lib.rom_destroy.argtypes = [_vp]
        lib.rom_step_rank1.restype = C.c_int
        lib.rom_step_rank1.argtypes = [_vp, _vp, _vp, _i64, _d, _vp]
        lib.rom_run_rank1.restype = C.c_int
        lib.rom_run_rank1.argtypes = [_vp, _vp, _vp, _d, _i64, _i64, _vp]
        lib.rom_run_rank1_batch.restype = C.c_int
        lib.rom_run_rank1_batch.argtypes = [_vp, _i32, _vp, _i64, _i64, _vp, _vp, _vp]
        lib.rom_run_rank2.restype = C.c_int
        lib.rom_run_rank2.argtypes = [_vp, _i32, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp]
        lib.rom_run_rank2_noalloc.restype = C.c_int
        lib.rom_run_rank2_noalloc.argtypes = [_vp, _i32, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp]
        lib.rom_adjoint.restype = C.c_int
        lib.rom_adjoint.argtypes = [_vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                    _i32, _vp]
        lib.rom_run_grouped.restype = C.c_int
        lib.rom_run_grouped.argtypes = [C.POINTER(_vp), _i32, C.POINTER(_i32), C.POINTER(_vp),
                                        _i64, C.POINTER(_vp), C.POINTER(_vp), _vp]
        lib.rom_group_create.restype = C.c_int
        lib.rom_group_create.argtypes = [C.POINTER(_vp), _i32, C.POINTER(_i32), C.POINTER(_vp),
                                         C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp)]
        lib.rom_group_run.restype = C.c_int
        lib.rom_group_run.argtypes = [_vp, _i64, _i64, _vp]
        lib.rom_group_destroy.restype = C.c_int
        lib.rom_group_destroy.argtypes = [_vp]
        _pi32 = C.POINTER(_i32)
        lib.rom_fom_create.restype = C.c_int
        lib.rom_fom_create.argtypes = [_i32, _i32, _pi32, _pi32, _pd, _pi32, _pi32, _pd, _pd, _d, C.c_uint32, _vp,
                                       C.POINTER(_vp)]
        lib.rom_fom_run.restype = C.c_int
        lib.rom_fom_run.argtypes = [_vp, _i32, _vp, _i64, _i64, _vp, _vp, _vp]
        lib.rom_fom_project.restype = C.c_int
        lib.rom_fom_project.argtypes = [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp]
        lib.rom_fom_destroy.restype = C.c_int
        lib.rom_fom_destroy.argtypes = [_vp]
        lib.rom_pod.restype = C.c_int
        lib.rom_pod.argtypes = [_i64, _i32, _vp, _d, _i32, _vp, _pd, _pi32, _vp]
        lib.rom_check_finite.restype = C.c_int
        lib.rom_check_finite.argtypes = [_vp, _i32, _vp, _vp, _vp]
        lib.rom_group_schedule.restype = _i32
        lib.rom_group_schedule.argtypes = [_vp]
        lib.rom_group_split_k.restype = _i32
        lib.rom_group_split_k.argtypes = [_vp]
        lib.rom_group_times.restype = C.c_int
        lib.rom_group_times.argtypes = [_vp, _pd]
        lib.rom_group_check.restype = C.c_int
        lib.rom_group_check.argtypes = [_vp, _vp]
        lib.rom_get_operators.restype = C.c_int
        lib.rom_get_operators.argtypes = [_vp, _pd, _pd, _pd]
        lib.rom_energy.restype = C.c_int
        lib.rom_energy.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp]
        lib.rom_check.restype = C.c_int
        lib.rom_check.argtypes = [_vp, _vp]
        lib.rom_debug_force_timeout.restype = C.c_int
        lib.rom_debug_force_timeout.argtypes = [_i32]
        lib.rom_debug_pack_groups.restype = _i32
        lib.rom_debug_pack_groups.argtypes = [C.POINTER(_i32), _i32, C.POINTER(_i32), C.POINTER(_i32),
                                              C.POINTER(_i32), _i32]
        lib.rom_last_schedule.restype = C.c_int32
        lib.rom_last_schedule.argtypes = [_vp]
        lib.rom_schedule_times.restype = C.c_int
        lib.rom_schedule_times.argtypes = [_vp, _i32, C.POINTER(_d)]
        lib.rom_affine_create.restype = C.c_int
        lib.rom_affine_create.argtypes = [C.POINTER(RomConfig), _i32, _pd, _pd, _pd, _vp, C.POINTER(_vp)]
        lib.rom_affine_instance.restype = C.c_int
        lib.rom_affine_instance.argtypes = [_vp, _pd, _d, _vp, C.POINTER(_vp)]
        lib.rom_affine_destroy.restype = C.c_int
        lib.rom_affine_destroy.argtypes = [_vp]
        lib.rom_run_receivers.restype = C.c_int
        lib.rom_run_receivers.argtypes = [_vp, _i32, _vp, _i64, _i64, _vp, _vp, _i32, _vp, _vp, _vp, _vp]
        lib.rom_tune_count.restype = C.c_int32
        lib.rom_tune_count.argtypes = []
        lib.rom_tune_get.restype = C.c_int
        lib.rom_tune_get.argtypes = [_i32, C.POINTER(RomTuneEntry)]
        lib.rom_tune_put.restype = C.c_int
        lib.rom_tune_put.argtypes = [C.POINTER(RomTuneEntry)]
        lib.rom_tune_clear.restype = None
        lib.rom_tune_clear.argtypes = []
        lib.rom_last_error.restype = C.c_char_p
        lib.rom_last_error.argtypes = []
        lib.rom_version.restype = C.c_char_p
        lib.rom_version.argtypes = []
        _lib = lib
        return lib


def check(status: int):
    if status != ROM_OK:
        msg = load().rom_last_error().decode(errors="replace")
        raise RomError(status, msg)
