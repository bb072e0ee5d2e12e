"""Process-wide schedule tuning table of the library (argument marshalling).

The library's autotuner fills the table on the first run of each shape; a
table measured earlier can be loaded instead, so runs of known shapes start
without tuning launches.  The text format has one entry per line:

    kv_pad ks_pad m_pad op schedule us_columns us_rowsplit us_columns8 us_resident us_panel

sizes padded to multiples of 64 (m_pad 0: the grouped launch's per-workgroup
tile times), ``op`` one of f64 / f32 / bf16 / fp8, ``schedule`` one of
columns / rowsplit / columns8 / resident / panel, times in microseconds per step
(negative: not applicable; lines of earlier formats, without the resident
or panel times, have none).  ``#`` starts a comment.

``load_default()`` loads the table shipped beside this module
(``tune_mi355x.txt``, written by ``python -m paper_2009_11742_amd.tune``) or
the file named by ``ROM_TUNE_TABLE`` (empty: none).
"""
from __future__ import annotations

import os

from . import _lib

SCHEDULES = ("columns", "rowsplit", "columns8", "resident", "panel")
OPS = ("f64", "f32", "bf16", "fp8")
DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_mi355x.txt")
_loaded_default = False


def entries():
    """The table as a list of dicts (key order)."""
    lib = _lib.load()
    out = []
    for i in range(lib.rom_tune_count()):
        e = _lib.RomTuneEntry()
        _lib.check(lib.rom_tune_get(i, e))
        out.append({"kv_pad": e.kv_pad, "ks_pad": e.ks_pad, "m_pad": e.m_pad, "op": OPS[e.op_type],
                    "schedule": SCHEDULES[e.schedule], "us": [float(u) for u in e.us]})
    return out


def put(kv_pad, ks_pad, m_pad, op, schedule, us):
    """Add or replace one entry; times missing at the end count as not
    measured (-1)."""
    e = _lib.RomTuneEntry(kv_pad, ks_pad, m_pad, OPS.index(op), SCHEDULES.index(schedule))
    us = list(us) + [-1.0] * (_lib.ROM_NSCHEDULES - len(us))
    for i, u in enumerate(us):
        e.us[i] = float(u)
    _lib.check(_lib.load().rom_tune_put(e))


def clear():
    _lib.load().rom_tune_clear()


def format_entry(d):
    return "%d %d %d %s %s %s" % (d["kv_pad"], d["ks_pad"], d["m_pad"], d["op"], d["schedule"],
                                  " ".join("%.3f" % u for u in d["us"]))


def save(path, header=""):
    lines = ["# " + h for h in header.splitlines()] if header else []
    lines += [format_entry(d) for d in entries()]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def load(path):
    """Add every entry of a table file (replacing entries with the same key)."""
    n = 0
    with open(path) as f:
        for ln, line in enumerate(f, 1):
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            p = line.split()
            if not 8 <= len(p) <= 5 + _lib.ROM_NSCHEDULES:
                raise ValueError("%s:%d: expected 8 to %d fields" % (path, ln, 5 + _lib.ROM_NSCHEDULES))
            us = [float(u) for u in p[5:]]
            us += [-1.0] * (_lib.ROM_NSCHEDULES - len(us))
            put(int(p[0]), int(p[1]), int(p[2]), p[3], p[4], us)
            n += 1
    return n


def load_default():
    """Load the shipped table (or $ROM_TUNE_TABLE) once per process."""
    global _loaded_default
    if _loaded_default:
        return
    _loaded_default = True
    path = os.environ.get("ROM_TUNE_TABLE", DEFAULT_TABLE)
    if path and os.path.exists(path):
        load(path)
