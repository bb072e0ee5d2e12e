"""Measure the schedule tuning table of this GPU and write it to a file.

    python -m paper_2009_11742_amd.tune [--out PATH] [--quick]

Empties the process table, then runs the library's autotuner on the shapes
of the standard workloads: FP32-state rank-2 runs for K in {256, 512, 1024}
x M in {64, 256, 1024} and K = 2048 at M in {512, 1024} (FP32 operators; BF16
and FP8 at K = M = 1024), and
the grouped launch's per-workgroup tile times for K in {128, 192, ..., 768}.
The operators are random skew pairs (timing does not depend on the values).
Every entry is what the autotuner measured; nothing is edited by hand.
"""
from __future__ import annotations

import argparse
import datetime

import numpy as np
import torch

from . import tuning
from .rom import GroupPlan, Rom

RUN_SHAPES = [(K, M, "f32") for K in (256, 512, 1024) for M in (64, 256, 1024)] + \
             [(2048, 512, "f32"), (2048, 1024, "f32"), (1024, 1024, "bf16"), (1024, 1024, "fp8")]
TILE_K = list(range(128, 769, 64))


def _skew(K, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((K, K)) / np.sqrt(K)
    b = rng.standard_normal(K)
    dt = 0.5 / np.linalg.norm(A, 2)
    return A, -A.T.copy(), b, dt


def tune_runs(shapes, log=print):
    for K, M, ops in shapes:
        A, B, b, dt = _skew(K, K + M)
        rom = Rom(A, B, b, dt, state="f32", ops=ops)
        mu = torch.full((M,), 0.75, dtype=torch.float64, device="cuda")
        V, S = rom.zeros(M)
        rom.run_rank2(mu, V, S, 1)
        rom.check()
        log("K=%d M=%d %s: %s %s" % (K, M, ops, rom.last_schedule, rom.schedule_times(M)))
        rom.close()


def tune_tiles(ks, log=print):
    roms, mus, Vs, Ss = [], [], [], []
    for K in ks:
        A, B, b, dt = _skew(K, K)
        rom = Rom(A, B, b, dt, state="f32")
        V, S = rom.zeros(8)
        roms.append(rom); Vs.append(V); Ss.append(S)
        mus.append(torch.full((8,), 0.75, dtype=torch.float64, device="cuda"))
    plan = GroupPlan(roms, mus, Vs, Ss)      # tunes every bucket's tiles
    plan.close()
    for r in roms:
        r.close()
    for d in tuning.entries():
        if d["m_pad"] == 0:
            log("tile K=%d: %s %s" % (d["kv_pad"], d["schedule"], d["us"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=tuning.DEFAULT_TABLE)
    ap.add_argument("--quick", action="store_true", help="c1 shape and two tile buckets only")
    args = ap.parse_args()
    tuning.clear()
    if args.quick:
        tune_runs([(256, 256, "f32")])
        tune_tiles([128, 768])
    else:
        tune_runs(RUN_SHAPES)
        tune_tiles(TILE_K)
    dev = torch.cuda.get_device_properties(0)
    tuning.save(args.out, header="schedule tuning table: python -m paper_2009_11742_amd.tune\n"
                "device: %s (%d CUs), %s\n"
                "kv_pad ks_pad m_pad op schedule us_columns us_rowsplit us_columns8 us_resident us_panel"
                % (dev.name, dev.multi_processor_count, datetime.date.today().isoformat()))
    print("wrote %s (%d entries)" % (args.out, len(tuning.entries())))


if __name__ == "__main__":
    main()
