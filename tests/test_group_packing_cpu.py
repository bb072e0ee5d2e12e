"""Host logic of the grouped plans' row-split part (no GPU): the packing of
64-sample groups of different padded K into cooperative launches of 8 XCDs
x 32 workgroups, through the rom_debug_pack_groups test hook.

Checked on random K lists and on the 64-instance grouped workload's
draws: every group is placed once; its K / 64 row tiles sit in consecutive
slots of one XCD of its launch, numbered 0 .. R-1; no slot holds two tiles;
the largest group opens the first launch; groups are placed in order of
decreasing K, so a launch never holds a group larger than every group of
an earlier launch; and no launch could be avoided by the first-fit rule
(a group opened a new launch only when no earlier launch had room).
"""
import ctypes as C

import numpy as np
import pytest

import synth
from paper_2009_11742_amd import _lib


def _pack(kp, max_launches=64):
    lib = _lib.load()
    n = len(kp)
    arr = (C.c_int32 * max(n, 1))(*kp)
    launch = (C.c_int32 * max(n, 1))()
    member = (C.c_int32 * max(n, 1))()
    maps = (C.c_int32 * (256 * max_launches))()
    nl = lib.rom_debug_pack_groups(arr, n, launch, member, maps, max_launches)
    return nl, list(launch)[:n], list(member)[:n], np.array(maps, dtype=np.int64).reshape(max_launches, 256)


def _check(kp):
    nl, launch, member, maps = _pack(kp)
    assert nl >= (1 if kp else 0)
    n = len(kp)
    seen = set()
    for q in range(n):
        l, lg, R = launch[q], member[q], kp[q] // 64
        assert 0 <= l < nl
        assert (l, lg) not in seen
        seen.add((l, lg))
        slots = np.nonzero((maps[l] >= 0) & (maps[l] // 32 == lg))[0]
        assert len(slots) == R, (q, len(slots), R)
        xcds = set(int(s) // 32 for s in slots)
        assert len(xcds) == 1                                   # one XCD
        assert sorted(maps[l][slots] % 32) == list(range(R))    # tiles 0 .. R-1
        assert np.all(np.diff(slots) == 1)                      # consecutive slots
    for l in range(nl):
        used = maps[l][maps[l] >= 0]
        assert len(used) == len(set(used.tolist()))             # no slot twice
        assert len(used) <= 256
    # placement order: the largest group opens launch 0
    if n:
        big = [q for q in range(n) if kp[q] == max(kp)]
        assert launch[big[0]] == 0 and member[big[0]] == 0
    # first fit: the group that opened launch l (member 0) did not fit any
    # earlier launch (no XCD there had R free slots when it was placed)
    order = sorted(range(n), key=lambda q: -kp[q])
    free = {}
    for q in order:
        l, R = launch[q], kp[q] // 64
        if member[q] == 0 and l > 0:
            for l2 in range(l):
                assert max(free[l2]) < R, (q, l2)
        if l not in free:
            free[l] = [32] * 8
        # recover the XCD from the slot map
        x = int(np.nonzero((maps[l] >= 0) & (maps[l] // 32 == member[q]))[0][0]) // 32
        free[l][x] -= R
        assert free[l][x] >= 0
    return nl


def test_pack_single_sizes():
    assert _check([1024] * 16) == 1          # 2 groups of 16 tiles per XCD
    assert _check([1024] * 17) == 2
    assert _check([704] * 16) == 1           # 2 x 11 of 32 slots per XCD
    assert _check([704] * 18) == 2
    assert _check([2048] * 8) == 1
    assert _check([128] * 128) == 1          # 16 groups of 2 tiles per XCD
    assert _check([]) == 0


def test_pack_random_lists():
    rng = np.random.default_rng(7)
    for trial in range(200):
        n = int(rng.integers(1, 120))
        kp = [int(64 * rng.integers(2, 33)) for _ in range(n)]
        _check(kp)


def test_pack_grouped_workload_draws():
    """The 64-instance grouped workload from K = 384 up (the plan's measured
    threshold): 1194 row tiles in 138 groups fit 5 launches."""
    kp = []
    for K, M, _ in synth.grouped_draws(64, base_seed=0):
        if K >= 384:
            kp += [K] * ((M + 63) // 64)
    nl = _check(kp)
    tiles = sum(k // 64 for k in kp)
    assert nl >= -(-tiles // 256)
    assert nl <= -(-tiles // 256) + 1
    print("grouped workload: %d groups, %d tiles, %d launches" % (len(kp), tiles, nl))


def test_pack_rejects_bad_sizes():
    assert _pack([96])[0] == -1
    assert _pack([4096])[0] == -1
    assert _pack([1024] * 40, max_launches=2)[0] == -1
