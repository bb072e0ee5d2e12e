"""The oracle against the fixtures of tests/golden/ (written by
tests/golden/make_golden.py; see its header for what each file holds).

* leapfrog_1x1_exact.txt: the staggered leapfrog of Sec. 3.1 on 1x1 skew
  blocks in exact rational arithmetic; the oracle (FP64) must follow it to
  rounding (<= 1e-12 over 2000 steps), and the closed form
  G^n = (sin(n th) G - sin((n-1) th) I) / sin th, th = 2 asin(a dt / 2),
  must reproduce the exact values too (so the fixture itself is pinned).
* ricker_points.txt: closed-form special points of the Ricker wavelet.
* oracle_K8_M3_N50.txt: regression fixture of the oracle's own output.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_leapfrog_1x1_exact_fixture():
    rows = _rows("leapfrog_1x1_exact.txt")
    assert len(rows) == 21
    by_case = {}
    for a, dt, n, v, s in rows:
        by_case.setdefault((a, dt), []).append((int(n), float(v), float(s)))
    for (a_s, dt_s), pts in by_case.items():
        a, dt = float(Fraction(a_s)), float(Fraction(dt_s))
        nmax = max(n for n, _, _ in pts)
        r = oracle.run_rank2(np.array([[a]]), np.array([[-a]]), np.zeros(1), dt, np.array([0.75]), nmax,
                             V=np.ones((1, 1)), S=np.zeros((1, 1)), trace=False)
        # the oracle at intermediate steps: split runs
        for n, v, s in pts:
            rn = oracle.run_rank2(np.array([[a]]), np.array([[-a]]), np.zeros(1), dt, np.array([0.75]), n,
                                  V=np.ones((1, 1)), S=np.zeros((1, 1)))
            assert abs(rn["V"][0, 0] - v) <= 1e-12 and abs(rn["S"][0, 0] - s) <= 1e-12, (a, dt, n)
            # the closed form agrees with the exact rational values
            th = 2.0 * math.asin(a * dt / 2.0)
            G = np.array([[1.0, a * dt], [-a * dt, 1.0 - (a * dt) ** 2]])
            Gn = (math.sin(n * th) * G - math.sin((n - 1) * th) * np.eye(2)) / math.sin(th)
            assert abs(Gn[0, 0] - v) <= 1e-11 and abs(Gn[1, 0] - s) <= 1e-11, (a, dt, n)
        assert abs(r["V"][0, 0] - pts[-1][1]) <= 1e-12


def test_ricker_points_fixture():
    rows = _rows("ricker_points.txt")
    assert len(rows) == 15
    for mu, t, u in rows:
        mu, t, u = float(mu), float(t), float(u)
        assert oracle.ricker(t, mu) == pytest.approx(u, rel=1e-13, abs=1e-14)


def test_oracle_regression_fixture():
    rows = _rows("oracle_K8_M3_N50.txt")
    V = np.array([[float(x) for x in r[1:]] for r in rows if r[0] == "V"])
    S = np.array([[float(x) for x in r[1:]] for r in rows if r[0] == "S"])
    J = np.array([float(x) for x in rows[-1][1:]])
    inst = synth.make_instance(8, 8, 3, seed=123)
    r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 50, c=inst["c"])
    scale = max(np.max(np.abs(V)), np.max(np.abs(S)))
    assert np.max(np.abs(r["V"] - V)) <= 1e-14 * scale
    assert np.max(np.abs(r["S"] - S)) <= 1e-14 * scale
    assert np.allclose(r["J"], J, rtol=1e-14, atol=0)
