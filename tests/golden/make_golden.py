"""Write the fixtures of this folder.  Run from the repository root:

    python tests/golden/make_golden.py

* leapfrog_1x1_exact.txt -- the staggered leapfrog of Sec. 3.1 (eq. (3.3),
  velocity first, then stress with the new velocity) on 1x1 blocks
  Avs = a, Asv = -a, no source, v0 = 1, s0 = 0, stepped in exact rational
  arithmetic (fractions.Fraction; a and dt rational), printed to 25
  significant digits.  One step is the map
  (v, s) -> (v + dt a s, s - dt a (v + dt a s)).
* ricker_points.txt -- closed-form special points of the Ricker wavelet
  (Sec. 3.2 names the signal; unit-peak form u = (1 - 2x) e^{-x},
  x = pi^2 (mu t - 1.5)^2): the peak u = 1 at mu t = 1.5, the zeros at
  mu t - 1.5 = +-1/(sqrt(2) pi), the minima -2 e^{-3/2} at
  mu t - 1.5 = +-sqrt(1.5)/pi.
* oracle_K8_M3_N50.txt -- the oracle's own output on a small seeded
  instance (synth.make_instance(8, 8, 3, seed=123), probe c, 50 steps), as
  a regression fixture for the oracle's arithmetic; written by calling only
  the oracle.
"""
import decimal
import math
import os
import sys
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

CASES = [(Fraction(13, 10), Fraction(1, 10)), (Fraction(1), Fraction(1, 4)), (Fraction(7, 4), Fraction(1, 64))]
STEPS = [1, 2, 3, 10, 100, 1000, 2000]


def dec(x, digits=25):
    ctx = decimal.Context(prec=digits)
    return format(ctx.divide(decimal.Decimal(x.numerator), decimal.Decimal(x.denominator)), ".24e")


def leapfrog_exact():
    lines = ["# staggered leapfrog on 1x1 blocks, exact rationals: a dt n v_n s_n",
             "# written by tests/golden/make_golden.py"]
    for a, dt in CASES:
        v, s = Fraction(1), Fraction(0)
        want = set(STEPS)
        for n in range(1, max(STEPS) + 1):
            v = v + dt * a * s
            s = s - dt * a * v
            if n in want:
                lines.append("%s %s %d %s %s" % (a, dt, n, dec(v), dec(s)))
    return lines


def ricker_points():
    lines = ["# Ricker special points: mu t u(t; mu)", "# written by tests/golden/make_golden.py"]
    for mu in (0.5, 0.8, 1.0):
        pts = [(1.5, 1.0),
               (1.5 + 1.0 / (math.sqrt(2.0) * math.pi), 0.0), (1.5 - 1.0 / (math.sqrt(2.0) * math.pi), 0.0),
               (1.5 + math.sqrt(1.5) / math.pi, -2.0 * math.exp(-1.5)),
               (1.5 - math.sqrt(1.5) / math.pi, -2.0 * math.exp(-1.5))]
        for x, u in pts:
            lines.append("%r %r %r" % (mu, x / mu, u))
    return lines


def oracle_regression():
    import oracle
    import synth
    inst = synth.make_instance(8, 8, 3, seed=123)
    r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 50, c=inst["c"])
    lines = ["# oracle.run_rank2 on synth.make_instance(8, 8, 3, seed=123), c probe, 50 steps",
             "# written by tests/golden/make_golden.py; rows: V (8 x 3), S (8 x 3), J (3)"]
    for name in ("V", "S"):
        for row in r[name]:
            lines.append(name + " " + " ".join(repr(float(x)) for x in row))
    lines.append("J " + " ".join(repr(float(x)) for x in r["J"]))
    return lines


def main():
    for fname, lines in (("leapfrog_1x1_exact.txt", leapfrog_exact()), ("ricker_points.txt", ricker_points()),
                         ("oracle_K8_M3_N50.txt", oracle_regression())):
        with open(os.path.join(HERE, fname), "w") as f:
            f.write("\n".join(lines) + "\n")
        print("wrote", fname)


if __name__ == "__main__":
    main()
