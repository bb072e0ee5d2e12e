"""Seeded synthetic inputs for the rank-2 Galerkin ROM workloads.

This module only draws and rounds inputs; it holds none of the method's
arithmetic (no forcing signal, no stepping).  Both the HIP path's tests and the
oracle's tests take their inputs from here.

The paper's own ROM performance study fills the reduced operators with random
data (Sec. 4.2) and uses equal velocity/stress sizes; the recipe below is that
study moved to seeded numpy draws:

  rng  = numpy.random.default_rng(seed)
  Avs  = rng.standard_normal((Kv, Ks)) / sqrt(Ks)     (entries N(0, 1/K))
  Asv  = -Avs^T                                       (skew coupling: the
         leapfrog then conserves a discrete energy)
  b    = rng.standard_normal(Kv)                      (reduced point source)
  mu   = rng.uniform(0.5, 1.0, M)                     (Ricker centre frequencies)
  c    = rng.standard_normal(Kv)                      (probe / receiver row)
  dt   = 0.5 / sigma_max(Avs)                         (FP64 SVD)

All matrices are returned column-major (numpy Fortran order).  ``round_to``
rounds every floating input except mu (kept FP64) to the run's input precision,
so that the oracle and the GPU see the same numbers.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["make_instance", "round_to", "grouped_draws", "make_affine_family", "make_shear_fom",
           "shear_fom_sizes", "fom_periods", "CONFIGS"]

# The five workloads (sizes and step counts) this build measures or checks.
CONFIGS = {
    # plain method, FP64: K=64, M in {1, 8}, 2000 steps
    "plain_fp64": dict(kv=64, ks=64, M=8, nsteps=2000, dtype="f64", seed=0),
    # rank-2 FP32 bench workload: K=256, M=256, 10000 steps
    "rank2_fp32": dict(kv=256, ks=256, M=256, nsteps=10000, dtype="f32", seed=0),
    # precision study: K=M=1024, 5000 steps (BF16 / FP8 / FP32)
    "precision": dict(kv=1024, ks=1024, M=1024, nsteps=5000, dtype="f32", seed=0),
    # batching: 64 instances of uneven K and M, 4000 steps each
    "grouped": dict(G=64, nsteps=4000, dtype="f32", seed=0),
    # differentiation: K=512, M=256, 5000 steps
    "adjoint": dict(kv=512, ks=512, M=256, nsteps=5000, dtype="f32", seed=0),
}


def _fortran(x):
    return np.asfortranarray(x)


def make_instance(kv: int, ks: int, M: int, seed: int = 0, skew: bool = True,
                  random_asv: bool = False):
    """Draw one instance in FP64 (see the module docstring for the recipe).

    With ``skew=False`` the stress operator is a weighted transpose
    Asv = -diag(w) Avs^T, w ~ U[0.5, 1.5] drawn after the other draws: not
    skew, but of the form the staggered finite-difference operators have
    (a positive material weight times the negative transpose, Sec. 3.1), so the
    leapfrog stays stable.  With ``random_asv=True`` Asv is an independent
    N(0, 1/Kv) matrix instead: general, and unstable over long horizons.
    """
    rng = np.random.default_rng(seed)
    Avs = rng.standard_normal((kv, ks)) / math.sqrt(ks)
    b = rng.standard_normal(kv)
    mu = rng.uniform(0.5, 1.0, M)
    c = rng.standard_normal(kv)
    if random_asv:
        Asv = rng.standard_normal((ks, kv)) / math.sqrt(kv)
    elif skew:
        Asv = -Avs.T
    else:
        w = rng.uniform(0.5, 1.5, ks)
        Asv = -(w[:, None] * Avs.T)
    smax = float(np.linalg.svd(Avs, compute_uv=False)[0])
    dt = 0.5 / smax
    return {
        "Avs": _fortran(Avs), "Asv": _fortran(Asv), "b": b.copy(), "mu": mu.copy(),
        "c": c.copy(), "dt": dt, "kv": kv, "ks": ks, "M": M, "seed": seed,
    }


def round_to(inst: dict, dtype: str) -> dict:
    """Round Avs, Asv, b, c and dt to ``dtype`` ('f64' or 'f32'), returned as
    float64 arrays holding exactly representable values; mu stays FP64."""
    if dtype == "f64":
        return dict(inst)
    if dtype != "f32":
        raise ValueError("input precision must be 'f64' or 'f32'")
    out = dict(inst)
    for k in ("Avs", "Asv"):
        out[k] = _fortran(inst[k].astype(np.float32).astype(np.float64))
    for k in ("b", "c"):
        out[k] = inst[k].astype(np.float32).astype(np.float64)
    out["dt"] = float(np.float32(inst["dt"]))
    return out


def grouped_draws(G: int = 64, base_seed: int = 0):
    """(K, M, seed) for each of G instances: K uniform over {128, 192, ..., 768},
    M = clamp(round(exp(U(ln 16, ln 512))), 16, 512), instance seed = base + i."""
    rng = np.random.default_rng(base_seed)
    ks = np.arange(128, 769, 64)
    out = []
    for i in range(G):
        K = int(rng.choice(ks))
        M = int(min(512, max(16, round(math.exp(rng.uniform(math.log(16), math.log(512)))))))
        out.append((K, M, base_seed + i))
    return out


def make_affine_family(kv: int, ks: int, Q: int, P: int, M: int, seed: int = 0, skew: bool = True):
    """Q affine terms of each operator and P parameter points, in FP64.

    Avs_q ~ N(0, 1/Ks) entrywise, Asv_q = -Avs_q^T (skew) or
    -diag(w) Avs_q^T with one w ~ U[0.5, 1.5] shared by all terms; b as in
    ``make_instance``; theta[p] ~ U[0.2, 0.8]^Q; mu[p] ~ U[0.5, 1.0]^M.
    ``smax`` holds sigma_max of each Avs term (FP64 SVD), so a caller can
    bound sigma_max of any combination by sum_q |theta_q| smax_q.  Terms are
    returned as (Q, Kv, Ks) and (Q, Ks, Kv) arrays (row index second).
    """
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((Q, kv, ks)) / math.sqrt(ks)
    b = rng.standard_normal(kv)
    if skew:
        B = -np.transpose(A, (0, 2, 1)).copy()
    else:
        w = rng.uniform(0.5, 1.5, ks)
        B = -(w[None, :, None] * np.transpose(A, (0, 2, 1)))
    theta = rng.uniform(0.2, 0.8, (P, Q))
    mu = rng.uniform(0.5, 1.0, (P, M))
    smax = np.array([float(np.linalg.svd(A[q], compute_uv=False)[0]) for q in range(Q)])
    return {"Avs_terms": A, "Asv_terms": B, "b": b, "theta": theta, "mu": mu, "smax": smax,
            "kv": kv, "ks": ks, "Q": Q, "P": P, "M": M, "seed": seed}


def _csr(nrows, rows, cols, vals):
    """CSR (rowptr int32, col int32, val float64) from COO lists; entries of a
    row sorted by column."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.add.at(ptr, rows + 1, 1)
    ptr = np.cumsum(ptr)
    return ptr.astype(np.int32), cols.astype(np.int32), vals


def shear_fom_sizes(nr: int, nth: int):
    """(N_v, N_s) of the staggered grid of ``make_shear_fom``."""
    return nr * nth, (nr - 1) * nth + nr * (nth - 1)


def make_shear_fom(nr: int, nth: int, rho: float = 2500.0, vs: float = 5000.0, r_cmb: float = 3480e3,
                   r_earth: float = 6371e3, src_depth: float = 640e3, dt: float | None = None):
    """Sparse full-order operators of the axisymmetric shear-wave system on
    a staggered grid (Sec. 3, eqs. (3.1)-(3.2)), for a single homogeneous
    layer (density rho, shear velocity vs: the setup of the paper's FOM
    scaling runs, Appendix A).  Second-order centred differences:

    grid      velocity v at (r_i, th_j), r_i = r_cmb + i dr (i < nr),
              th_j = j dth (j < nth, dth = pi / (nth - 1));
              s_rp at (r_{i+1/2}, th_j), i < nr - 1;  s_tp at (r_i, th_{j+1/2}),
              j < nth - 1.  Index v: i nth + j; stresses: all s_rp (i (nth) + j)
              first, then s_tp (i (nth - 1) + j).
    velocity  rho dv/dt = d s_rp/dr + (1/r) d s_tp/dth + (3 s_rp + 2 cot(th) s_tp)/r + f;
              d/dr and d/dth as centred differences of the two neighbours, the
              undifferentiated stresses as their two-neighbour means.  Rows on
              the axis (j = 0, nth - 1) are zero (v = 0 there).  At r_cmb and
              r_earth (i = 0, nr - 1) the free surface sets s_rp = 0 at the
              velocity point: d s_rp/dr is the one-sided difference over half
              a cell, and the s_rp mean is zero.
    stresses  d s_rp/dt = mu (dv/dr - v/r) at r_{i+1/2} (zero on the axis);
              d s_tp/dt = mu ((1/r) dv/dth - cot(th) v / r) at th_{j+1/2}; v
              undifferentiated as the two-neighbour mean; mu = rho vs^2.
    source    f = e_src / rho at the velocity point nearest to depth
              src_depth in r, at the first theta > 0 (Sec. 3.2).
    dt        default 0.4 min(dr, r_cmb dth) / vs (inside the CFL limit).

    Returns Av (N_v x N_s) and As (N_s x N_v) as CSR (ptr, col, val), f, the
    grid sizes and dt.
    """
    dr = (r_earth - r_cmb) / (nr - 1)
    dth = math.pi / (nth - 1)
    mu_s = rho * vs * vs
    nv = nr * nth
    nrp = (nr - 1) * nth
    ntp = nr * (nth - 1)
    ns = nrp + ntp

    cat = np.concatenate
    # velocity rows (off-axis j = 1 .. nth - 2)
    I, J = np.meshgrid(np.arange(nr), np.arange(1, nth - 1), indexing="ij")
    I, J = I.ravel(), J.ravel()
    r = r_cmb + I * dr
    cot = np.cos(J * dth) / np.sin(J * dth)
    row = I * nth + J
    inner = (I > 0) & (I < nr - 1)
    lo, hi = I == 0, I == nr - 1
    rows = [row[inner], row[inner], row[lo], row[hi], row, row]
    cols = [I[inner] * nth + J[inner], (I[inner] - 1) * nth + J[inner], 0 * nth + J[lo], (nr - 2) * nth + J[hi],
            nrp + I * (nth - 1) + J, nrp + I * (nth - 1) + J - 1]
    vals = [(1.0 / dr + 1.5 / r[inner]) / rho, (-1.0 / dr + 1.5 / r[inner]) / rho,
            np.full(lo.sum(), (2.0 / dr) / rho), np.full(hi.sum(), (-2.0 / dr) / rho),
            (1.0 / (r * dth) + cot / r) / rho, (-1.0 / (r * dth) + cot / r) / rho]
    Av = _csr(nv, cat(rows), cat(cols), cat(vals))

    # s_rp rows (off-axis), then s_tp rows
    I, J = np.meshgrid(np.arange(nr - 1), np.arange(1, nth - 1), indexing="ij")
    I, J = I.ravel(), J.ravel()
    rh = r_cmb + (I + 0.5) * dr
    row = I * nth + J
    rows = [row, row]
    cols = [(I + 1) * nth + J, I * nth + J]
    vals = [mu_s * (1.0 / dr - 0.5 / rh), mu_s * (-1.0 / dr - 0.5 / rh)]
    I, J = np.meshgrid(np.arange(nr), np.arange(nth - 1), indexing="ij")
    I, J = I.ravel(), J.ravel()
    r = r_cmb + I * dr
    coth = np.cos((J + 0.5) * dth) / np.sin((J + 0.5) * dth)
    row = nrp + I * (nth - 1) + J
    rows += [row, row]
    cols += [I * nth + J + 1, I * nth + J]
    vals += [mu_s * (1.0 / (r * dth) - 0.5 * coth / r), mu_s * (-1.0 / (r * dth) - 0.5 * coth / r)]
    As = _csr(ns, cat(rows), cat(cols), cat(vals))

    i_src = int(round((r_earth - src_depth - r_cmb) / dr))
    i_src = min(max(i_src, 0), nr - 1)
    f = np.zeros(nv)
    f[i_src * nth + 1] = 1.0 / rho
    if dt is None:
        dt = 0.4 * min(dr, r_cmb * dth) / vs
    return {"Av": Av, "As": As, "f": f, "nv": nv, "ns": ns, "nr": nr, "nth": nth, "dr": dr, "dth": dth,
            "r_cmb": r_cmb, "rho": rho, "vs": vs, "src": i_src * nth + 1, "dt": float(dt)}


def fom_periods(M: int, seed: int = 0, lo: float = 60.0, hi: float = 80.0):
    """Centre frequencies mu = 1 / T of M forcing samples, periods
    T ~ U(lo, hi) seconds (the rank-2 FOM runs of Appendix A)."""
    rng = np.random.default_rng(seed)
    return 1.0 / rng.uniform(lo, hi, M)
