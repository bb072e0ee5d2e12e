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

__all__ = ["make_instance", "round_to", "grouped_draws", "make_affine_family", "CONFIGS"]

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
