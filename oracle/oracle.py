"""ctypes front end of the FP64 oracle in ``rom_oracle.c`` (test infrastructure).

All matrices are numpy float64 arrays in column-major (Fortran) order:
operators ``Avs`` (Kv x Ks) and ``Asv`` (Ks x Kv), states ``V`` (Kv x M) and
``S`` (Ks x M), one sample per column.  The functions copy what they must and
never touch the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rom_oracle.c")
_LIB = os.path.join(_HERE, "liborom.so")
_lock = threading.Lock()
_lib = None

_d = C.c_double
_i = C.c_int
_i64 = C.c_int64
_pd = C.POINTER(C.c_double)


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=True)
            lib = C.CDLL(_LIB)
            lib.orc_ricker.restype = _d
            lib.orc_ricker.argtypes = [_d, _d]
            lib.orc_ricker_dmu.restype = _d
            lib.orc_ricker_dmu.argtypes = [_d, _d]
            lib.orc_step_rank1.restype = None
            lib.orc_step_rank1.argtypes = [_i, _i, _pd, _pd, _pd, _d, _i64, _d, _pd, _pd, _i]
            lib.orc_run_rank2.restype = _i
            lib.orc_run_rank2.argtypes = [_i, _i, _pd, _pd, _pd, _d, _i, _pd, _i64, _i64,
                                          _pd, _pd, _pd, _pd, _pd, _i]
            lib.orc_energy.restype = None
            lib.orc_energy.argtypes = [_i, _i, _pd, _d, _i, _pd, _pd, _pd]
            lib.orc_adjoint.restype = _i
            lib.orc_adjoint.argtypes = [_i, _i, _pd, _pd, _pd, _d, _i, _pd, _i64, _pd,
                                        _pd, _pd, _pd, _pd, _pd, _pd, _i64, _i]
            lib.orc_num_threads.restype = _i
            lib.orc_num_threads.argtypes = []
            lib.orc_round_bf16.restype = _d
            lib.orc_round_bf16.argtypes = [_d]
            lib.orc_quantize_e4m3.restype = _d
            lib.orc_quantize_e4m3.argtypes = [_i64, _pd, _pd, _d]
            _pi = C.POINTER(C.c_int32)
            lib.orc_fom_run.restype = _i
            lib.orc_fom_run.argtypes = [_i, _i, _pi, _pi, _pd, _pi, _pi, _pd, _pd, _d, _i, _pd, _i64, _i64,
                                        _pd, _pd, _i]
            lib.orc_gauss1.restype = _d
            lib.orc_gauss1.argtypes = [_d, _d]
            lib.orc_gauss1_dmu.restype = _d
            lib.orc_gauss1_dmu.argtypes = [_d, _d]
            _lib = lib
    return _lib


def _f64(a, shape=None):
    """Column-major float64 copy/view of ``a`` (Fortran order)."""
    x = np.asfortranarray(np.asarray(a, dtype=np.float64))
    if shape is not None and x.shape != tuple(shape):
        x = x.reshape(shape, order="F")
    return x


def _p(x):
    return None if x is None else x.ctypes.data_as(_pd)


def num_threads() -> int:
    return int(_load().orc_num_threads())


SOURCES = {"ricker": 0, "gauss1": 1}


def _src(source):
    """Source kind: 'ricker' (0) or 'gauss1' (1, first derivative of a
    Gaussian); see rom_oracle.c for both signals."""
    if isinstance(source, str):
        return SOURCES[source]
    if int(source) not in (0, 1):
        raise ValueError("source must be 'ricker' or 'gauss1'")
    return int(source)


def gauss1(t, mu):
    lib = _load()
    return np.vectorize(lambda tt, mm: lib.orc_gauss1(float(tt), float(mm)))(t, mu)


def gauss1_dmu(t, mu):
    lib = _load()
    return np.vectorize(lambda tt, mm: lib.orc_gauss1_dmu(float(tt), float(mm)))(t, mu)


def ricker(t, mu):
    lib = _load()
    return np.vectorize(lambda tt, mm: lib.orc_ricker(float(tt), float(mm)))(t, mu)


def ricker_dmu(t, mu):
    lib = _load()
    return np.vectorize(lambda tt, mm: lib.orc_ricker_dmu(float(tt), float(mm)))(t, mu)


def step_rank1(Avs, Asv, b, dt, n, mu, v, s, source="ricker"):
    """One rank-1 leapfrog step of one sample; returns new (v, s)."""
    Avs = _f64(Avs); Asv = _f64(Asv)
    kv, ks = Avs.shape
    assert Asv.shape == (ks, kv)
    b = _f64(b).reshape(kv)
    v = np.array(v, dtype=np.float64).reshape(kv).copy()
    s = np.array(s, dtype=np.float64).reshape(ks).copy()
    _load().orc_step_rank1(kv, ks, _p(Avs), _p(Asv), _p(b), float(dt), int(n), float(mu),
                           _p(v), _p(s), _src(source))
    return v, s


def run_rank2(Avs, Asv, b, dt, mu, nsteps, V=None, S=None, n0=0, c=None, trace=False, source="ricker"):
    """Integrate ``nsteps`` steps from step index ``n0``.

    Returns a dict with V, S (Kv x M / Ks x M, Fortran order) and, when a probe
    ``c`` is given, J (M, accumulated from zero) and optionally the trace y
    (nsteps x M).
    """
    Avs = _f64(Avs); Asv = _f64(Asv)
    kv, ks = Avs.shape
    assert Asv.shape == (ks, kv)
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1))
    M = mu.size
    b = _f64(b).reshape(kv)
    V = np.zeros((kv, M), order="F") if V is None else np.array(V, dtype=np.float64, order="F", copy=True)
    S = np.zeros((ks, M), order="F") if S is None else np.array(S, dtype=np.float64, order="F", copy=True)
    assert V.shape == (kv, M) and S.shape == (ks, M)
    cc = None if c is None else np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(kv))
    J = np.zeros(M) if cc is not None else None
    y = np.zeros((int(nsteps), M)) if (cc is not None and trace) else None
    rc = _load().orc_run_rank2(kv, ks, _p(Avs), _p(Asv), _p(b), float(dt), M, _p(mu), int(n0),
                               int(nsteps), _p(V), _p(S), _p(cc), _p(J), _p(y), _src(source))
    if rc != 0:
        raise MemoryError("oracle run failed")
    out = {"V": V, "S": S}
    if cc is not None:
        out["J"] = J
        if trace:
            out["y"] = y
    return out


def receivers(Avs, Asv, b, dt, mu, nsteps, C, V=None, S=None, n0=0, source="ricker"):
    """Seismograms at R receivers (the reconstruction of the velocity at
    target points from single rows of the velocity basis, Sec. 4.5):
    Y[k, r, m] = C[r] . V_m after step n0 + k, for k = 0 .. nsteps - 1.

    C is R x Kv (one receiver row per row).  The run is stepped one step at a
    time through run_rank2, which is bitwise identical to one run in the
    oracle.  Returns Y (nsteps, R, M) and the final V, S.
    """
    Avs = _f64(Avs); Asv = _f64(Asv)
    kv, ks = Avs.shape
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1))
    M = mu.size
    Cm = np.asarray(C, dtype=np.float64).reshape(-1, kv)
    R = Cm.shape[0]
    V = np.zeros((kv, M), order="F") if V is None else np.array(V, dtype=np.float64, order="F", copy=True)
    S = np.zeros((ks, M), order="F") if S is None else np.array(S, dtype=np.float64, order="F", copy=True)
    Y = np.zeros((int(nsteps), R, M))
    for k in range(int(nsteps)):
        out = run_rank2(Avs, Asv, b, dt, mu, 1, V=V, S=S, n0=n0 + k, source=source)
        V, S = out["V"], out["S"]
        for r in range(R):
            for m in range(M):
                Y[k, r, m] = float(np.dot(Cm[r], V[:, m]))
    return {"Y": Y, "V": V, "S": S}


def affine_operator(terms, theta):
    """Operator of an affinely parametrised family at one parameter point:
    sum_q theta_q T_q, the parametrisation under which the reduced operators
    of many parameter points can be assembled from Q precomputed terms
    (Sec. 2 allows an affine system matrix; Sec. 5 names fast assembly as the
    condition for the rank-3 generalisation).

    terms: (Q, R, C) array, theta: Q coefficients.  Summed in FP64 in the
    order q = 0, 1, ..., Q-1, each product and sum rounded on its own.
    """
    T = np.asarray(terms, dtype=np.float64)
    th = np.asarray(theta, dtype=np.float64).reshape(-1)
    if T.ndim != 3 or T.shape[0] != th.size:
        raise ValueError("terms must be (Q, R, C) with Q = len(theta)")
    acc = th[0] * T[0]
    for q in range(1, th.size):
        acc = acc + th[q] * T[q]
    return acc


def _csr3(A):
    ptr, col, val = A
    return (np.ascontiguousarray(ptr, dtype=np.int32), np.ascontiguousarray(col, dtype=np.int32),
            np.ascontiguousarray(val, dtype=np.float64))


def fom_run(Av, As, f, dt, mu, nsteps, V=None, S=None, n0=0, source="ricker"):
    """Rank-2 full-order model of the staggered system (Sec. 3, eq. (3.2)),
    leapfrog as for the ROM.  Av (Nv x Ns) and As (Ns x Nv) are CSR triples
    (ptr, col, val); f the Nv source vector; states row-major (N x M, one
    sample per column).  Returns the final V and S."""
    avp, avc, avv = _csr3(Av)
    asp, asc, asv = _csr3(As)
    nv, ns = avp.size - 1, asp.size - 1
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1))
    M = mu.size
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(nv))
    V = np.zeros((nv, M)) if V is None else np.array(V, dtype=np.float64, order="C", copy=True)
    S = np.zeros((ns, M)) if S is None else np.array(S, dtype=np.float64, order="C", copy=True)
    assert V.shape == (nv, M) and S.shape == (ns, M)
    pi = C.POINTER(C.c_int32)
    rc = _load().orc_fom_run(nv, ns, avp.ctypes.data_as(pi), avc.ctypes.data_as(pi), _p(avv),
                             asp.ctypes.data_as(pi), asc.ctypes.data_as(pi), _p(asv), _p(f), float(dt), M,
                             _p(mu), int(n0), int(nsteps), _p(V), _p(S), _src(source))
    if rc != 0:
        raise MemoryError("oracle run failed")
    return {"V": V, "S": S}


def csr_dense(A, ncols):
    """Dense form of a CSR triple (duplicates summed)."""
    ptr, col, val = _csr3(A)
    n = ptr.size - 1
    D = np.zeros((n, ncols))
    for r in range(n):
        for k in range(ptr[r], ptr[r + 1]):
            D[r, col[k]] += val[k]
    return D


def project(Av, As, f, Phi_v, Phi_s):
    """Galerkin projection of the full-order operators onto orthonormal
    bases (Sec. 2.2 and eq. (3.3)): Avs = Phi_v^T Av Phi_s,
    Asv = Phi_s^T As Phi_v, b = Phi_v^T f.  Phi_v (Nv x Kv), Phi_s (Ns x Kv)
    dense; the sparse products go row by row over the stored entries, the
    reductions over the full-order index are library matrix products."""
    Phi_v = np.asarray(Phi_v, dtype=np.float64)
    Phi_s = np.asarray(Phi_s, dtype=np.float64)

    def spmm(A, X):
        ptr, col, val = _csr3(A)
        Y = np.zeros((ptr.size - 1, X.shape[1]))
        rows = np.repeat(np.arange(ptr.size - 1), np.diff(ptr))
        np.add.at(Y, rows, val[:, None] * X[col])
        return Y
    Avs = Phi_v.T @ spmm(Av, Phi_s)
    Asv = Phi_s.T @ spmm(As, Phi_v)
    b = Phi_v.T @ np.asarray(f, dtype=np.float64)
    return Avs, Asv, b


def pod_rank(sigma, tol):
    """Smallest k whose leading singular values hold at least 1 - tol of
    the snapshot energy sum sigma_i^2 (Sec. 4.4's truncation criterion)."""
    e = np.asarray(sigma, dtype=np.float64) ** 2
    tot = e.sum()
    c = np.cumsum(e)
    return int(np.searchsorted(c, (1.0 - tol) * tot, side="left") + 1) if tot > 0 else 0


def pod(X, tol=None, k=None):
    """Proper orthogonal decomposition of a snapshot matrix X (N x ns, one
    snapshot per column): the left singular vectors of the thin SVD, kept to
    k columns (given, or by the energy criterion with tolerance tol).
    Returns (Phi (N x k), sigma (all ns, descending), k)."""
    X = np.asarray(X, dtype=np.float64)
    U, s, _ = np.linalg.svd(X, full_matrices=False)
    if k is None:
        k = pod_rank(s, tol) if tol is not None else s.size
    k = min(int(k), s.size)
    return U[:, :k], s, k


def percentile_index(p, M):
    """0-based index of the nearest-rank p-th percentile of M sorted values:
    the ceil(p M / 100)-th smallest, at least the smallest."""
    return max(1, -(-int(p) * int(M) // 100)) - 1


def ensemble_stats(Y, percentiles=(5, 50, 95)):
    """Statistics over the sample axis (last) of Y (..., M): mean, variance
    (population, 1/M) and nearest-rank percentiles.  Returns an array
    (..., 2 + len(percentiles)): mean, var, then the percentiles."""
    Y = np.asarray(Y, dtype=np.float64)
    M = Y.shape[-1]
    mean = Y.sum(axis=-1) / M
    var = ((Y - mean[..., None]) ** 2).sum(axis=-1) / M
    srt = np.sort(Y, axis=-1)
    cols = [mean, var] + [srt[..., percentile_index(p, M)] for p in percentiles]
    return np.stack(cols, axis=-1)


def energy(Avs, dt, V, S):
    """Modified discrete energy |v|^2 + |s|^2 + dt v^T Avs s per column."""
    Avs = _f64(Avs)
    kv, ks = Avs.shape
    V = _f64(V); S = _f64(S)
    M = V.shape[1]
    E = np.zeros(M)
    _load().orc_energy(kv, ks, _p(Avs), float(dt), M, _p(V), _p(S), _p(E))
    return E


def adjoint(Avs, Asv, b, dt, mu, nsteps, c, V0=None, S0=None, stride=0, source="ricker"):
    """J and its partial gradients w.r.t. Avs, Asv and mu (discrete adjoint)."""
    Avs = _f64(Avs); Asv = _f64(Asv)
    kv, ks = Avs.shape
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1))
    M = mu.size
    b = _f64(b).reshape(kv)
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(kv))
    V0 = None if V0 is None else _f64(V0, (kv, M))
    S0 = None if S0 is None else _f64(S0, (ks, M))
    J = np.zeros(M); dmu = np.zeros(M)
    dAvs = np.zeros((kv, ks), order="F"); dAsv = np.zeros((ks, kv), order="F")
    rc = _load().orc_adjoint(kv, ks, _p(Avs), _p(Asv), _p(b), float(dt), M, _p(mu), int(nsteps),
                             _p(c), _p(V0), _p(S0), _p(J), _p(dAvs), _p(dAsv), _p(dmu), int(stride),
                             _src(source))
    if rc != 0:
        raise MemoryError("oracle adjoint failed")
    return {"J": J, "dAvs": dAvs, "dAsv": dAsv, "dmu": dmu}


def round_bf16(x):
    """Elementwise x -> FP32 -> bfloat16 (RNE), as float64."""
    lib = _load()
    x = np.asarray(x, dtype=np.float64)
    return np.vectorize(lambda v: lib.orc_round_bf16(float(v)))(x).astype(np.float64)


def run_rank2_state_bf16(Avs, Asv, b, dt, mu, nsteps, V=None, S=None, n0=0, source="ricker"):
    """The leapfrog of eq. (3.3) (Sec. 3.1) with the state operand of every
    product rounded to BF16 (x -> FP32 -> bfloat16, RNE), the precision
    extension's single-operand form: per step
        V <- V + dt (Avs bf16(S) + b u(t_n; mu)^T),  then  S <- S + dt Asv bf16(V)
    with the new V; everything else in FP64.  A plain numpy loop (the
    rounding makes the result depend on every intermediate), for a few steps
    on small sizes.  Returns V, S (Fortran order).
    """
    Avs = _f64(Avs); Asv = _f64(Asv)
    kv, ks = Avs.shape
    assert Asv.shape == (ks, kv)
    mu = np.asarray(mu, dtype=np.float64).reshape(-1)
    M = mu.size
    b = _f64(b).reshape(kv)
    V = np.zeros((kv, M), order="F") if V is None else np.array(V, dtype=np.float64, order="F", copy=True)
    S = np.zeros((ks, M), order="F") if S is None else np.array(S, dtype=np.float64, order="F", copy=True)
    signal = ricker if _src(source) == 0 else gauss1
    for n in range(int(n0), int(n0) + int(nsteps)):
        u = np.atleast_1d(signal(n * float(dt), mu))
        V = V + float(dt) * (Avs @ round_bf16(S) + np.outer(b, u))
        S = S + float(dt) * (Asv @ round_bf16(V))
    return {"V": np.asfortranarray(V), "S": np.asfortranarray(S)}


def quantize_e4m3(x, amax=0.0):
    """Per-tensor scaled FP8 E4M3 quantisation; returns (dequantised, scale)."""
    x = np.asarray(x, dtype=np.float64)
    flat = np.ascontiguousarray(x.reshape(-1, order="F"))
    out = np.zeros_like(flat)
    scale = _load().orc_quantize_e4m3(flat.size, _p(flat), _p(out), float(amax))
    return out.reshape(x.shape, order="F"), scale
