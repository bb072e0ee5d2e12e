"""Python front end of the HIP library (argument marshalling only).

Every computation runs in the library's kernels; torch provides device memory
and streams.  State layout: a state matrix of K rows and M samples is a torch
tensor of shape (M, K), contiguous, i.e. K x M column-major with one sample per
contiguous row of the tensor (the library's column-major convention).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib, tuning
from ._lib import RomConfig, check

tuning.load_default()

_DT = {"f64": (_lib.ROM_F64, torch.float64), "f32": (_lib.ROM_F32, torch.float32)}
_OPS = {"f64": _lib.ROM_F64, "f32": _lib.ROM_F32, "bf16": _lib.ROM_BF16, "fp8": _lib.ROM_F8E4M3}
# FP32-state rank-2 schedule: "auto" (the autotuner's table), "columns"
# (4-column blocks), "rowsplit" (row-split where it applies), "columns8"
# (8-column blocks, FP32 operators), "resident" (skew FP32 pairs with Kv, Ks
# <= 256: the whole operator in each workgroup's registers, one sample each),
# "panel" (FP32 operators, any size: one matrix-product launch per half-step)
# source signal: the Ricker wavelet or the first derivative of a Gaussian
_SOURCE = {"ricker": 0, "gauss1": _lib.ROM_SOURCE_GAUSS1}
# state operand of the BF16 / FP8 products: the BF16 pair or bf16(x) alone
_STATE_OPERAND = {"pair": 0, "single": _lib.ROM_STATE_BF16}
_SCHED = {"auto": 0, "columns": _lib.ROM_SCHED_COLUMNS, "rowsplit": _lib.ROM_SCHED_ROWSPLIT,
          "columns8": _lib.ROM_SCHED_COLUMNS8, "resident": _lib.ROM_SCHED_RESIDENT, "panel": _lib.ROM_SCHED_PANEL}


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _host_f64(a, shape):
    x = np.asfortranarray(np.asarray(a, dtype=np.float64))
    if x.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (shape, x.shape))
    return x


class Rom:
    """One ROM instance on the current device.

    Avs (Kv x Ks), Asv (Ks x Kv) and b (Kv) are host arrays (copied).  ``state``
    is 'f64' or 'f32'; ``ops`` is the operator precision in the products
    ('f64', 'f32', 'bf16', 'fp8'; default: the state precision).  With BF16 /
    FP8 operators and FP32 states, ``state_operand`` 'pair' feeds each state
    value to the products as two BF16 values (about 16 bits), 'single' as one
    (one MFMA pass, about 8 bits; faster, less accurate).
    """

    def __init__(self, Avs, Asv, b, dt, state="f32", ops=None, skew_check=False, schedule="auto", stream=None,
                 source="ricker", state_operand="pair"):
        Avs = np.asarray(Avs)
        kv, ks = Avs.shape
        self.kv, self.ks, self.dt, self.state = int(kv), int(ks), float(dt), state
        code, self.torch_dtype = _DT[state]
        A = _host_f64(Avs, (kv, ks))
        B = _host_f64(Asv, (ks, kv))
        bb = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(kv))
        self.ops = state if ops is None else ops
        flags = ((_lib.ROM_SKEW_CHECK if skew_check else 0) | _SCHED[schedule] | _SOURCE[source] |
                 _STATE_OPERAND[state_operand])
        cfg = RomConfig(kv, ks, float(dt), _OPS[self.ops], code, flags)
        ctx = C.c_void_p()
        lib = _lib.load()
        pd = C.POINTER(C.c_double)
        check(lib.rom_create(C.byref(cfg), A.ctypes.data_as(pd), B.ctypes.data_as(pd),
                             bb.ctypes.data_as(pd), _stream_handle(stream), C.byref(ctx)))
        self._ctx = ctx

    @classmethod
    def _adopt(cls, ctx, kv, ks, dt, state, ops):
        """Wrap a context the library created (it is destroyed with this object)."""
        self = cls.__new__(cls)
        self.kv, self.ks, self.dt, self.state = int(kv), int(ks), float(dt), state
        _, self.torch_dtype = _DT[state]
        self.ops = ops
        self._ctx = ctx
        return self

    def check_finite(self, V, S, stream=None):
        """Raise RomError (ROM_E_NONFINITE) if V or S holds NaN or Inf."""
        M = int(V.shape[0])
        self._chk_state(V, self.kv, M, "V")
        self._chk_state(S, self.ks, M, "S")
        check(_lib.load().rom_check_finite(self._ctx, M, _ptr(V), _ptr(S), _stream_handle(stream)))

    def check(self, stream=None):
        """Synchronise `stream` and raise if an in-kernel wait of the work
        enqueued so far timed out (ROM_E_TIMEOUT; results invalid)."""
        check(_lib.load().rom_check(self._ctx, _stream_handle(stream)))

    @property
    def last_schedule(self):
        """'columns', 'rowsplit' or 'columns8' for the last FP32-state rank-2
        run (None if none)."""
        v = _lib.load().rom_last_schedule(self._ctx)
        return None if v < 0 else tuning.SCHEDULES[v]

    def schedule_times(self, M):
        """The tuning table's per-step times in microseconds for this
        context's shape at M samples: {schedule name: t or None}."""
        us = (C.c_double * _lib.ROM_NSCHEDULES)()
        check(_lib.load().rom_schedule_times(self._ctx, int(M), us))
        return {name: (us[i] if us[i] >= 0 else None) for i, name in enumerate(tuning.SCHEDULES)}

    def run_receivers(self, mu, V, S, nsteps, C, n0=0, want_Y=True, want_stats=True, stream=None):
        """Advance like run_rank2 and return the seismograms at the receiver
        rows C ((R, Kv) tensor of the state dtype): {"Y": (nsteps, R, M)
        float64 or None, "stats": (nsteps, R, 5) float64 or None} with
        stats = mean, population variance, 5th / 50th / 95th percentile
        (nearest rank) over the M samples."""
        M = int(mu.numel())
        if mu.dtype != torch.float64 or not mu.is_cuda or not mu.is_contiguous():
            raise ValueError("mu must be a contiguous float64 CUDA tensor")
        self._chk_state(V, self.kv, M, "V")
        self._chk_state(S, self.ks, M, "S")
        if C.dim() != 2 or C.shape[1] != self.kv or C.dtype != self.torch_dtype or not C.is_cuda \
                or not C.is_contiguous():
            raise ValueError("C must be a contiguous (R, Kv) CUDA tensor of the state dtype")
        R = int(C.shape[0])
        dev = mu.device
        Y = torch.empty((int(nsteps), R, M), dtype=torch.float64, device=dev) if want_Y else None
        st = torch.empty((int(nsteps), R, 5), dtype=torch.float64, device=dev) if want_stats else None
        check(_lib.load().rom_run_receivers(self._ctx, M, _ptr(mu), int(n0), int(nsteps), _ptr(V), _ptr(S), R,
                                            _ptr(C), _ptr(Y), _ptr(st), _stream_handle(stream)))
        return {"Y": Y, "stats": st}

    def operators(self):
        """(Avs, Asv, scale) exactly as the products use them (float64 numpy)."""
        A = np.zeros((self.kv, self.ks), order="F")
        B = np.zeros((self.ks, self.kv), order="F")
        sc = C.c_double(0.0)
        pd = C.POINTER(C.c_double)
        check(_lib.load().rom_get_operators(self._ctx, A.ctypes.data_as(pd), B.ctypes.data_as(pd), C.byref(sc)))
        return A, B, sc.value

    @property
    def handle(self):
        return self._ctx

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            _lib.load().rom_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state helpers -------------------------------------------------
    def zeros(self, M, device="cuda"):
        """Zero (V, S) of shapes (M, Kv), (M, Ks) in the state dtype."""
        V = torch.zeros((M, self.kv), dtype=self.torch_dtype, device=device)
        S = torch.zeros((M, self.ks), dtype=self.torch_dtype, device=device)
        return V, S

    def _chk_state(self, X, K, M, name):
        if X.dtype != self.torch_dtype or not X.is_cuda or not X.is_contiguous() or tuple(X.shape) != (M, K):
            raise ValueError("%s must be a contiguous CUDA tensor of shape (%d, %d) and dtype %s"
                             % (name, M, K, self.torch_dtype))

    # ---- entry points --------------------------------------------------
    def step_rank1(self, v, s, n, mu, stream=None):
        """One rank-1 step of one sample (v: (Kv,), s: (Ks,) device tensors)."""
        self._chk_state(v.view(1, -1), self.kv, 1, "v")
        self._chk_state(s.view(1, -1), self.ks, 1, "s")
        check(_lib.load().rom_step_rank1(self._ctx, _ptr(v), _ptr(s), int(n), float(mu),
                                         _stream_handle(stream)))

    def run_rank1(self, v, s, mu, nsteps, n0=0, stream=None):
        self._chk_state(v.view(1, -1), self.kv, 1, "v")
        self._chk_state(s.view(1, -1), self.ks, 1, "s")
        check(_lib.load().rom_run_rank1(self._ctx, _ptr(v), _ptr(s), float(mu), int(n0), int(nsteps),
                                        _stream_handle(stream)))

    def run_rank1_batch(self, mu, V, S, nsteps, n0=0, stream=None):
        """The rank-1 formulation for all M samples in one launch (one
        workgroup per sample, the operator re-read every half-step)."""
        M = int(mu.numel())
        if mu.dtype != torch.float64 or not mu.is_cuda or not mu.is_contiguous():
            raise ValueError("mu must be a contiguous float64 CUDA tensor")
        self._chk_state(V, self.kv, M, "V")
        self._chk_state(S, self.ks, M, "S")
        check(_lib.load().rom_run_rank1_batch(self._ctx, M, _ptr(mu), int(n0), int(nsteps), _ptr(V), _ptr(S),
                                              _stream_handle(stream)))

    def run_rank2(self, mu, V, S, nsteps, n0=0, c=None, J=None, y=None, stream=None):
        """Advance all samples ``nsteps`` steps in place.

        mu: (M,) float64 CUDA tensor; V: (M, Kv), S: (M, Ks) state tensors;
        c: (Kv,) state-dtype probe or None; J: (M,) float64 (accumulated);
        y: (nsteps, M) float64 probe trace.
        """
        M = int(mu.numel())
        if mu.dtype != torch.float64 or not mu.is_cuda or not mu.is_contiguous():
            raise ValueError("mu must be a contiguous float64 CUDA tensor")
        self._chk_state(V, self.kv, M, "V")
        self._chk_state(S, self.ks, M, "S")
        if c is not None:
            self._chk_state(c.view(1, -1), self.kv, 1, "c")
        if J is not None and (J.dtype != torch.float64 or J.numel() != M or not J.is_contiguous()):
            raise ValueError("J must be a contiguous float64 tensor of M entries")
        if y is not None and (y.dtype != torch.float64 or tuple(y.shape) != (int(nsteps), M) or not y.is_contiguous()):
            raise ValueError("y must be a contiguous float64 tensor of shape (nsteps, M)")
        check(_lib.load().rom_run_rank2(self._ctx, M, _ptr(mu), int(n0), int(nsteps), _ptr(V), _ptr(S),
                                        _ptr(c), _ptr(J), _ptr(y), _stream_handle(stream)))

    def run_rank2_noalloc(self, mu, V, S, nsteps, n0=0, c=None, J=None, y=None, stream=None):
        """run_rank2 on the row-split schedule without any device allocation
        (the library's static per-GPU scratch; calls overlapping on one GPU
        race).  Raises ROM_E_UNSUPPORTED where the row-split schedule does
        not apply."""
        M = int(mu.numel())
        if mu.dtype != torch.float64 or not mu.is_cuda or not mu.is_contiguous():
            raise ValueError("mu must be a contiguous float64 CUDA tensor")
        self._chk_state(V, self.kv, M, "V")
        self._chk_state(S, self.ks, M, "S")
        if c is not None:
            self._chk_state(c.view(1, -1), self.kv, 1, "c")
        if J is not None and (J.dtype != torch.float64 or J.numel() != M or not J.is_contiguous()):
            raise ValueError("J must be a contiguous float64 tensor of M entries")
        if y is not None and (y.dtype != torch.float64 or tuple(y.shape) != (int(nsteps), M) or not y.is_contiguous()):
            raise ValueError("y must be a contiguous float64 tensor of shape (nsteps, M)")
        check(_lib.load().rom_run_rank2_noalloc(self._ctx, M, _ptr(mu), int(n0), int(nsteps), _ptr(V), _ptr(S),
                                                _ptr(c), _ptr(J), _ptr(y), _stream_handle(stream)))

    def energy(self, V, S, stream=None):
        """Per-sample modified energy |v|^2 + |s|^2 + dt v^T Avs s (float64 tensor)."""
        M = int(V.shape[0])
        self._chk_state(V, self.kv, M, "V")
        self._chk_state(S, self.ks, M, "S")
        E = torch.zeros(M, dtype=torch.float64, device=V.device)
        check(_lib.load().rom_energy(self._ctx, M, _ptr(V), _ptr(S), _ptr(E), _stream_handle(stream)))
        return E

    def adjoint(self, mu, nsteps, c, V0=None, S0=None, stride=0, grads=("dAvs", "dAsv", "dmu"),
                stream=None):
        """Probe QoI J_m = sum_n dt (c^T V_m^(n+1))^2 and its gradients.
        ``stride``: checkpoint stride (0: ceil(sqrt(nsteps))), or -1 for no
        checkpoints (states rebuilt by stepping the leapfrog backwards).

        Returns a dict with J (M,) float64 and the requested gradients of
        J = sum_m J_m: dAvs (Kv, Ks) and dAsv (Ks, Kv) as float32 tensors
        (row-major views of the column-major results), dmu (M,) float64.
        """
        M = int(mu.numel())
        dev = mu.device
        if mu.dtype != torch.float64 or not mu.is_cuda or not mu.is_contiguous():
            raise ValueError("mu must be a contiguous float64 CUDA tensor")
        self._chk_state(c.view(1, -1), self.kv, 1, "c")
        if V0 is not None:
            self._chk_state(V0, self.kv, M, "V0")
        if S0 is not None:
            self._chk_state(S0, self.ks, M, "S0")
        J = torch.zeros(M, dtype=torch.float64, device=dev)
        # column-major Kv x Ks == row-major (Ks, Kv)
        dAvs = torch.zeros((self.ks, self.kv), dtype=torch.float32, device=dev) if "dAvs" in grads else None
        dAsv = torch.zeros((self.kv, self.ks), dtype=torch.float32, device=dev) if "dAsv" in grads else None
        dmu = torch.zeros(M, dtype=torch.float64, device=dev) if "dmu" in grads else None
        check(_lib.load().rom_adjoint(self._ctx, M, _ptr(mu), int(nsteps), _ptr(c), _ptr(V0), _ptr(S0),
                                      _ptr(J), _ptr(dAvs), _ptr(dAsv), _ptr(dmu), int(stride),
                                      _stream_handle(stream)))
        out = {"J": J}
        if dAvs is not None:
            out["dAvs"] = dAvs.t()
        if dAsv is not None:
            out["dAsv"] = dAsv.t()
        if dmu is not None:
            out["dmu"] = dmu
        return out


class RomQoI(torch.autograd.Function):
    """J = sum_m sum_n dt (c^T V_m^(n+1))^2 of an FP32 rank-2 run from zero state.

    forward(Avs, Asv, mu, b, c, dt, nsteps) -> scalar J (float64).
    Gradients flow to Avs (Kv x Ks), Asv (Ks x Kv) and mu (M,) through the
    library's discrete adjoint (rom_adjoint); b, c and dt are constants.
    The operators may live on any device; a library context is built from
    their current values on every forward call.
    """

    @staticmethod
    def forward(ctx, Avs, Asv, mu, b, c, dt, nsteps):
        A = Avs.detach().to("cpu", torch.float64).numpy()
        B = Asv.detach().to("cpu", torch.float64).numpy()
        bb = torch.as_tensor(b).detach().to("cpu", torch.float64).numpy()
        rom = Rom(A, B, bb, float(dt), state="f32")
        dev = mu.device if mu.is_cuda else torch.device("cuda")
        mu_d = mu.detach().to(dev, torch.float64).contiguous()
        c_d = torch.as_tensor(c).detach().to(dev, torch.float32).contiguous()
        try:
            if any(ctx.needs_input_grad[:3]):
                # the adjoint's forward sweep gives J; the gradients are kept
                # for backward
                out = rom.adjoint(mu_d, int(nsteps), c_d)
            else:
                # no gradient wanted: the forward run alone
                M = int(mu_d.numel())
                V, S = rom.zeros(M, device=dev)
                J = torch.zeros(M, dtype=torch.float64, device=dev)
                rom.run_rank2(mu_d, V, S, int(nsteps), c=c_d, J=J)
                out = {"J": J}
            # a row-split group barrier that timed out invalidates J and the
            # gradients: raise instead of returning them
            rom.check()
        finally:
            rom.close()
        ctx.save_for_backward(Avs, Asv, mu)
        ctx.grads = out
        return out["J"].sum().to(mu.device)

    @staticmethod
    def backward(ctx, gJ):
        Avs, Asv, mu = ctx.saved_tensors
        g = ctx.grads
        gA = (gJ.to(g["dAvs"].device, torch.float64) * g["dAvs"].to(torch.float64)).to(Avs.device, Avs.dtype)
        gB = (gJ.to(g["dAsv"].device, torch.float64) * g["dAsv"].to(torch.float64)).to(Asv.device, Asv.dtype)
        gm = (gJ.to(g["dmu"].device, torch.float64) * g["dmu"]).to(mu.device, mu.dtype)
        return gA, gB, gm, None, None, None, None


def _ptr_array(ptrs):
    arr = (C.c_void_p * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr


def _group_args(roms, mus, Vs, Ss):
    G = len(roms)
    if not (len(mus) == len(Vs) == len(Ss) == G) or G < 1:
        raise ValueError("roms, mus, Vs, Ss must have the same nonzero length")
    for r, mu, V, S in zip(roms, mus, Vs, Ss):
        M = int(mu.numel())
        if mu.dtype != torch.float64 or not mu.is_cuda or not mu.is_contiguous():
            raise ValueError("mu must be a contiguous float64 CUDA tensor")
        r._chk_state(V, r.kv, M, "V")
        r._chk_state(S, r.ks, M, "S")
    ctxs = _ptr_array([r.handle.value for r in roms])
    Ms = (C.c_int32 * G)(*[int(mu.numel()) for mu in mus])
    return (ctxs, G, Ms, _ptr_array([mu.data_ptr() for mu in mus]),
            _ptr_array([V.data_ptr() for V in Vs]), _ptr_array([S.data_ptr() for S in Ss]))


def run_grouped(roms, mus, Vs, Ss, nsteps, stream=None):
    """Advance G instances (list of Rom, FP32) ``nsteps`` steps from 0 together
    (one column-block launch, or the row-split plan's launches; see
    GroupPlan).  Synchronises the stream."""
    ctxs, G, Ms, mup, Vp, Sp = _group_args(roms, mus, Vs, Ss)
    check(_lib.load().rom_run_grouped(ctxs, G, Ms, mup, int(nsteps), Vp, Sp, _stream_handle(stream)))


class GroupPlan:
    """Uploaded descriptor table of a grouped run.  ``run`` enqueues the
    plan's launches (column blocks: one launch, which may be captured in a
    HIP graph; with a row-split part: its cooperative launches, groups of
    different K side by side, then one column-block launch over the other
    instances; a captured run takes the all-column form).  ``schedule`` is
    "rowsplit" (a plan with a row-split part) or "columns"; ``split_k`` the
    smallest padded K on the row-split part (0: none); ``times`` the timed
    per-step microseconds of the column-block plan and of the fastest plan
    with a row-split part, if this plan timed them.  Keeps references to its
    tensors."""

    def __init__(self, roms, mus, Vs, Ss):
        ctxs, G, Ms, mup, Vp, Sp = _group_args(roms, mus, Vs, Ss)
        self._keep = (list(roms), list(mus), list(Vs), list(Ss))
        h = C.c_void_p()
        check(_lib.load().rom_group_create(ctxs, G, Ms, mup, Vp, Sp, C.byref(h)))
        self._h = h

    def run(self, nsteps, n0=0, stream=None):
        check(_lib.load().rom_group_run(self._h, int(n0), int(nsteps), _stream_handle(stream)))

    @property
    def schedule(self):
        sc = _lib.load().rom_group_schedule(self._h)
        return "rowsplit" if sc == _lib.ROM_SCHEDULE_ROWSPLIT else "columns"

    @property
    def split_k(self):
        return int(_lib.load().rom_group_split_k(self._h))

    @property
    def times(self):
        us = (C.c_double * 2)()
        check(_lib.load().rom_group_times(self._h, us))
        return {"columns": us[0] if us[0] >= 0 else None, "rowsplit": us[1] if us[1] >= 0 else None}

    def check(self, stream=None):
        check(_lib.load().rom_group_check(self._h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().rom_group_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AffineFamily:
    """Operators that depend affinely on parameters, Avs(theta) = sum_q
    theta_q Avs_q and Asv(theta) likewise, kept as their Q terms on the
    device.  ``instance(theta)`` returns a Rom whose operators are assembled
    on the device (the rank-3 direction: run many instances together with
    run_grouped)."""

    def __init__(self, Avs_terms, Asv_terms, b, dt, state="f32", ops=None, skew_check=False, schedule="auto",
                 stream=None, source="ricker", state_operand="pair"):
        At = np.asarray(Avs_terms, dtype=np.float64)
        Bt = np.asarray(Asv_terms, dtype=np.float64)
        Q, kv, ks = At.shape
        if Bt.shape != (Q, ks, kv):
            raise ValueError("Asv_terms must have shape (Q, Ks, Kv)")
        # Q consecutive column-major matrices
        Ac = np.ascontiguousarray(np.transpose(At, (0, 2, 1)))
        Bc = np.ascontiguousarray(np.transpose(Bt, (0, 2, 1)))
        bb = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(kv))
        self.Q, self.kv, self.ks, self.dt, self.state = int(Q), int(kv), int(ks), float(dt), state
        code, _ = _DT[state]
        self.ops = state if ops is None else ops
        flags = ((_lib.ROM_SKEW_CHECK if skew_check else 0) | _SCHED[schedule] | _SOURCE[source] |
                 _STATE_OPERAND[state_operand])
        cfg = RomConfig(kv, ks, float(dt), _OPS[self.ops], code, flags)
        h = C.c_void_p()
        pd = C.POINTER(C.c_double)
        check(_lib.load().rom_affine_create(C.byref(cfg), int(Q), Ac.ctypes.data_as(pd), Bc.ctypes.data_as(pd),
                                            bb.ctypes.data_as(pd), _stream_handle(stream), C.byref(h)))
        self._h = h

    def instance(self, theta, dt=0.0, stream=None):
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(self.Q))
        ctx = C.c_void_p()
        check(_lib.load().rom_affine_instance(self._h, th.ctypes.data_as(C.POINTER(C.c_double)), float(dt),
                                              _stream_handle(stream), C.byref(ctx)))
        return Rom._adopt(ctx, self.kv, self.ks, dt if dt > 0 else self.dt, self.state, self.ops)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().rom_affine_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _f64_dev(X, name, shape=None):
    if not isinstance(X, torch.Tensor) or X.dtype != torch.float64 or not X.is_cuda or not X.is_contiguous():
        raise ValueError("%s must be a contiguous float64 CUDA tensor" % name)
    if shape is not None and tuple(X.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(X.shape)))
    return X


class Fom:
    """Full-order model of the staggered system on the device (sparse Av,
    As in CSR, source f, time step dt).  States are row-major torch tensors
    (N x M, float64): ``zeros(M)`` makes a pair."""

    def __init__(self, Av, As, f, dt, stream=None, source="ricker"):
        avp, avc, avv = (np.ascontiguousarray(Av[0], dtype=np.int32), np.ascontiguousarray(Av[1], dtype=np.int32),
                         np.ascontiguousarray(Av[2], dtype=np.float64))
        asp, asc, asv = (np.ascontiguousarray(As[0], dtype=np.int32), np.ascontiguousarray(As[1], dtype=np.int32),
                         np.ascontiguousarray(As[2], dtype=np.float64))
        self.nv, self.ns = avp.size - 1, asp.size - 1
        ff = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(self.nv))
        self.dt = float(dt)
        pi = C.POINTER(C.c_int32)
        pd = C.POINTER(C.c_double)
        h = C.c_void_p()
        check(_lib.load().rom_fom_create(self.nv, self.ns, avp.ctypes.data_as(pi), avc.ctypes.data_as(pi),
                                         avv.ctypes.data_as(pd), asp.ctypes.data_as(pi), asc.ctypes.data_as(pi),
                                         asv.ctypes.data_as(pd), ff.ctypes.data_as(pd), self.dt, _SOURCE[source],
                                         _stream_handle(stream), C.byref(h)))
        self._h = h

    def zeros(self, M, device="cuda"):
        return (torch.zeros((self.nv, M), dtype=torch.float64, device=device),
                torch.zeros((self.ns, M), dtype=torch.float64, device=device))

    def run(self, mu, V, S, nsteps, n0=0, stream=None):
        M = int(mu.numel())
        _f64_dev(mu, "mu")
        _f64_dev(V, "V", (self.nv, M))
        _f64_dev(S, "S", (self.ns, M))
        check(_lib.load().rom_fom_run(self._h, M, _ptr(mu), int(n0), int(nsteps), _ptr(V), _ptr(S),
                                      _stream_handle(stream)))

    def project(self, phi_v, phi_s, stream=None):
        """ROM operators of the row-major bases phi_v (Nv x Kv) and phi_s
        (Ns x Ks): returns (Avs (Kv x Ks), Asv (Ks x Kv), b (Kv)) as float64
        CUDA tensors (the operators column-major, i.e. transposed views)."""
        _f64_dev(phi_v, "phi_v")
        _f64_dev(phi_s, "phi_s")
        if phi_v.shape[0] != self.nv or phi_s.shape[0] != self.ns:
            raise ValueError("bases must have Nv and Ns rows")
        kv, ks = int(phi_v.shape[1]), int(phi_s.shape[1])
        Avs = torch.empty((ks, kv), dtype=torch.float64, device=phi_v.device)
        Asv = torch.empty((kv, ks), dtype=torch.float64, device=phi_v.device)
        b = torch.empty(kv, dtype=torch.float64, device=phi_v.device)
        check(_lib.load().rom_fom_project(self._h, kv, ks, _ptr(phi_v), _ptr(phi_s), _ptr(Avs), _ptr(Asv), _ptr(b),
                                          _stream_handle(stream)))
        return Avs.t(), Asv.t(), b

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().rom_fom_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pod(X, tol=None, kmax=None, stream=None):
    """POD modes of the row-major snapshot matrix X (n x ns float64 CUDA):
    returns (Phi (n x k) float64 CUDA, sigma (ns,) numpy, k).  With tol the
    energy criterion picks k (capped at kmax); without, k = kmax (default
    ns)."""
    _f64_dev(X, "X")
    n, ns = int(X.shape[0]), int(X.shape[1])
    kmax = ns if kmax is None else int(kmax)
    phi = torch.empty((n, kmax), dtype=torch.float64, device=X.device)
    sigma = np.zeros(ns)
    k = C.c_int32(0)
    check(_lib.load().rom_pod(n, ns, _ptr(X), -1.0 if tol is None else float(tol), kmax, _ptr(phi),
                              sigma.ctypes.data_as(C.POINTER(C.c_double)), C.byref(k), _stream_handle(stream)))
    kk = int(k.value)
    return (phi if kk == kmax else phi[:, :kk].contiguous()), sigma, kk
