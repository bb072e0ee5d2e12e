"""The adjoint's recompute and reverse sweeps on the row-split kernels.

With a checkpointed forward sweep on the row-split schedule, each segment
is recomputed by the traced row-split kernel and reversed by its adjoint
mode; where two runs of the shape fit one launch, segment g's reverse sweep
and segment g - 1's recompute share a launch (disjoint groups).  Checked
against the FP64 oracle adjoint (bar 1e-4, norm-wise relative, as the
column-block adjoint), against the column-block adjoint of the same inputs
(FP32 against FP32: 1e-5), with the side-by-side launch (K = 256, 512) and
without it (K = 1536, M = 260: 5 groups of 64 run, 10 would not fit the 8
a launch holds), including a ragged last segment and a nonzero start.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
TOL = 1e-4
GPU_TOL = 1e-5


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _adjoint(inst, N, schedule, stride=0, V0=None, S0=None):
    from paper_2009_11742_amd import Rom
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule=schedule)
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    v0 = None if V0 is None else torch.tensor(np.ascontiguousarray(V0.T), dtype=torch.float32, device="cuda")
    s0 = None if S0 is None else torch.tensor(np.ascontiguousarray(S0.T), dtype=torch.float32, device="cuda")
    out = rom.adjoint(mu, N, c, V0=v0, S0=s0, stride=stride)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    rom.close()
    return res


@pytest.mark.parametrize("K,M,N,stride", [(256, 40, 300, 0), (256, 70, 257, 16), (192, 20, 200, 0)])
def test_split_adjoint_matches_oracle(K, M, N, stride):
    inst = synth.round_to(synth.make_instance(K, K, M, seed=K + M), "f32")
    g = _adjoint(inst, N, "rowsplit", stride=stride)
    r = oracle.adjoint(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, inst["c"])
    errs = {k: _rel(g[k], r[k]) for k in ("J", "dAvs", "dAsv", "dmu")}
    print("row-split adjoint", (K, M, N, stride), {k: "%.2e" % v for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL, (k, v)


def test_split_adjoint_nonzero_start():
    inst = synth.round_to(synth.make_instance(256, 256, 24, seed=31), "f32")
    rng = np.random.default_rng(2)
    V0 = (0.1 * rng.standard_normal((256, 24))).astype(np.float32).astype(np.float64)
    S0 = (0.1 * rng.standard_normal((256, 24))).astype(np.float32).astype(np.float64)
    g = _adjoint(inst, 180, "rowsplit", V0=V0, S0=S0)
    r = oracle.adjoint(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], 180, inst["c"], V0=V0, S0=S0)
    for k in ("J", "dAvs", "dAsv", "dmu"):
        assert _rel(g[k], r[k]) <= TOL, k


@pytest.mark.parametrize("K,M,N", [(512, 256, 400), (1536, 260, 12)])
def test_split_adjoint_matches_column_block_adjoint(K, M, N):
    """Side by side (K = 512, M = 256) and one after the other (K = 1536,
    M = 260) against the column-block adjoint of the same inputs."""
    inst = synth.round_to(synth.make_instance(K, K, M, seed=K + 1), "f32")
    g = _adjoint(inst, N, "rowsplit")
    ref = _adjoint(inst, N, "columns")
    errs = {k: _rel(g[k], ref[k]) for k in ("J", "dAvs", "dAsv", "dmu")}
    print("row-split vs column-block adjoint", (K, M, N), {k: "%.2e" % v for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= GPU_TOL, (k, v)
