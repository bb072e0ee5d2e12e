"""Rank-1 formulation of many samples in one launch (rom_run_rank1_batch):
one workgroup per sample, the operator re-read every half-step.  Parity
against the FP64 oracle at the FP32 bar (1e-5) with the state rounded once
per half-step, as the single-sample rank-1 step does; and, since it does
each row's arithmetic in the same order as that step, bitwise equality
with rom_run_rank1 on the first and last samples."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
BAR = 1e-5


def _relcol(X, R):
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.linalg.norm(R, axis=0)))


@pytest.mark.parametrize("kv,ks,M,N,skew", [(256, 256, 12, 1500, True), (70, 45, 5, 700, False),
                                            (300, 520, 3, 400, False), (1024, 1024, 2, 200, True)])
def test_rank1_batch_parity(kv, ks, M, N, skew):
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(kv, ks, M, seed=kv + ks + M, skew=skew), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = rom.zeros(M)
    rom.run_rank1_batch(mu, V, S, N // 3)
    rom.run_rank1_batch(mu, V, S, N - N // 3, n0=N // 3)
    torch.cuda.synchronize()
    ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N)
    Vg, Sg = V.cpu().numpy().astype(np.float64).T, S.cpu().numpy().astype(np.float64).T
    ev, es = _relcol(Vg, ref["V"]), _relcol(Sg, ref["S"])
    print("rank-1 batch K=(%d,%d) M=%d N=%d: V %.2e S %.2e" % (kv, ks, M, N, ev, es))
    assert max(ev, es) <= BAR
    # the first and last samples stepped by the single-sample rank-1 entry point
    for m in (0, M - 1):
        v = torch.zeros(kv, dtype=torch.float32, device="cuda")
        s = torch.zeros(ks, dtype=torch.float32, device="cuda")
        rom.run_rank1(v, s, float(inst["mu"][m]), N)
        torch.cuda.synchronize()
        assert torch.equal(v, V[m]) and torch.equal(s, S[m]), m
    rom.close()
