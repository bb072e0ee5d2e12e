"""Low-precision operator products (BF16, FP8-E4M3) with FP32 states.

* The operators the GPU products use equal the oracle's BF16 / E4M3
  roundings bitwise (same per-tensor FP8 scale).
* Trajectories are compared with two FP64 oracles: the same-input oracle
  (integrating the rounded operators) and the original-input oracle (the
  unrounded FP32 operators).  The same-input bar follows from the state
  operand: each FP32 state value enters the product as a BF16 hi + lo pair
  (relative error <= 2^-17), i.e. a per-step relative perturbation of about
  dt * 2^-17 * ||A|| ~ 2e-6 that random-walks to ~1.4e-4 after 5000 steps;
  the bar is three times that walk, lowp_bars.pair_bar(N) = 6e-6 sqrt(N).
  The single BF16 operand must land within a factor of two of its numpy
  emulation (lowp_bars).  The original-input error (operator rounding
  itself) is reported, not bounded: it is the physics of the rounded model.
"""
import concurrent.futures as cf
import time

import numpy as np
import pytest

import lowp_bars
import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _relcol(X, R):
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.linalg.norm(R, axis=0)))


def _oracle_ops(inst, ops):
    A, B = inst["Avs"], inst["Asv"]
    if ops == "bf16":
        return oracle.round_bf16(A), oracle.round_bf16(B), 1.0
    amax = max(np.max(np.abs(A.astype(np.float32))), np.max(np.abs(B.astype(np.float32))))
    Aq, s1 = oracle.quantize_e4m3(A, amax=float(amax))
    Bq, s2 = oracle.quantize_e4m3(B, amax=float(amax))
    assert s1 == s2
    return Aq, Bq, s1


@pytest.mark.parametrize("ops", ["bf16", "fp8"])
@pytest.mark.parametrize("kv,ks,skew", [(128, 128, True), (100, 70, False)])
def test_quantized_operators_equal_oracle_rounding(ops, kv, ks, skew):
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(kv, ks, 2, seed=kv + ks, skew=skew), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", ops=ops)
    A, B, sc = rom.operators()
    Ar, Br, scr = _oracle_ops(inst, ops)
    assert np.array_equal(A, Ar) and np.array_equal(B, Br)
    assert sc == scr
    if skew:
        assert np.array_equal(B, -A.T)     # one shared scale keeps the pair skew
    rom.close()


def _run(inst, ops, nsteps, cols=None, operand="pair"):
    from paper_2009_11742_amd import Rom
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", ops=ops, state_operand=operand)
    mu_np = inst["mu"] if cols is None else inst["mu"][cols]
    M = len(mu_np)
    mu = torch.tensor(mu_np, dtype=torch.float64, device="cuda")
    V, S = rom.zeros(M)
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    J = torch.zeros(M, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rom.run_rank2(mu, V, S, nsteps, c=c, J=J)
    torch.cuda.synchronize()
    dt_run = time.perf_counter() - t0
    ops_used = rom.operators()
    rom.close()
    return (V.cpu().numpy().astype(np.float64).T, S.cpu().numpy().astype(np.float64).T, J.cpu().numpy(),
            dt_run, ops_used)


@pytest.mark.parametrize("ops", ["bf16", "fp8"])
@pytest.mark.parametrize("kv,ks,M,N,skew", [(128, 128, 8, 2000, True), (100, 70, 5, 1500, False)])
def test_lowp_same_input_parity(ops, kv, ks, M, N, skew):
    inst = synth.round_to(synth.make_instance(kv, ks, M, seed=3 * kv + ks, skew=skew), "f32")
    V, S, J, _, (A, B, _) = _run(inst, ops, N)
    same = oracle.run_rank2(A, B, inst["b"], inst["dt"], inst["mu"], N, c=inst["c"])
    orig = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N, c=inst["c"])
    e_same = max(_relcol(V, same["V"]), _relcol(S, same["S"]))
    e_orig = max(_relcol(V, orig["V"]), _relcol(S, orig["S"]))
    e_J = float(np.max(np.abs(J - same["J"]) / same["J"]))
    bar = lowp_bars.pair_bar(N)
    print("%s K=(%d,%d) M=%d N=%d: same-input %.2e  original-input %.2e  QoI(same) %.2e  (bar %.2e)"
          % (ops, kv, ks, M, N, e_same, e_orig, e_J, bar))
    assert e_same <= bar and e_J <= bar
    assert np.all(np.isfinite(V)) and np.all(np.isfinite(S))


def test_precision_workload_k1024_m1024():
    """K = M = 1024, 5000 steps: BF16 and FP8 operators with the state
    operand as a BF16 pair or as one BF16 value (and FP32 for reference),
    errors on 3 sampled columns against both oracles."""
    inst = synth.round_to(synth.make_instance(1024, 1024, 1024, seed=0), "f32")
    N = 5000
    cols = np.array([0, 511, 1023])
    results = {}
    modes = (("f32", "pair"), ("bf16", "pair"), ("fp8", "pair"), ("bf16", "single"), ("fp8", "single"))
    for ops, operand in modes:
        key = ops if operand == "pair" else ops + "_single"
        V, S, J, secs, (A, B, sc) = _run(inst, ops, N, operand=operand)
        results[key] = (V[:, cols], S[:, cols], J[cols], secs, A, B)
        print("%s: %.1f ms per run, %.2f us per step, %.1f TFLOP/s algorithmic"
              % (key, secs * 1e3, secs / N * 1e6, 4.0 * 1024 ** 3 * N / secs / 1e12))

    jobs = {"orig": (inst["Avs"], inst["Asv"]), "bf16": results["bf16"][4:6], "fp8": results["fp8"][4:6]}

    def ref(key_col):
        key, ci = key_col
        A, B = jobs[key]
        return key, ci, oracle.run_rank2(A, B, inst["b"], inst["dt"], inst["mu"][cols[ci]:cols[ci] + 1], N,
                                         c=inst["c"])
    def emulate(key):
        A, B = jobs[key]
        return key, lowp_bars.single_operand_emulation(A, B, inst["b"], inst["dt"], inst["mu"][cols], N)
    with cf.ThreadPoolExecutor(max_workers=9) as ex:
        emu_f = [ex.submit(emulate, k) for k in ("bf16", "fp8")]
        outs = list(ex.map(ref, [(k, ci) for k in jobs for ci in range(len(cols))]))
        emus = dict(f.result() for f in emu_f)
    refs = {}
    for key, ci, r in outs:
        refs.setdefault(key, [None] * len(cols))[ci] = r
    for key in results:
        V, S, J = results[key][:3]
        ops = key.split("_")[0]
        same_key = "orig" if ops == "f32" else ops
        e_same = max(max(_relcol(V[:, i:i + 1], refs[same_key][i]["V"]), _relcol(S[:, i:i + 1], refs[same_key][i]["S"]))
                     for i in range(len(cols)))
        e_orig = max(max(_relcol(V[:, i:i + 1], refs["orig"][i]["V"]), _relcol(S[:, i:i + 1], refs["orig"][i]["S"]))
                     for i in range(len(cols)))
        q_same = max(abs(J[i] - refs[same_key][i]["J"][0]) / refs[same_key][i]["J"][0] for i in range(len(cols)))
        q_orig = max(abs(J[i] - refs["orig"][i]["J"][0]) / refs["orig"][i]["J"][0] for i in range(len(cols)))
        print("%s K=M=1024 N=5000: state err same-input %.2e original %.2e | QoI err same-input %.2e original %.2e"
              % (key, e_same, e_orig, q_same, q_orig))
        if key.endswith("_single"):
            Ve, Se = emus[ops]
            e_emu = max(max(_relcol(Ve[:, i:i + 1], refs[ops][i]["V"]), _relcol(Se[:, i:i + 1], refs[ops][i]["S"]))
                        for i in range(len(cols)))
            band = lowp_bars.SINGLE_BAND
            print("%s: emulation %.2e" % (key, e_emu))
            assert e_emu / band <= e_same <= band * e_emu and q_same <= band * e_emu
        else:
            bar = 1e-5 if ops == "f32" else lowp_bars.pair_bar(N)
            assert e_same <= bar and q_same <= bar


@pytest.mark.parametrize("ops", ["bf16", "fp8"])
def test_fp64_state_rounded_operators_stability(ops):
    """Long-horizon reference of the rounded model: FP64 states with the
    BF16 / FP8 operators.  Parity with the oracle on the same operators
    (FP64 bar), exact energy conservation after the source has decayed, and
    the FP32-state low-precision run's energy drift against it."""
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(128, 128, 4, seed=17), "f32")
    r64 = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f64", ops=ops)
    r32 = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", ops=ops)
    A, B, _ = r64.operators()
    A32, B32, _ = r32.operators()
    assert np.array_equal(A, A32) and np.array_equal(B, B32)
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device="cuda")
    V, S = r64.zeros(4)
    r64.run_rank2(mu, V, S, 300)
    torch.cuda.synchronize()
    ref = oracle.run_rank2(A, B, inst["b"], inst["dt"], inst["mu"], 300)
    Vg = V.cpu().numpy().T
    assert _relcol(Vg, ref["V"]) <= 1e-12 and _relcol(S.cpu().numpy().T, ref["S"]) <= 1e-12
    E0 = r64.energy(V, S)
    Eo = oracle.energy(A, inst["dt"], ref["V"], ref["S"])
    assert np.allclose(E0.cpu().numpy(), Eo, rtol=1e-13, atol=0)
    V32, S32 = r32.zeros(4)
    r32.run_rank2(mu, V32, S32, 300)
    r64.run_rank2(mu, V, S, 20000, n0=300)
    r32.run_rank2(mu, V32, S32, 20000, n0=300)
    torch.cuda.synchronize()
    E1 = r64.energy(V, S).cpu().numpy()
    E32 = r32.energy(V32, S32).cpu().numpy()
    drift64 = float(np.max(np.abs(E1 - E0.cpu().numpy()) / E0.cpu().numpy()))
    drift32 = float(np.max(np.abs(E32 - E1) / E1))
    print("%s: FP64-state energy drift over 2e4 steps %.2e; FP32-state vs FP64-state energy %.2e" % (ops, drift64, drift32))
    assert drift64 <= 1e-10
    assert drift32 <= 1e-3
    r64.close(); r32.close()


def test_energy_kernel_matches_oracle():
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(70, 45, 6, seed=3, skew=False), "f32")
    rng = np.random.default_rng(0)
    V0 = rng.standard_normal((70, 6)).astype(np.float32).astype(np.float64)
    S0 = rng.standard_normal((45, 6)).astype(np.float32).astype(np.float64)
    ref = oracle.energy(inst["Avs"], inst["dt"], V0, S0)
    for state, tdt in (("f32", torch.float32), ("f64", torch.float64)):
        rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state=state)
        V = torch.tensor(np.ascontiguousarray(V0.T), dtype=tdt, device="cuda")
        S = torch.tensor(np.ascontiguousarray(S0.T), dtype=tdt, device="cuda")
        E = rom.energy(V, S).cpu().numpy()
        assert np.allclose(E, ref, rtol=1e-13, atol=0)
        rom.close()
