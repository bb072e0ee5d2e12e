"""The differentiation workload at its full horizon: K = 512, 5000 steps.

The GPU adjoint (FP32 states and operators, checkpointed and time-reversal
variants) is compared on a subset of sample columns with

* the FP64 oracle adjoint on the same columns and the same FP32-rounded
  inputs: J, dJ/dAvs, dJ/dAsv and dJ/dmu, norm-wise relative error <= 1e-4;
* central finite differences (h = 1e-6) of the FP64 oracle's forward QoI at
  the same size: dJ/dmu by perturbing every mu_m at once (J_m depends on
  mu_m only, so one pair of runs gives all partials), dJ/dAvs along two
  random unit directions and dJ/dAsv along one (the other operator held
  fixed, reading of the gradient as a partial derivative), <= 1e-4 relative.

Columns are independent (Sec. 2.4: the rank-2 columns are separate forcing
samples), so the operator gradients of a column subset are the gradients of
that subset's QoI; the full 256-column run is covered by the additivity
test of test_gpu_adjoint.py.  The oracle work (one adjoint and seven forward
runs of 4 columns x 5000 steps at K = 512) runs concurrently on the host.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
TOL = 1e-4
K, N = 512, 5000
COLS = np.array([0, 37, 128, 255])
H = 1e-6


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def horizon():
    inst = synth.round_to(synth.make_instance(K, K, 256, seed=0), "f32")
    mu = inst["mu"][COLS]
    rng = np.random.default_rng(11)
    dirs = {}
    for name, count in (("Avs", 2), ("Asv", 1)):
        for i in range(count):
            D = rng.standard_normal(inst[name].shape)
            dirs["%s%d" % (name, i)] = (name, D / np.linalg.norm(D))

    def J_of(Avs, Asv, mus):
        return oracle.run_rank2(Avs, Asv, inst["b"], inst["dt"], mus, N, c=inst["c"])["J"]

    jobs = {"adjoint": lambda: oracle.adjoint(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], mu, N, inst["c"]),
            # mu + h and mu - h as 2 x 4 columns of one run (same operators)
            "mu": lambda: J_of(inst["Avs"], inst["Asv"], np.concatenate([mu + H, mu - H]))}
    for key, (name, D) in dirs.items():
        for sgn in (1, -1):
            def job(name=name, D=D, sgn=sgn):
                ops = {"Avs": inst["Avs"], "Asv": inst["Asv"]}
                ops[name] = ops[name] + sgn * H * D
                return float(np.sum(J_of(ops["Avs"], ops["Asv"], mu)))
            jobs[(key, sgn)] = job
    with cf.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        futs = {k: ex.submit(f) for k, f in jobs.items()}
        res = {k: f.result() for k, f in futs.items()}
    fd = {"mu": (res["mu"][:len(COLS)] - res["mu"][len(COLS):]) / (2 * H)}
    for key, (name, D) in dirs.items():
        fd[key] = (name, D, (res[(key, 1)] - res[(key, -1)]) / (2 * H))
    return inst, res["adjoint"], fd


def _gpu(inst, stride):
    from paper_2009_11742_amd import Rom
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"][COLS], dtype=torch.float64, device="cuda")
    c = torch.tensor(inst["c"], dtype=torch.float32, device="cuda")
    out = rom.adjoint(mu, N, c, stride=stride)
    rom.check()
    res = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    rom.close()
    return res


@pytest.mark.parametrize("stride", [0, -1])
def test_adjoint_full_horizon_vs_oracle_and_fd(horizon, stride):
    inst, ref, fd = horizon
    g = _gpu(inst, stride)
    errs = {k: _rel(g[k], ref[k]) for k in ("J", "dAvs", "dAsv", "dmu")}
    errs["dmu_fd"] = _rel(g["dmu"], fd["mu"])
    for key, val in fd.items():
        if key == "mu":
            continue
        name, D, d = val
        an = float(np.sum(g["d" + name] * D))
        errs[key + "_fd"] = abs(an - d) / abs(d)
    # the oracle's own adjoint against its finite differences (both FP64)
    errs["oracle_dmu_fd"] = _rel(ref["dmu"], fd["mu"])
    for key, val in fd.items():
        if key != "mu":
            name, D, d = val
            errs["oracle_" + key + "_fd"] = abs(float(np.sum(ref["d" + name] * D)) - d) / abs(d)
    print("adjoint K=%d N=%d cols=%s stride=%d:" % (K, N, list(COLS), stride),
          {k: "%.2e" % v for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL, (k, v)
