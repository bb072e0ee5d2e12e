"""Full-order model and offline stage on the GPU: rank-2 FOM stepping over
CSR operators (row-major states), the Galerkin projection of bases onto
ROM operators, and POD by Cholesky QR + Jacobi SVD, each against the FP64
oracle; then the whole chain (FOM snapshots -> POD -> projection -> ROM run)
against the FOM it reduces.

FP64 throughout; bars: 1e-12 (stepping, projection: sums of a few terms per
entry), 1e-10 (singular values above 1e-5 of the largest: an SVD's
u sigma_1 / sigma_i), modes by their subspace angles.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _rel(X, R):
    return float(np.linalg.norm(X - R) / np.linalg.norm(R))


def _relcol(X, R):
    return float(np.max(np.linalg.norm(X - R, axis=0) / np.linalg.norm(R, axis=0)))


def _fom(d):
    from paper_2009_11742_amd import Fom
    return Fom(d["Av"], d["As"], d["f"], d["dt"])


@pytest.mark.parametrize("nr,nth,M,N", [(12, 20, 5, 600), (9, 33, 1, 400), (20, 16, 17, 300)])
def test_fom_run_matches_oracle(nr, nth, M, N):
    d = synth.make_shear_fom(nr, nth)
    mu = synth.fom_periods(M, seed=nr)
    F = _fom(d)
    mut = torch.tensor(mu, dtype=torch.float64, device="cuda")
    V, S = F.zeros(M)
    F.run(mut, V, S, N)
    torch.cuda.synchronize()
    r = oracle.fom_run(d["Av"], d["As"], d["f"], d["dt"], mu, N)
    ev, es = _relcol(V.cpu().numpy(), r["V"]), _relcol(S.cpu().numpy(), r["S"])
    print("FOM %dx%d M=%d N=%d: V %.2e S %.2e" % (nr, nth, M, N, ev, es))
    assert ev <= 1e-12 and es <= 1e-12
    # a run split in two equals one run; one sample alone equals its column
    V2, S2 = F.zeros(M)
    F.run(mut, V2, S2, N // 3)
    F.run(mut, V2, S2, N - N // 3, n0=N // 3)
    V1, S1 = F.zeros(1)
    F.run(mut[M - 1:], V1, S1, N)
    torch.cuda.synchronize()
    assert torch.equal(V2, V) and torch.equal(S2, S)
    assert torch.equal(V1[:, 0], V[:, M - 1]) and torch.equal(S1[:, 0], S[:, M - 1])
    F.close()


def test_fom_paper_grid_sampled():
    """The 256 x 1024 velocity grid (785,152 DOF), 16 samples, 150 steps at
    the paper's dt = 0.05 s; two sampled columns against the oracle."""
    d = synth.make_shear_fom(256, 1024, dt=0.05)
    M, N = 16, 150
    mu = synth.fom_periods(M, seed=1)
    # start from a nonzero state so that 150 steps move every DOF
    rng = np.random.default_rng(0)
    V0 = rng.standard_normal((d["nv"], M)) * 1e-3
    S0 = rng.standard_normal((d["ns"], M)) * 1e4
    F = _fom(d)
    mut = torch.tensor(mu, dtype=torch.float64, device="cuda")
    V = torch.tensor(V0, device="cuda")
    S = torch.tensor(S0, device="cuda")
    F.run(mut, V, S, N)
    torch.cuda.synchronize()
    for m in (0, 11):
        r = oracle.fom_run(d["Av"], d["As"], d["f"], d["dt"], mu[m:m + 1], N, V=V0[:, m:m + 1], S=S0[:, m:m + 1])
        ev = _rel(V[:, m].cpu().numpy(), r["V"][:, 0])
        es = _rel(S[:, m].cpu().numpy(), r["S"][:, 0])
        print("FOM 256x1024 column %d: V %.2e S %.2e" % (m, ev, es))
        assert ev <= 1e-12 and es <= 1e-12
    F.close()


@pytest.mark.parametrize("nr,nth,kv,ks", [(12, 20, 30, 41), (40, 70, 100, 65), (8, 9, 72, 1)])
def test_projection_matches_oracle(nr, nth, kv, ks):
    d = synth.make_shear_fom(nr, nth)
    rng = np.random.default_rng(kv)
    Pv, _ = np.linalg.qr(rng.standard_normal((d["nv"], kv)))
    Ps, _ = np.linalg.qr(rng.standard_normal((d["ns"], ks)))
    F = _fom(d)
    Avs, Asv, b = F.project(torch.tensor(Pv, device="cuda"), torch.tensor(Ps, device="cuda"))
    torch.cuda.synchronize()
    Ar, Br, br = oracle.project(d["Av"], d["As"], d["f"], Pv, Ps)
    e = (_rel(Avs.cpu().numpy(), Ar), _rel(Asv.cpu().numpy(), Br), _rel(b.cpu().numpy(), br))
    print("projection %dx%d Kv=%d Ks=%d: %s" % (nr, nth, kv, ks, ["%.2e" % x for x in e]))
    assert max(e) <= 1e-12
    F.close()


@pytest.mark.parametrize("n,ns,decay", [(5000, 60, 0.5), (700, 64, 0.25), (4096, 256, 0.05)])
def test_pod_matches_oracle(n, ns, decay):
    from paper_2009_11742_amd import pod
    rng = np.random.default_rng(ns)
    U, _ = np.linalg.qr(rng.standard_normal((n, ns)))
    W, _ = np.linalg.qr(rng.standard_normal((ns, ns)))
    s = 10.0 ** (-decay * np.arange(ns))
    X = (U * s) @ W.T
    Phi, sig, k = pod(torch.tensor(X, device="cuda"), tol=3e-8)
    Pr, sr, kr = oracle.pod(X, tol=3e-8)
    assert k == kr
    big = sr > 1e-5 * sr[0]          # well above the rank threshold (~2e-6 sigma_1 at ns = 256)
    es = float(np.max(np.abs(sig[big] - sr[big]) / sr[big]))
    P = Phi.cpu().numpy()
    orth = float(np.max(np.abs(P.T @ P - np.eye(k))))
    # subspace agreement: cosines of the principal angles between the spans
    cos = np.linalg.svd(P.T @ Pr, compute_uv=False)
    print("POD n=%d ns=%d: k=%d sigma %.2e orth %.2e min cos %.12f" % (n, ns, k, es, orth, cos.min()))
    assert es <= 1e-10 and orth <= 1e-12 and cos.min() >= 1.0 - 1e-10


def test_pod_keeps_kmax_without_tolerance():
    from paper_2009_11742_amd import pod
    rng = np.random.default_rng(3)
    X = rng.standard_normal((900, 40))
    Phi, sig, k = pod(torch.tensor(X, device="cuda"), kmax=12)
    assert k == 12 and tuple(Phi.shape) == (900, 12)
    sr = np.linalg.svd(X, compute_uv=False)
    assert np.max(np.abs(sig - sr) / sr) <= 1e-12


def test_offline_online_chain_reproduces_the_fom():
    """FOM snapshots of 4 training periods (every 3rd of 600 steps) -> POD
    bases (energy 1e-9) -> Galerkin operators -> FP64 ROM runs: the
    reconstructed velocity field matches the FOM's for the training periods
    and for 3 new ones (the reproductive and predictive scenarios of
    Sec. 4.4), and the GPU chain matches the oracle's chain on the same
    snapshots (POD ranks, operators, reconstructed fields)."""
    from paper_2009_11742_amd import Fom, Rom, pod
    d = synth.make_shear_fom(24, 48)
    F = Fom(d["Av"], d["As"], d["f"], d["dt"])
    train = synth.fom_periods(4, seed=10)
    N, every = 600, 3
    mut = torch.tensor(train, dtype=torch.float64, device="cuda")
    V, S = F.zeros(4)
    XV, XS = [], []
    for c in range(N // every):
        F.run(mut, V, S, every, n0=c * every)
        XV.append(V.clone()); XS.append(S.clone())
    XV = torch.cat(XV, dim=1).contiguous()       # Nv x (60 snapshots x 4 samples)
    XS = torch.cat(XS, dim=1).contiguous()
    Pv, sv, kv = pod(XV, tol=1e-9)
    Ps, ss, ks = pod(XS, tol=1e-9)
    Avs, Asv, b = F.project(Pv, Ps)
    torch.cuda.synchronize()
    # oracle chain on the same snapshots
    Pvr, svr, kvr = oracle.pod(XV.cpu().numpy(), tol=1e-9)
    Psr, ssr, ksr = oracle.pod(XS.cpu().numpy(), tol=1e-9)
    assert (kv, ks) == (kvr, ksr)
    Ar, Br, br = oracle.project(d["Av"], d["As"], d["f"], Pv.cpu().numpy(), Ps.cpu().numpy())
    assert _rel(Avs.cpu().numpy(), Ar) <= 1e-12 and _rel(b.cpu().numpy(), br) <= 1e-12
    # online: the training periods (reproductive) and 3 new ones
    # (predictive), FP64 ROM on the GPU vs FOM on the GPU
    rom = Rom(Avs.cpu().numpy(), Asv.cpu().numpy(), b.cpu().numpy(), d["dt"], state="f64")
    errs, chain = [], []
    Ar2, Br2, br2 = oracle.project(d["Av"], d["As"], d["f"], Pvr, Psr)
    for mus in (train, synth.fom_periods(3, seed=11)):
        mu_t = torch.tensor(mus, dtype=torch.float64, device="cuda")
        Vr, Sr = rom.zeros(len(mus))
        rom.run_rank2(mu_t, Vr, Sr, N)
        Vf, Sf = F.zeros(len(mus))
        F.run(mu_t, Vf, Sf, N)
        torch.cuda.synchronize()
        recon = Pv.cpu().numpy() @ Vr.cpu().numpy().T      # ROM states: (M, Kv) = Kv x M column-major
        errs.append(_relcol(recon, Vf.cpu().numpy()))
        ro = oracle.run_rank2(Ar2, Br2, br2, d["dt"], mus, N)
        chain.append(_relcol(recon, Pvr @ ro["V"]))
    print("chain: kv=%d ks=%d, ROM vs FOM velocity error: reproductive %.2e, predictive %.2e; "
          "GPU chain vs oracle chain %.2e %.2e" % (kv, ks, errs[0], errs[1], chain[0], chain[1]))
    assert errs[0] <= 1e-3 and errs[1] <= 2e-3
    assert max(chain) <= 1e-6
    rom.close()
    F.close()


def test_fom_wide_rows_take_the_csr_kernel():
    """Operators with a row of more than 8 entries keep the CSR kernel (no
    padded copy); a random sparse pair with rows of 0 - 12 entries, stepped
    and projected, against the oracle."""
    from paper_2009_11742_amd import Fom
    rng = np.random.default_rng(9)
    nv, ns = 50, 70

    def rand_csr(nr, nc, scale):
        lens = rng.integers(0, 13, nr)
        lens[3] = 12                        # at least one row wider than 8
        ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
        col = np.concatenate([np.sort(rng.choice(nc, l, replace=False)) for l in lens]).astype(np.int32)
        val = rng.standard_normal(int(ptr[-1])) * scale
        return ptr, col, val
    Av, As = rand_csr(nv, ns, 0.05), rand_csr(ns, nv, 0.05)
    f = np.zeros(nv); f[7] = 1.0
    mu = np.array([0.6, 0.8, 0.95])
    F = Fom(Av, As, f, 0.1)
    V, S = F.zeros(3)
    F.run(torch.tensor(mu, device="cuda"), V, S, 200)
    torch.cuda.synchronize()
    r = oracle.fom_run(Av, As, f, 0.1, mu, 200)
    assert _relcol(V.cpu().numpy(), r["V"]) <= 1e-12 and _relcol(S.cpu().numpy(), r["S"]) <= 1e-12
    Pv, _ = np.linalg.qr(rng.standard_normal((nv, 9)))
    Ps, _ = np.linalg.qr(rng.standard_normal((ns, 11)))
    Avs, Asv, b = F.project(torch.tensor(Pv, device="cuda"), torch.tensor(Ps, device="cuda"))
    Ar, Br, br = oracle.project(Av, As, f, Pv, Ps)
    assert _rel(Avs.cpu().numpy(), Ar) <= 1e-12 and _rel(Asv.cpu().numpy(), Br) <= 1e-12
    F.close()
