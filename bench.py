"""Benchmark: rank-2 vs rank-1 Galerkin ROM stepping on one MI355X.

Workload (one bench "step"): integrate M = 256 forcing samples of a synthetic
staggered LTI ROM with Kv = Ks = 256 (random N(0, 1/K) operators, skew coupled,
Ricker sources with mu ~ U[0.5, 1]) over 10^4 leapfrog steps in FP32, i.e.
one full rank-2 run.  Inputs are resident on the GPU before timing starts.

Prints ONE JSON line: sample-steps/s of the rank-2 path (whole job), the
rank-1 path's rate on the same GPU, the roofline of the rank-2 kernel, the
error against the FP64 oracle on sampled columns, and the oracle's own rate
on the host (cpu_baseline); beside them the K = M = 1024 record (FP32, BF16,
FP8 operators) and the plain FP64 record (K = 64, M in {1, 8}, 2000 steps,
with its rank-1 formulation).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

KV = KS = 256
M = 256
NSTEPS = 10000
SEED = 0
FP32_MFMA_PEAK_TFLOPS = 157.3

# Kernel of each FP32 schedule (rom_last_schedule), its sources, and the HBM
# bytes per launch at the bench workload from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) scaled by a plain 256 MiB copy (factors 2.0 and
# 1.0), valid only for the kernel sources they were taken on.
SCHEDULE_KERNELS = {
    "columns": ("rank2_f32_mfma_kernel", ("paper_2009_11742_amd/csrc/k_rank2_f32.hip",
                                          "paper_2009_11742_amd/csrc/k_tile_f32.h",
                                          "paper_2009_11742_amd/csrc/k_common.h")),
    "columns8": ("rank2_f32_mfma_kernel", ("paper_2009_11742_amd/csrc/k_rank2_f32.hip",
                                           "paper_2009_11742_amd/csrc/k_tile_f32.h",
                                           "paper_2009_11742_amd/csrc/k_common.h")),
    "rowsplit": ("rank2_split_f32_kernel", ("paper_2009_11742_amd/csrc/k_rank2_split.hip",
                                            "paper_2009_11742_amd/csrc/k_common.h")),
    "resident": ("rank2_resident_kernel", ("paper_2009_11742_amd/csrc/k_rank2_resident.hip",
                                           "paper_2009_11742_amd/csrc/k_lane.h",
                                           "paper_2009_11742_amd/csrc/k_common.h")),
}
MEASURED_TRAFFIC = {"fc1d167ba1c60b4cffde49fcd47937f7c17e8d02": 5.516e6,    # column blocks
                    "274d5ae594e2161ef42ffb424a65bd9601130973": 3.305e6}    # resident kernel
FP32_VECTOR_PEAK_TFLOPS = 157.3          # with packed FP32; 78.6 without
HBM_PEAK_GBS = 8000.0


def _sources_sha1(files):
    import hashlib
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _measured_traffic(schedule):
    files = SCHEDULE_KERNELS.get(schedule, (None, ()))[1]
    return MEASURED_TRAFFIC.get(_sources_sha1(files)) if files else None


def _err_cols(Xg, Xr):
    return float(np.max(np.linalg.norm(Xg - Xr, axis=0) / np.linalg.norm(Xr, axis=0)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--fom-point", default=None,
                    help="fom workload: one point only, GRIDxM (e.g. 512x2048x48), timed over --steps runs")
    ap.add_argument("--scaling-point", default=None,
                    help="scaling workload: one point only, KxM (e.g. 4096x1024)")
    ap.add_argument("--no-rank1", action="store_true", help="skip the rank-1 comparison")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain FP64 record (K = 64, M in {1, 8}, 2000 steps, with its rank-1 run)")
    ap.add_argument("--no-target", action="store_true",
                    help="skip the K = M = 1024 target record (FP32, BF16, FP8 runs and their oracle check)")
    ap.add_argument("--workload", default="rank2", choices=["rank2", "precision", "grouped", "adjoint", "copy", "sweep", "plain", "receivers", "rank3", "fom", "offline",
                             "forward512", "rank1batch", "scaling"],
                    help="rank2 (default, the reported line); the others print their own measurement line; "
                         "copy runs a plain device copy of known size (PMC calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(samples would shard across GPUs with no communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2009_11742_amd import Rom

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload != "rank2":
        print(json.dumps(OTHER[args.workload](args, torch, dev)))
        return
    # the oracle references of the K = M = 1024 record run on host threads
    # while the GPU is timed (they need nothing from it)
    target_refs = None if args.no_target else start_target_refs()
    inst = synth.round_to(synth.make_instance(KV, KS, M, seed=SEED), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device=dev)
    c = torch.tensor(inst["c"], dtype=torch.float32, device=dev)
    J = torch.zeros(M, dtype=torch.float64, device=dev)
    V, S = rom.zeros(M, device=dev)
    stream = torch.cuda.current_stream()

    def one_step():
        V.zero_(); S.zero_(); J.zero_()
        rom.run_rank2(mu, V, S, NSTEPS, c=c, J=J, stream=stream)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    # kernel-only timing: events around each run on the launching stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        V.zero_(); S.zero_(); J.zero_()
        ev[k][0].record(stream)
        rom.run_rank2(mu, V, S, NSTEPS, c=c, J=J, stream=stream)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    value = M * NSTEPS * args.steps / wall
    kavg_s = float(np.median(kern_ms)) * 1e-3
    flops_per_launch = 4.0 * KV * KS * M * NSTEPS
    achieved = flops_per_launch / kavg_s / 1e12
    schedule = rom.last_schedule
    kernel = SCHEDULE_KERNELS.get(schedule, (schedule, ()))[0]
    if schedule == "resident":
        # FP32 FMAs on the vector ALUs; the chip's FP32 vector peak counts
        # packed FP32 (this build issues none): 78.6 TFLOP/s without it
        roofline = {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "peak_without_packed_fp32": 78.6}
    else:
        roofline = {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP32_MFMA_PEAK_TFLOPS}
    roofline.update({"traffic": _measured_traffic(schedule), "kernel": kernel, "schedule": schedule,
                     "kernel_ms": float(np.median(kern_ms)), "kernel_ms_runs": [float(x) for x in kern_ms],
                     "flops_per_launch": flops_per_launch})

    Vg = V.cpu().numpy().astype(np.float64).T
    Sg = S.cpu().numpy().astype(np.float64).T
    Jg = J.cpu().numpy()

    # ---- rank-1 path on the same GPU: one sample per stream, each sample's
    # steps captured in a graph (2 kernel nodes per step), S concurrent streams
    rank1 = rank1b = None
    if not args.no_rank1:
        rank1 = rank1_rate(torch, rom, inst, 500)
        rank1b = rank1_batch_rate(torch, rom, inst, 2000)

    # ---- the K = M = 1024 record (FP32, BF16, FP8 operators)
    target = None
    if target_refs is not None:
        target = workload_target(torch, dev, target_refs)

    # ---- the plain FP64 record (K = 64, M in {1, 8}, 2000 steps) and its
    # rank-1 formulation, error against the oracle on every column
    plain = None if args.no_plain else workload_plain(args, torch, dev)

    # ---- CPU baseline: the FP64 oracle on a bounded column sample (all host
    # threads, plus its 1-thread rate), and a numpy/BLAS FP64 rank-2 loop as
    # the CPU + BLAS context
    cpu = None
    errs = None
    if not args.no_cpu:
        import oracle
        nthr = oracle.num_threads()
        ncol = min(M, 8 * max(2, nthr))      # ~10 s of oracle work on 16 host threads
        cols = np.linspace(0, M - 1, ncol).round().astype(int)
        t2 = time.perf_counter()
        ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][cols], NSTEPS,
                               c=inst["c"])
        tcpu = time.perf_counter() - t2
        n1 = 2000
        t3 = time.perf_counter()
        oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][:1], n1, c=inst["c"])
        t1thr = time.perf_counter() - t3
        cpu = {"value": len(cols) * NSTEPS / tcpu, "unit": "sample-steps/s", "cores": nthr, "kind": "oracle",
               "sample": "%d of %d columns x %d steps (K=%d, FP64 plain loops), %.1f s" % (len(cols), M, NSTEPS, KV, tcpu),
               "one_thread": {"value": n1 / t1thr, "sample": "1 column x %d steps" % n1},
               "numpy_blas": numpy_blas_rate(inst)}
        errs = {"max_rel_state_err": max(_err_cols(Vg[:, cols], ref["V"]), _err_cols(Sg[:, cols], ref["S"])),
                "max_rel_qoi_err": float(np.max(np.abs(Jg[cols] - ref["J"]) / ref["J"])),
                "cols_checked": int(len(cols))}

    out = {
        "metric": "sample-steps/s & MFMA util: rank-2 vs rank-1 on 1 MI355X at stated rel. error",
        "value": value,
        "unit": "sample-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rank-2 FP32 leapfrog, Kv=Ks=256, M=256 samples, 10000 steps per run",
                   "kv": KV, "ks": KS, "M": M, "nsteps": NSTEPS, "seed": SEED},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "rank1": rank1,
        "rank2_over_rank1": (value / rank1["value"]) if rank1 else None,
        "rank1_batch": rank1b,
        "rank2_over_rank1_batch": (value / rank1b["value"]) if rank1b else None,
        "accuracy": errs,
        "target_k1024_m1024": target,
        "plain_fp64": plain,
    }
    print(json.dumps(out))


def rank1_rate(torch, rom, inst, nsteps, stream_counts=(1, 8, 32)):
    """Rank-1 sample-steps/s: sample i's nsteps steps captured in graph i
    (two GEMV kernels per step), S graphs replayed on S streams at once; the
    best S is reported.  Graph 0's result is checked against an eager run."""
    kv, ks = inst["Avs"].shape
    dev = torch.device("cuda:0")
    ref_v = torch.zeros(kv, dtype=torch.float32, device=dev)
    ref_s = torch.zeros(ks, dtype=torch.float32, device=dev)
    rom.run_rank1(ref_v, ref_s, float(inst["mu"][0]), nsteps)
    torch.cuda.synchronize()
    cap = torch.cuda.Stream(device=dev)
    best, exact = None, True
    for nstreams in stream_counts:
        graphs, states = [], []
        for i in range(nstreams):
            v = torch.zeros(kv, dtype=torch.float32, device=dev)
            s = torch.zeros(ks, dtype=torch.float32, device=dev)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cap):
                rom.run_rank1(v, s, float(inst["mu"][i % len(inst["mu"])]), nsteps)
            graphs.append(g)
            states.append((v, s))
        streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)]
        rates = []
        for rep in range(3):
            for v, s in states:
                v.zero_(); s.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for g, st in zip(graphs, streams):
                with torch.cuda.stream(st):
                    g.replay()
            torch.cuda.synchronize()
            rates.append(nstreams * nsteps / (time.perf_counter() - t0))
            exact = exact and bool(torch.equal(states[0][0], ref_v) and torch.equal(states[0][1], ref_s))
        rate = float(np.median(rates))
        if best is None or rate > best[0]:
            best = (rate, nstreams)
        del graphs
    return {"value": best[0], "unit": "sample-steps/s", "streams": best[1],
            "graph_equals_eager": exact,
            "sample": "%d samples x %d steps, one graph per sample (2 kernels per step), best of S in %s"
                      % (best[1], nsteps, list(stream_counts))}


def rank1_batch_rate(torch, rom, inst, nsteps):
    """The chip-filling rank-1 reference: all M samples in one launch, one
    workgroup per sample, each half-step a matrix-vector product that reads
    the operator from device memory again (rom_run_rank1_batch).  Median of
    3 event-timed runs; the operator bytes it reads per sample-step give its
    achieved bandwidth (served from the L2s: both FP32 operators, 512 KB at
    K = 256, fit in every XCD's 4 MB L2)."""
    dev = torch.device("cuda:0")
    kv, ks = inst["Avs"].shape
    Mb = len(inst["mu"])
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device=dev)
    V, S = rom.zeros(Mb, device=dev)

    def run():
        V.zero_(); S.zero_()
        rom.run_rank1_batch(mu, V, S, nsteps)
    _, ms = _events_time(torch, run, 3, 1)
    ksec = float(np.median(ms)) * 1e-3
    rate = Mb * nsteps / ksec
    op_bytes = 2.0 * kv * ks * 4
    gbs = rate * op_bytes / 1e9
    return {"value": rate, "unit": "sample-steps/s", "us_per_step": ksec / nsteps * 1e6,
            "operator_bytes_per_sample_step": op_bytes, "operator_GB_per_s": gbs,
            "served_from": "L2" if op_bytes <= 4 * 2 ** 20 else "HBM",
            "ratio_to_hbm_peak": gbs / HBM_PEAK_GBS,
            "sample": "%d samples x %d steps in one launch (rom_run_rank1_batch), median of 3" % (Mb, nsteps)}


# ---- the K = M = 1024 record: FP32, BF16 and FP8 operators (with the state
# operand as a BF16 pair and as one BF16 value), 5000 steps, one sampled
# column checked against the same-input FP64 oracle over the whole run
TARGET_K, TARGET_M, TARGET_N, TARGET_COL = 1024, 1024, 5000, 511
TARGET_PEAKS = {"f32": 157.3, "bf16": 2516.6, "fp8": 5033.2}


def _target_inst():
    import synth
    return synth.round_to(synth.make_instance(TARGET_K, TARGET_K, TARGET_M, seed=0), "f32")


def start_target_refs():
    """FP64 oracle runs of the sampled column with the FP32, BF16-rounded and
    FP8-quantised operators (the oracle's own roundings), on host threads."""
    import concurrent.futures as cf
    import oracle
    inst = _target_inst()
    A, B = inst["Avs"], inst["Asv"]
    amax = float(max(np.max(np.abs(A.astype(np.float32))), np.max(np.abs(B.astype(np.float32)))))
    ops = {"f32": (A, B), "bf16": (oracle.round_bf16(A), oracle.round_bf16(B)),
           "fp8": (oracle.quantize_e4m3(A, amax=amax)[0], oracle.quantize_e4m3(B, amax=amax)[0])}
    ex = cf.ThreadPoolExecutor(max_workers=3)
    mu = inst["mu"][TARGET_COL:TARGET_COL + 1]
    futs = {k: ex.submit(oracle.run_rank2, a, b, inst["b"], inst["dt"], mu, TARGET_N, c=inst["c"])
            for k, (a, b) in ops.items()}
    return {"inst": inst, "futures": futs, "executor": ex, "t0": time.perf_counter()}


def workload_target(torch, dev, refs):
    from paper_2009_11742_amd import Rom
    inst = refs["inst"]
    K, Mt, N, col = TARGET_K, TARGET_M, TARGET_N, TARGET_COL
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device=dev)
    c = torch.tensor(inst["c"], dtype=torch.float32, device=dev)
    runs, states = {}, {}
    for ops, operand in (("f32", "pair"), ("bf16", "pair"), ("bf16", "single"), ("fp8", "pair"),
                         ("fp8", "single")):
        key = ops if operand == "pair" else ops + "_single"
        rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", ops=ops, state_operand=operand)
        V, S = rom.zeros(Mt, device=dev)
        J = torch.zeros(Mt, dtype=torch.float64, device=dev)

        def run():
            V.zero_(); S.zero_(); J.zero_()
            rom.run_rank2(mu, V, S, N, c=c, J=J)
        _, ms = _events_time(torch, run, 1, 1)
        rom.check()
        ksec = float(ms[0]) * 1e-3
        tf = 4.0 * K * K * Mt * N / ksec / 1e12
        runs[key] = {"us_per_step": ksec / N * 1e6, "value": Mt * N / ksec, "tflops": tf,
                     "peak_tflops": TARGET_PEAKS[ops], "frac": tf / TARGET_PEAKS[ops],
                     "schedule": rom.last_schedule,
                     "products": {"f32": "FP32 MFMA (v_mfma_f32_16x16x4f32)",
                                  "bf16": "BF16 MFMA (v_mfma_f32_16x16x32_bf16)",
                                  "fp8": "FP8-E4M3 storage, BF16 MFMA (exact widening)"}[ops],
                     "state_operand": "fp32" if ops == "f32" else ("bf16 pair" if operand == "pair" else "bf16")}
        states[key] = (V[col].cpu().numpy().astype(np.float64), S[col].cpu().numpy().astype(np.float64),
                       float(J[col].cpu()))
        rom.close()
    ref = {k: f.result() for k, f in refs["futures"].items()}
    refs["executor"].shutdown()
    for key, (v, s_, j) in states.items():
        r = ref[key.split("_")[0]]
        e = max(float(np.linalg.norm(v - r["V"][:, 0]) / np.linalg.norm(r["V"][:, 0])),
                float(np.linalg.norm(s_ - r["S"][:, 0]) / np.linalg.norm(r["S"][:, 0])))
        runs[key]["max_rel_state_err_vs_same_input_oracle"] = e
        runs[key]["rel_qoi_err_vs_same_input_oracle"] = abs(j - r["J"][0]) / r["J"][0]
    return {"workload": "Kv=Ks=1024, M=1024, 5000 steps; errors on column %d over all 5000 steps" % col,
            "unit": "sample-steps/s", "runs": runs,
            "oracle_wall_s": time.perf_counter() - refs["t0"]}


def numpy_blas_rate(inst, ncols=16, nsteps=1000):
    """FP64 rank-2 loop in numpy (BLAS GEMMs), the CPU + BLAS context."""
    from threadpoolctl import threadpool_info
    A, B, b, dt = inst["Avs"], inst["Asv"], inst["b"], inst["dt"]
    mu = inst["mu"][:ncols]
    V = np.zeros((A.shape[0], len(mu)))
    S = np.zeros((A.shape[1], len(mu)))
    t0 = time.perf_counter()
    for n in range(nsteps):
        a = (np.pi * (mu * (n * dt) - 1.5)) ** 2
        u = (1.0 - 2.0 * a) * np.exp(-a)
        V += dt * (A @ S + np.outer(b, u))
        S += dt * (B @ V)
    sec = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    return {"value": len(mu) * nsteps / sec, "threads": threads,
            "sample": "%d columns x %d steps, numpy FP64 GEMMs" % (len(mu), nsteps)}


def _events_time(torch, fn, steps, warmup):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in ev]


def workload_precision(args, torch, dev):
    """K = M = 1024, 5000 steps with FP32, BF16 and FP8 operators (the BF16 /
    FP8 products with the state operand as a BF16 pair, and as one BF16
    value: the *_single runs)."""
    import synth
    from paper_2009_11742_amd import Rom
    K, M, N = 1024, 1024, 5000
    inst = synth.round_to(synth.make_instance(K, K, M, seed=0), "f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device=dev)
    out = {"workload": "precision: Kv=Ks=1024, M=1024, 5000 steps", "unit": "sample-steps/s", "runs": {}}
    for ops, operand in (("f32", "pair"), ("bf16", "pair"), ("fp8", "pair"), ("bf16", "single"),
                         ("fp8", "single")):
        rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", ops=ops, state_operand=operand)
        V, S = rom.zeros(M, device=dev)

        def run():
            V.zero_(); S.zero_()
            rom.run_rank2(mu, V, S, N)
        wall, ms = _events_time(torch, run, 3, 1)
        ksec = float(np.median(ms)) * 1e-3
        peak = {"f32": 157.3, "bf16": 2516.6, "fp8": 5033.2}[ops]
        tf = 4.0 * K * K * M * N / ksec / 1e12
        out["runs"][ops if operand == "pair" else ops + "_single"] = {"value": M * N / ksec, "us_per_step": ksec / N * 1e6, "tflops": tf,
                            "mfma_peak_tflops": peak, "frac": tf / peak, "schedule": rom.last_schedule}
        rom.close()
    return out


def workload_grouped(args, torch, dev):
    """64 instances, K in {128..768}, M log-uniform in [16, 512], 4000 steps.
    The headline run takes each instance's column tile (4 or 8 samples per
    workgroup) from the tile autotuner; all-4 and all-8 runs are timed beside
    it, and the tuner's per-bucket tile table is reported."""
    import synth
    from paper_2009_11742_amd import GroupPlan, Rom, tuning
    N = 4000
    draws = synth.grouped_draws(64, base_seed=0)
    insts, flops, ss = [], 0.0, 0
    for K, M, seed in draws:
        insts.append(synth.round_to(synth.make_instance(K, K, M, seed=seed), "f32"))
        flops += 4.0 * K * K * M * N
        ss += M * N
    mus = [torch.tensor(inst["mu"], dtype=torch.float64, device=dev) for inst in insts]

    info = {}

    def timed(schedule):
        roms, Vs, Ss = [], [], []
        for inst in insts:
            rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule=schedule)
            V, S = rom.zeros(len(inst["mu"]), device=dev)
            roms.append(rom); Vs.append(V); Ss.append(S)
        plan = GroupPlan(roms, mus, Vs, Ss)
        if schedule == "auto":
            info["split_k"] = plan.split_k
            info["plan_times_us_per_step"] = plan.times
        wall, ms = _events_time(torch, lambda: plan.run(N), 3, 1)
        plan.close()
        for r in roms:
            r.close()
        return float(np.median(ms)) * 1e-3

    ksec = timed("auto")
    fixed = {"4": timed("columns") * 1e3, "8": timed("columns8") * 1e3}
    table = {}
    for d in tuning.entries():
        if d["m_pad"] == 0 and d["kv_pad"] == d["ks_pad"]:
            table[d["kv_pad"]] = {"us_wg_4": round(d["us"][0], 3), "us_wg_8": round(d["us"][2], 3)}
    n8 = 0
    for (K, M, _), inst in zip(draws, insts):
        t = table.get(-(-K // 64) * 64)
        if t and 0 <= t["us_wg_8"] and -(-M // 8) * t["us_wg_8"] < -(-M // 4) * t["us_wg_4"]:
            n8 += 1
    out = {"workload": "grouped: 64 instances, K in {128..768}, M log-uniform [16,512], 4000 steps",
           "value": ss / ksec, "unit": "sample-steps/s", "tflops": flops / ksec / 1e12,
           "frac_fp32_mfma": flops / ksec / 1e12 / 157.3, "ms_per_run": ksec * 1e3,
           "ms_per_run_fixed_tile": fixed, "instances_on_8_column_tiles": n8,
           "rowsplit_from_padded_k": info.get("split_k"),
           "plan_times_us_per_step": info.get("plan_times_us_per_step"),
           "tile_table_us_per_workgroup_step": table}
    return out


def workload_adjoint(args, torch, dev):
    """K = 512, M = 256, 5000 steps: forward + checkpointed adjoint."""
    import synth
    from paper_2009_11742_amd import Rom
    K, M, N = 512, 256, 5000
    inst = synth.round_to(synth.make_instance(K, K, M, seed=0), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device=dev)
    c = torch.tensor(inst["c"], dtype=torch.float32, device=dev)
    wall, ms = _events_time(torch, lambda: rom.adjoint(mu, N, c), 5, 1)
    ksec = float(np.median(ms)) * 1e-3
    _, ms_rev = _events_time(torch, lambda: rom.adjoint(mu, N, c, stride=-1), 5, 1)
    fwd = 4.0 * K * K * M * N
    out = {"workload": "adjoint: Kv=Ks=512, M=256, 5000 steps, checkpoint stride ceil(sqrt(N))",
           "value": M * N / ksec, "unit": "sample-steps/s (forward + reverse)", "ms_per_gradient": ksec * 1e3,
           "forward_equivalent_tflops": fwd / ksec / 1e12,
           "algorithmic_tflops": (3 * fwd + 2 * 2.0 * K * K * M * N) / ksec / 1e12,
           "ms_per_gradient_time_reversal": float(np.median(ms_rev))}
    rom.close()
    return out


def workload_copy(args, torch, dev):
    """Plain device copy of 256 MiB (PMC FETCH_SIZE / WRITE_SIZE calibration)."""
    n = 64 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    wall, ms = _events_time(torch, lambda: b.copy_(a), 3, 1)
    return {"workload": "copy", "bytes_read": n * 4, "bytes_written": n * 4, "ms": float(np.mean(ms)),
            "GB_per_s": 2 * n * 4 / (float(np.mean(ms)) * 1e-3) / 1e9}


def workload_rank1batch(args, torch, dev):
    """The chip-filling rank-1 reference alone (K = M = 256, 2000 steps, three
    launches): the run profiled for its L2 counters."""
    import synth
    from paper_2009_11742_amd import Rom
    inst = synth.round_to(synth.make_instance(256, 256, 256, seed=0), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    r = rank1_batch_rate(torch, rom, inst, 2000)
    rom.close()
    return dict(workload="rank-1 batch reference: Kv=Ks=256, M=256, 2000 steps", **r)


def workload_sweep(args, torch, dev):
    """Rank-2 vs rank-1 over K in {256, 512, 1024} x M in {1, 4, 16, 64, 256,
    1024} (FP32 operators and states, median of 3 timed runs per point).
    Rank-1 twice: the graph path (one sample per graph, two GEMV launches
    per step, best of 8 / 32 streams) and the batch reference (all M samples
    in one launch, rom_run_rank1_batch)."""
    import synth
    from paper_2009_11742_amd import Rom
    Ms = (1, 4, 16, 64, 256, 1024)
    out = {"workload": "sweep: rank-2 vs rank-1, FP32, K x M", "unit": "sample-steps/s", "points": []}
    for K in (256, 512, 1024):
        inst = synth.round_to(synth.make_instance(K, K, max(Ms), seed=0), "f32")
        rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
        r1 = rank1_rate(torch, rom, inst, 200, stream_counts=(8, 32))
        N = {256: 2000, 512: 1000, 1024: 500}[K]
        for M in Ms:
            mu = torch.tensor(inst["mu"][:M], dtype=torch.float64, device=dev)
            V, S = rom.zeros(M, device=dev)

            def run():
                V.zero_(); S.zero_()
                rom.run_rank2(mu, V, S, N)
            wall, ms = _events_time(torch, run, 3, 1)
            ksec = float(np.median(ms)) * 1e-3

            def run_b():
                V.zero_(); S.zero_()
                rom.run_rank1_batch(mu, V, S, N)
            _, msb = _events_time(torch, run_b, 3, 1)
            kb = float(np.median(msb)) * 1e-3
            pt = {"K": K, "M": M, "nsteps": N, "rank2": M * N / ksec,
                  "rank2_us_per_step": ksec / N * 1e6, "rank1": r1["value"],
                  "rank1_streams": r1["streams"], "ratio": M * N / ksec / r1["value"],
                  "rank1_batch": M * N / kb, "rank1_batch_us_per_step": kb / N * 1e6,
                  "ratio_batch": kb / ksec,
                  "tflops": 4.0 * K * K * M * N / ksec / 1e12, "schedule": rom.last_schedule}
            try:
                pt["tuner_us_per_step"] = rom.schedule_times(M)
            except Exception:
                pt["tuner_us_per_step"] = None     # row-split does not apply: column-block only
            out["points"].append(pt)
        rom.close()
    return out


def workload_scaling(args, torch, dev):
    """The paper's ROM scaling range above the sweep (Sec. 4.2 goes to
    K = 4096): FP32 rank-2 runs at K in {2048, 3072, 4096} x M in {64, 256,
    1024} on the schedule the autotuner picks (the panel schedule above
    Kv_pad + Ks_pad = 4096), median of 3 timed runs; at M = 1024 the error
    of one sampled column against the oracle over the timed run length.
    Per K the rank-1 formulation as launched work (graphs of two GEMV
    launches per step, best of 8 / 32 streams) and the rank-2 / rank-1
    ratio of each point."""
    import oracle
    import synth
    from paper_2009_11742_amd import Rom
    Ks, Ms = (2048, 3072, 4096), (64, 256, 1024)
    if args.scaling_point:
        k, m = (int(v) for v in args.scaling_point.lower().split("x"))
        Ks, Ms = (k,), (m,)
    out = {"workload": "scaling: rank-2 FP32, K in %s x M in %s" % (list(Ks), list(Ms)),
           "unit": "sample-steps/s", "points": []}
    for K in Ks:
        inst = synth.round_to(synth.make_instance(K, K, max(1024, max(Ms)), seed=0), "f32")
        rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
        N = 50 if K <= 2048 else (30 if K <= 3072 else 20)
        r1 = rank1_rate(torch, rom, inst, N, stream_counts=(8, 32))
        out.setdefault("rank1", {})[str(K)] = {"value": r1["value"], "streams": r1["streams"],
                                               "graph_equals_eager": r1["graph_equals_eager"]}
        for M in Ms:
            mu = torch.tensor(inst["mu"][:M], dtype=torch.float64, device=dev)
            V, S = rom.zeros(M, device=dev)

            def run():
                V.zero_(); S.zero_()
                rom.run_rank2(mu, V, S, N)
            wall, ms = _events_time(torch, run, 3, 1)
            rom.check()
            ksec = float(np.median(ms)) * 1e-3
            tf = 4.0 * K * K * M * N / ksec / 1e12
            pt = {"K": K, "M": M, "nsteps": N, "value": M * N / ksec, "us_per_step": ksec / N * 1e6,
                  "tflops": tf, "frac": tf / 157.3, "schedule": rom.last_schedule,
                  "rank2_over_rank1": M * N / ksec / r1["value"]}
            if M >= 1024:
                ci = 517
                r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][ci:ci + 1], N)
                Vg = V.cpu().numpy().astype(np.float64).T[:, ci:ci + 1]
                Sg = S.cpu().numpy().astype(np.float64).T[:, ci:ci + 1]
                pt["max_rel_err_vs_oracle"] = max(_err_cols(Vg, r["V"]), _err_cols(Sg, r["S"]))
            out["points"].append(pt)
        rom.close()
    return out


def workload_forward512(args, torch, dev):
    """The forward run at the adjoint's shape: K = 512, M = 256, 5000 steps,
    FP32, on the schedule the tuning table gives (the row-split kernel with
    16-sample groups on 128 CUs); median of 5 runs, error against the oracle
    on 3 sampled columns."""
    import oracle
    import synth
    from paper_2009_11742_amd import Rom
    K, M, N = 512, 256, 5000
    inst = synth.round_to(synth.make_instance(K, K, M, seed=0), "f32")
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device=dev)
    V, S = rom.zeros(M, device=dev)

    def run():
        V.zero_(); S.zero_()
        rom.run_rank2(mu, V, S, N)
    wall, ms = _events_time(torch, run, 5, 1)
    rom.check()
    ksec = float(np.median(ms)) * 1e-3
    tf = 4.0 * K * K * M * N / ksec / 1e12
    cols = (0, 128, 255)
    Vg, Sg = V.cpu().numpy().astype(np.float64).T, S.cpu().numpy().astype(np.float64).T
    err = 0.0
    for ci in cols:
        r = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"][ci:ci + 1], N)
        err = max(err, _err_cols(Vg[:, ci:ci + 1], r["V"]), _err_cols(Sg[:, ci:ci + 1], r["S"]))
    out = {"workload": "forward512: rank-2 FP32, Kv=Ks=512, M=256, 5000 steps", "unit": "sample-steps/s",
           "value": M * N / ksec, "us_per_step": ksec / N * 1e6, "tflops": tf, "mfma_peak_tflops": 157.3,
           "frac": tf / 157.3, "schedule": rom.last_schedule, "max_rel_err_vs_oracle": err,
           "cols_checked": len(cols)}
    rom.close()
    return out


def workload_plain(args, torch, dev):
    """The plain-method workload: K = 64, M in {1, 8}, 2000 steps, FP64
    states and operators (latency bound: two dependent half-steps per step,
    no roofline; the operator-resident kernel, and at M = 8 also the vector-
    ALU column blocks for comparison), and the rank-1 formulation of sample 0
    (two GEMV launches per step).  Error against the FP64 oracle on every
    column."""
    import oracle
    import synth
    from paper_2009_11742_amd import Rom
    N = 2000
    out = {"workload": "plain: Kv=Ks=64, M in {1, 8}, 2000 steps, FP64", "unit": "sample-steps/s", "runs": {}}
    for M, sched in ((1, "auto"), (8, "auto"), (8, "columns")):
        inst = synth.make_instance(64, 64, M, seed=0)
        rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f64", schedule=sched)
        mu = torch.tensor(inst["mu"], dtype=torch.float64, device=dev)
        V, S = rom.zeros(M, device=dev)

        def run():
            V.zero_(); S.zero_()
            rom.run_rank2(mu, V, S, N)
        wall, ms = _events_time(torch, run, 5, 1)
        ksec = float(np.median(ms)) * 1e-3
        ref = oracle.run_rank2(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], inst["mu"], N)
        err = max(_err_cols(V.cpu().numpy().T, ref["V"]), _err_cols(S.cpu().numpy().T, ref["S"]))
        rec = {"value": M * N / ksec, "us_per_step": ksec / N * 1e6, "max_rel_err_vs_oracle": err,
               "schedule": rom.last_schedule or "columns"}
        if M == 1:
            # the rank-1 formulation of the same sample: two GEMV launches per
            # step (eager, one stream), error against the oracle likewise
            v = torch.zeros(64, dtype=torch.float64, device=dev)
            s = torch.zeros(64, dtype=torch.float64, device=dev)

            def run1():
                v.zero_(); s.zero_()
                rom.run_rank1(v, s, float(inst["mu"][0]), N)
            _, ms1 = _events_time(torch, run1, 5, 1)
            k1 = float(np.median(ms1)) * 1e-3
            e1 = max(_err_cols(v.cpu().numpy()[:, None], ref["V"]), _err_cols(s.cpu().numpy()[:, None], ref["S"]))
            out["rank1"] = {"value": N / k1, "us_per_step": k1 / N * 1e6, "max_rel_err_vs_oracle": e1}
        out["runs"]["M%d" % M + ("" if sched == "auto" else "_" + sched)] = rec
        rom.close()
    out["rank2_M8_over_rank1"] = out["runs"]["M8"]["value"] / out["rank1"]["value"]
    return out


def workload_receivers(args, torch, dev):
    """The bench workload (K = 256, M = 256, 10^4 steps, FP32) with 16
    receiver rows: seismograms (FP64) and per-step ensemble statistics,
    timed against the plain run of the same shape (4-column schedule)."""
    import synth
    from paper_2009_11742_amd import Rom
    R = 16
    inst = synth.round_to(synth.make_instance(KV, KS, M, seed=SEED), "f32")
    C = torch.tensor(np.asarray(np.random.default_rng(7).standard_normal((R, KV)), dtype=np.float32), device=dev)
    rom = Rom(inst["Avs"], inst["Asv"], inst["b"], inst["dt"], state="f32", schedule="columns")
    mu = torch.tensor(inst["mu"], dtype=torch.float64, device=dev)
    V, S = rom.zeros(M, device=dev)
    Y = torch.empty((NSTEPS, R, M), dtype=torch.float64, device=dev)
    st = torch.empty((NSTEPS, R, 5), dtype=torch.float64, device=dev)
    from paper_2009_11742_amd import _lib
    from paper_2009_11742_amd.rom import _ptr, _stream_handle

    def run_rc():
        V.zero_(); S.zero_()
        _lib.check(_lib.load().rom_run_receivers(rom.handle, M, _ptr(mu), 0, NSTEPS, _ptr(V), _ptr(S), R, _ptr(C),
                                                 _ptr(Y), _ptr(st), _stream_handle(None)))

    def run_plain():
        V.zero_(); S.zero_()
        rom.run_rank2(mu, V, S, NSTEPS)
    _, ms_rc = _events_time(torch, run_rc, 3, 1)
    _, ms_pl = _events_time(torch, run_plain, 3, 1)
    t_rc, t_pl = float(np.median(ms_rc)) * 1e-3, float(np.median(ms_pl)) * 1e-3
    rom.close()
    return {"workload": "receivers: Kv=Ks=256, M=256, 10000 steps, R=16 receivers, Y + mean/var/p5/p50/p95 per step",
            "value": M * NSTEPS / t_rc, "unit": "sample-steps/s", "ms_per_run": t_rc * 1e3,
            "plain_ms_per_run": t_pl * 1e3, "overhead": t_rc / t_pl - 1.0}


def workload_rank3(args, torch, dev):
    """Affine family: Q = 4 terms of Kv = Ks = 512, P = 64 parameter points
    of M = 64 samples each, 2000 steps.  Each point's operators are assembled
    and packed on the device from the resident terms (timed per instance);
    the P instances then run in one grouped launch (timed per run)."""
    import synth
    from paper_2009_11742_amd import AffineFamily, GroupPlan
    K, Q, P, M, N = 512, 4, 64, 64, 2000
    fam_in = synth.make_affine_family(K, K, Q, P, M, seed=0)
    b32 = fam_in["b"].astype(np.float32).astype(np.float64)
    fam = AffineFamily(fam_in["Avs_terms"], fam_in["Asv_terms"], b32, 0.1, state="f32")
    dts = [float(np.float32(0.5 / float(np.abs(th) @ fam_in["smax"]))) for th in fam_in["theta"]]
    torch.cuda.synchronize()
    roms = [fam.instance(fam_in["theta"][0], dt=dts[0])]   # first call: warm
    roms[0].close()
    t0 = time.perf_counter()
    roms = [fam.instance(th, dt=d) for th, d in zip(fam_in["theta"], dts)]
    torch.cuda.synchronize()
    t_asm = (time.perf_counter() - t0) / P
    mus = [torch.tensor(m, dtype=torch.float64, device=dev) for m in fam_in["mu"]]
    Vs, Ss = [], []
    for r in roms:
        V, S = r.zeros(M, device=dev)
        Vs.append(V); Ss.append(S)
    plan = GroupPlan(roms, mus, Vs, Ss)
    schedule, plan_us = plan.schedule, plan.times
    _, ms = _events_time(torch, lambda: plan.run(N), 3, 1)
    ksec = float(np.median(ms)) * 1e-3
    plan.check()
    plan.close()
    for r in roms:
        r.close()
    fam.close()
    # the column-block plan of the same instances, for comparison
    famc = AffineFamily(fam_in["Avs_terms"], fam_in["Asv_terms"], b32, 0.1, state="f32", schedule="columns")
    romc = [famc.instance(th, dt=d) for th, d in zip(fam_in["theta"], dts)]
    planc = GroupPlan(romc, mus, Vs, Ss)
    _, msc = _events_time(torch, lambda: planc.run(N), 3, 1)
    planc.close()
    for r in romc:
        r.close()
    famc.close()
    flops = 4.0 * K * K * M * N * P
    return {"workload": "rank3: affine family, Q=4 terms, Kv=Ks=512, P=64 points x M=64 samples, 2000 steps",
            "value": P * M * N / ksec, "unit": "sample-steps/s", "ms_per_run": ksec * 1e3,
            "tflops": flops / ksec / 1e12, "frac_fp32_mfma": flops / ksec / 1e12 / 157.3,
            "plan": schedule, "plan_tuning_us_per_step": plan_us,
            "column_plan_ms_per_run": float(np.median(msc)),
            "assembly_ms_per_instance": t_asm * 1e3}


def _fom_bytes(d, M):
    """Algorithmic HBM bytes of one FOM step (FP64): both CSR operators once,
    per half-step the updated state read and written and the other state
    read once, and the source vector."""
    nzv, nzs = int(d["Av"][0][-1]), int(d["As"][0][-1])
    a = 4 * (d["nv"] + 1) + 12 * nzv + 4 * (d["ns"] + 1) + 12 * nzs
    return a + 8 * M * (3 * d["nv"] + 3 * d["ns"]) + 8 * d["nv"]


def workload_fom(args, torch, dev):
    """Rank-2 FOM stepping (the contrast workload: sparse, bandwidth-bound):
    velocity grids 256 x 1024 and 512 x 2048 (785,152 and 3,143,168 DOF),
    M in {1, 4, 16, 48} forcing periods, dt = 0.05 s (Appendix A), 200 timed
    steps.  Reports per point the step time, sample-steps/s, algorithmic
    GB/s against the 8 TB/s HBM peak, and the rank-2 gain
    s(M) = M t(1) / t(M) of Appendix B."""
    import synth
    from paper_2009_11742_amd import Fom
    N = 200
    out = {"workload": "fom: shear-wave FOM, grids 256x1024 and 512x2048, M in {1,4,16,48}, dt 0.05, 200 steps",
           "unit": "sample-steps/s", "hbm_peak_GBps": 8000.0, "points": []}
    grids, Ms, runs = ((256, 1024), (512, 2048)), (1, 4, 16, 48), 3
    if args.fom_point:
        nr, nth, mm = (int(x) for x in args.fom_point.split("x"))
        grids, Ms, runs = ((nr, nth),), (mm,), max(1, args.steps)
        out["workload"] = "fom: shear-wave FOM, grid %dx%d, M = %d, dt 0.05, 200 steps" % (nr, nth, mm)
    for nr, nth in grids:
        d = synth.make_shear_fom(nr, nth, dt=0.05)
        F = Fom(d["Av"], d["As"], d["f"], d["dt"])
        t1 = None
        for M in Ms:
            mu = torch.tensor(synth.fom_periods(M, seed=M), dtype=torch.float64, device=dev)
            V, S = F.zeros(M, device=dev)

            def run():
                F.run(mu, V, S, N)
            _, ms = _events_time(torch, run, runs, 1)
            t = float(np.median(ms)) * 1e-3 / N
            t1 = t if M == 1 else (t1 if t1 is not None else float("nan"))
            gbs = _fom_bytes(d, M) / t / 1e9
            out["points"].append({"grid": "%dx%d" % (nr, nth), "dof": d["nv"] + d["ns"], "M": M,
                                  "us_per_step": t * 1e6, "value": M / t, "GBps": gbs, "frac_hbm": gbs / 8000.0,
                                  "rank2_gain": M * t1 / t})
        F.close()
    return out


def workload_offline(args, torch, dev):
    """Offline stage on the 256 x 1024 grid: 256 FOM snapshots (8 periods x
    32 snapshots, every 10th step at the CFL time step), POD of the velocity
    and stress snapshot matrices (energy 1e-10), Galerkin projection onto the
    resulting bases.  Reports times and the ranks."""
    import synth
    from paper_2009_11742_amd import Fom, pod
    d = synth.make_shear_fom(256, 1024)
    F = Fom(d["Av"], d["As"], d["f"], d["dt"])
    M, nsnap, every = 8, 32, 10
    mu = torch.tensor(synth.fom_periods(M, seed=0), dtype=torch.float64, device=dev)
    V, S = F.zeros(M, device=dev)
    XV = torch.empty((d["nv"], M * nsnap), dtype=torch.float64, device=dev)
    XS = torch.empty((d["ns"], M * nsnap), dtype=torch.float64, device=dev)
    for c in range(nsnap):
        F.run(mu, V, S, every, n0=c * every)
        XV[:, c * M:(c + 1) * M] = V
        XS[:, c * M:(c + 1) * M] = S
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Pv, sv, kv = pod(XV, tol=1e-10)
    t1 = time.perf_counter()
    Ps, ss, ks = pod(XS, tol=1e-10)
    t2 = time.perf_counter()
    Pv2, _, _ = pod(XV, tol=1e-10)                    # second call: warm
    t3 = time.perf_counter()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    F.project(Pv, Ps)                                 # warm-up
    ev[0].record()
    for _ in range(3):
        F.project(Pv, Ps)
    ev[1].record()
    torch.cuda.synchronize()
    F.close()
    return {"workload": "offline: 256x1024 grid, 256 snapshots, POD (energy 1e-10) + Galerkin projection",
            "kv": kv, "ks": ks, "pod_velocity_ms": (t1 - t0) * 1e3, "pod_stress_ms": (t2 - t1) * 1e3,
            "pod_velocity_warm_ms": (t3 - t2) * 1e3, "project_ms": ev[0].elapsed_time(ev[1]) / 3,
            "sigma_ratio_kept": float(sv[kv - 1] / sv[0])}


OTHER = {"forward512": workload_forward512, "precision": workload_precision, "grouped": workload_grouped, "adjoint": workload_adjoint,
         "copy": workload_copy, "sweep": workload_sweep, "plain": workload_plain, "rank1batch": workload_rank1batch,
         "receivers": workload_receivers, "rank3": workload_rank3, "fom": workload_fom,
         "offline": workload_offline, "scaling": workload_scaling}


if __name__ == "__main__":
    main()
