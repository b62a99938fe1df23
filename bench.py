"""Benchmark: full RQRCP (Alg. 4) in fp64 on one MI355X against the unpivoted
blocked QR built from the same kernels (the paper's "qr" comparator).

Workload (default): 8192 x 8192 i.i.d. N(0, 1), b = 64, p = 8, seed 2.
A step is one whole RQRCP factorization of a fresh copy of A that is already
resident in HBM (the copies are made before the timed region).  The line
printed reports the RQRCP rate in QR-equivalent GFLOP/s (2 m n^2 - 2 n^3 / 3),
the time of both factorizations and their ratio, the stage breakdown (a pass
of K steps with HIP events around every stage), the roofline position of the
dominant stage (its launches timed with HIP events inside the timed region,
where only that stage records events) and the CPU oracle timed on a bounded
sample of the same workload.  Unless --no-extras is given, the same line also
carries the rest of the metric: the 512 x 512 latency (`c1_rqrcp`, per call
and per block) and TUXV at k = 256 on the 20000 x 10000 matrix in FP64 and
both mixed levels (`tuxv_c3*`: solves/s, p99, truncation error next to the
oracle's and the optimum).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--no-extras] [--check] [--no-lookahead]

Other workloads (one JSON line each, same keys):
    --workload c2_lr        RQRCP of the 8192 x 8192 rank-512 product of
                            Gaussians plus 1e-8 noise (numerical rank, pivots)
    --workload c1           512 x 512, b = 32: latency per call and per block
    --workload rsrqrcp_c2   RSRQRCP (Alg. 5, a new sample per block) on the
                            default matrix, with RQRCP and QR timed beside it
    --workload c3 [--jmax J]  TRQRCP + TUXV (Alg. 7 with j_max = J) at k = 256
    --workload c3 --precision mixed|mixed_bf16
                            the same TUXV in mixed precision (FP32 matrix cores
                            for the products with A, the sketch on the FP32 or
                            BF16 ones, FP64 otherwise)
    --workload c4 [--tune-cache F]
                            512 uneven matrices (TRQRCP + TUXV at k = 32) in one
                            captured batch, mixed and FP64, b and tiles from the
                            autotuner cache
    --workload c5 [--requests R --serve-max N --serve-streams S --hbm-budget-gb G]
                            the request server: a stream of TUXV requests of
                            mixed sizes and ranks, solves/s and p50/p99 latency
    --workload select_expect  the selection experiment of Section 3.2 replayed
                            through the sketch and the sample QRCP (trials/s)
    --copy-calibration MIB  only a plain device copy (HBM counter calibration)
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("RQRCP time vs GPU unpivoted QR (8192² fp64); TUXV solves/s + p99 at stated err")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6          # dense fp64 MFMA
FP64_VALU_PEAK_TFLOPS = 78.6     # 256 CUs x 4 SIMDs x 16 fp64 FMA lanes x 2 flops x 2.4 GHz

# Stages whose arithmetic is plain vector fp64 (no matrix cores): their roofline
# is the vector-ALU peak, not the HBM/MFMA one.
ALU_STAGES = {"sample_qrcp"}
# Kernel behind each stage (for the counter summaries under profiles/).
STAGE_KERNEL = {"sample_qrcp": ("sample_qrcp_kernel", "paper_1509_06820_amd/csrc/qrcp.hip"),
                "panel": ("recon_kernel", "paper_1509_06820_amd/csrc/cholqr.hip"),
                "gemm_update": ("gemm_kernel", "paper_1509_06820_amd/csrc/gemm.hip"),
                "gemm_yta": ("gemm_kernel", "paper_1509_06820_amd/csrc/gemm.hip")}


def qr_flops(m, n):
    k = min(m, n)
    # Householder QR of an m x n matrix: 2 k^2 (max(m, n) - k / 3) flops
    # (2 m n^2 - 2 n^3 / 3 for m >= n; 4 n^3 / 3 for m = n), the same count
    # as flops_first_columns over all columns
    return 2.0 * k * k * max(m, n) - 2.0 * k ** 3 / 3.0


def flops_first_columns(m, n, k):
    """QR-equivalent flops of the first k columns (reflector j applied to the
    n - j - 1 columns to its right over m - j rows, plus its own norm)."""
    j = np.arange(k, dtype=np.float64)
    return float(np.sum(4.0 * (m - j) * (n - j - 1) + 3.0 * (m - j)))


def host_cpu():
    """CPU model and physical core count of this host (from /proc/cpuinfo)."""
    model, cores = None, set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ":" not in ln:
                    continue
                key, val = [x.strip() for x in ln.split(":", 1)]
                if key == "model name" and model is None:
                    model = val
                elif key == "physical id":
                    phys = val
                elif key == "core id":
                    core = val
                    cores.add((phys, core))
    except OSError:  # pragma: no cover
        pass
    return model, (len(cores) or os.cpu_count())


def cpu_baseline(A, b, p, seed, nblocks):
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    model, phys = host_cpu()
    m, n = A.shape
    k = nblocks * b
    t0 = time.perf_counter()
    oracle.rqrcp(A, b, p, seed=seed, k=k)
    dt = time.perf_counter() - t0
    gflops = flops_first_columns(m, n, k) / dt / 1e9
    return {"value": round(gflops, 3), "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {nblocks} blocks (k = {k} pivots, sketch included) of the {m}x{n} RQRCP, "
                      f"QR-equivalent flops of those columns / wall time {dt:.2f} s",
            "cpu_model": model, "physical_cores": phys, "logical_cpus": os.cpu_count()}


def measured_traffic(stage, workload):
    """HBM bytes per launch of the stage's kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factor), or
    None when there is none or the kernel source changed since it was taken."""
    import hashlib
    if stage not in STAGE_KERNEL:
        return None
    kname, src = STAGE_KERNEL[stage]
    path = os.path.join(ROOT, "profiles", f"{kname}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for ln in f:
            if ":" in ln and not ln.startswith("#"):
                k, v = ln.split(":", 1)
                fields[k.strip()] = v.strip()
    with open(os.path.join(ROOT, src), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if fields.get("source_sha256") != digest:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mib):
    """A plain device copy of known size, for scaling the HBM counters."""
    import torch
    torch.cuda.set_device(0)
    n = mib * 1024 * 1024 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8,
                      "launches": 3}), flush=True)


def run_select_expect(args):
    """Replay of the selection experiment of Section 3.2 (Fig. selectExpect)
    through the product's sketch and sample QRCP: A = Q diag(phi^j) with Haar
    Q (512 x 512); per trial a new Philox seed, B = Omega A, the first sample
    pivot; the mean of ||a_jmax|| per cell (the GPU test of the same replay
    compares it with the exact expectation).  value: trials per second over
    all cells."""
    import torch
    from paper_1509_06820_amd import binding, inputs
    n, trials = 512, 1500 * max(1, args.steps // 5)
    cells = [(0.5, 8), (0.9, 8), (0.95, 16), (0.99, 4), (0.99, 32)]
    out, total_s = [], 0.0
    for phi, l in cells:
        Q = inputs.haar_columns(np.random.default_rng(int(phi * 1000) + l), n, n)
        A = torch.from_numpy(np.asfortranarray(Q * phi ** np.arange(n))).cuda()
        wk = binding.workspace(binding.RQ_OP_RQRCP, n, n, n, l, 0, A.device)
        ws = binding.workspace(binding.RQ_OP_SAMPLE_QRCP, l, n, 0, 1, 0, A.device)
        for sd in range(args.warmup):
            binding.rq_sample_qrcp(binding.rq_sketch(A, l, 10 ** 9 + sd, work=wk), 1, work=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pivs = [binding.rq_sample_qrcp(binding.rq_sketch(A, l, 7_000_000 + 10_000 * l + t, work=wk), 1, work=ws)[1]
                for t in range(trials)]
        torch.cuda.synchronize()
        total_s += time.perf_counter() - t0
        vals = phi ** torch.stack(pivs).cpu().numpy()[:, 0].astype(np.float64)
        out.append({"phi": phi, "l": l, "mean": round(float(vals.mean()), 5),
                    "se": round(float(vals.std(ddof=1) / np.sqrt(trials)), 5)})
    line = {
        "metric": METRIC, "value": round(len(cells) * trials / total_s, 1),
        "unit": "selection trials/s (sketch + first sample pivot, 512x512)", "n_gpus": 1, "steps": trials,
        "warmup": args.warmup, "ms_per_step": round(1e3 * total_s / (len(cells) * trials), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "select_expect_replay", "n": n, "trials_per_cell": trials,
                   "inputs": "Haar Q diag(phi^j)"},
        "cells": out,
    }
    print(json.dumps(line), flush=True)


def c3_measure(A, prm, K, W, prec="fp64", jmax=1, time_trq=True):
    """TUXV (and TRQRCP) at rank k on the resident C3 matrix A: per-solve HIP
    event latencies over K timed solves after W warm-up solves, the
    truncation error (evaluated after the timed region) against the
    Eckart-Young optimum and the oracle's stored error."""
    import torch
    from paper_1509_06820_amd import binding, inputs
    k, b, p, seed = prm["k"], prm["b"], prm["p"], prm["seed"]
    m, n = A.shape
    stream = torch.cuda.current_stream()
    mixed = prec != "fp64"
    w_tux = binding.workspace(binding.RQ_OP_TUXV, m, n, k, b, p, A.device, prec)
    for _ in range(W):
        binding.rq_tuxv(A, k, b, p, seed, work=w_tux, jmax=jmax, precision=prec)
    torch.cuda.synchronize()

    def time_trqrcp(level):
        # TRQRCP overwrites its input: each timed call gets its own copy of A,
        # made before the timed region
        work = binding.workspace(binding.RQ_OP_TRQRCP, m, n, k, b, p, A.device, level)
        for _ in range(W):
            binding.rq_trqrcp(A, k, b, p, seed, work=work, precision=level)
        L = binding.load()
        assert A.stride(0) == 1 and A.stride(1) == m  # column-major, ld = m
        jp = torch.empty(n, dtype=torch.int64, device=A.device)
        tk = torch.empty(k, dtype=torch.float64, device=A.device)
        inf = torch.zeros(1, dtype=torch.int32, device=A.device)
        ktr = min(K, 5)
        copies = [A.clone() for _ in range(ktr)]
        torch.cuda.synchronize()
        pairs = []
        for i in range(ktr):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rc = L.rq_trqrcp(stream.cuda_stream, m, n, k, copies[i].data_ptr(), m, b, p, seed,
                             binding.PRECISIONS[level], jp.data_ptr(), tk.data_ptr(), work.data_ptr(), work.numel(),
                             inf.data_ptr())
            e1.record(stream)
            assert rc == 0, (level, rc)
            pairs.append((e0, e1))
        torch.cuda.synchronize()
        assert int(inf.item()) == 0
        del copies, work
        return float(np.mean([a.elapsed_time(z) for a, z in pairs]))

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    res = None
    for i in range(K):
        ev[i][0].record(stream)
        res = binding.rq_tuxv(A, k, b, p, seed, work=w_tux, jmax=jmax, precision=prec)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(z) for a, z in ev])
    U, s, VT, info = res
    assert int(info.item()) == 0, int(info.item())
    err = (torch.linalg.norm(A - (U * s) @ VT) / torch.linalg.norm(A)).item()
    del U, s, VT, res, w_tux
    opt = inputs.optimal_truncation_error(inputs.sigma_power(n, 0.9, 10.0), k)
    ms = float(lat.mean())
    # TUXV flops: the TRQRCP(k) products (2kmn), one product with A per
    # step (2mnk each), the sketch (2lmn)
    flops = 2.0 * k * m * n + jmax * 2.0 * m * n * k + 2.0 * (b + p) * m * n
    out = {"solves_per_s": round(1e3 / ms, 3), "ms": round(ms, 3), "p50_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3), "gflops": round(flops / (ms * 1e-3) / 1e9, 2),
           "precision": prec, "truncation_error": err, "optimal_error": opt, "error_over_optimum": round(err / opt, 6)}
    if time_trq:
        out["trqrcp_ms"] = round(time_trqrcp(prec), 3)
    gold = os.path.join(ROOT, "tests", "golden", "c3_tuxv_oracle_error.txt")
    if jmax == 1 and os.path.exists(gold):
        with open(gold) as f:
            for ln in f:
                if ln.startswith("oracle_error:"):
                    out["oracle_error"] = float(ln.split(":", 1)[1])
                    out["error_over_oracle"] = round(err / out["oracle_error"], 6)
    return out


def run_c3(args):
    """TRQRCP and TUXV at rank k = 256 on the 20000 x 10000 matrix with
    sigma_i = 0.9^(i/10): solves/s and p99 latency of TUXV (j_max = --jmax,
    precision --precision) over the timed solves, TRQRCP time, and the
    truncation error against the Eckart-Young optimum and the oracle's."""
    import torch
    from paper_1509_06820_amd import inputs
    A_host, prm = inputs.config_matrix("c3")
    m, n = A_host.shape
    A = torch.from_numpy(A_host).cuda()
    del A_host
    prec, jmax = args.precision, args.jmax
    if prec != "fp64" and jmax != 1:
        raise SystemExit("--precision mixed takes j_max = 1")
    print(f"[bench] workload c3 {m}x{n} k={prm['k']} jmax={jmax} precision={prec}: {args.warmup} warmup + "
          f"{args.steps} timed solves", file=sys.stderr, flush=True)
    r = c3_measure(A, prm, args.steps, args.warmup, prec, jmax)
    line = {
        "metric": METRIC,
        "value": r["solves_per_s"],
        "unit": f"TUXV solves/s ({prec}, 20000x10000, k=256" + (f", j_max={jmax})" if jmax != 1 else ")"),
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms"], "p99_ms": r["p99_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"mixed": "f32/f64", "mixed_bf16": "bf16/f32/f64"}.get(prec, "f64"), "data": "synthetic",
        "config": {"workload": f"tuxv_c3_{prec}" if prec != "fp64" else "tuxv_c3" if jmax == 1 else
                   f"tuxv_c3_jmax{jmax}", "m": m, "n": n, "k": prm["k"], "b": prm["b"], "p": prm["p"],
                   "seed": prm["seed"], "jmax": jmax, "inputs": "U diag(0.9^(i/10)) V^T, Haar factors"},
        **{kk: v for kk, v in r.items() if kk not in ("solves_per_s", "ms", "p99_ms")},
    }
    print(json.dumps(line), flush=True)


def run_c4(args):
    """The batched workload: 512 matrices (m log-uniform on [64, 2048], n
    uniform on [64, m], sigma_j = 10^(-6 j/n), k = 32, p = 8), TRQRCP + TUXV
    for all of them as one planned batch, captured in a HIP graph and
    replayed; b and the tile of the grouped products from the autotuner.
    Timed: graph replays (HIP events), FP32 products ("mixed") and FP64;
    value = mixed solves/s.  Error: the truncation error of 16 matrices
    against the FP64 oracle (after the timed region)."""
    import torch
    from paper_1509_06820_amd import autotune, binding, inputs
    t_gen = time.perf_counter()
    batch = inputs.batch_c4(512)
    mats = [torch.from_numpy(A).cuda() for A, _ in batch]
    seeds = [prm["seed"] for _, prm in batch]
    k, p = 32, 8
    print(f"[bench] c4: 512 matrices generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    W, K = args.warmup, args.steps
    res = {}
    outs = {}
    for prec in ("mixed", "fp64"):
        choice = autotune.tune(mats, k, p, seeds, precision=prec, cache_path=args.tune_cache,
                               log=lambda s_: print(s_, file=sys.stderr, flush=True))
        bt = binding.BatchTUXV(mats, k, choice["b"], p, seeds, precision=prec, tile=choice["tile"])
        bt.run()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            with torch.cuda.graph(g, stream=st):
                bt.run()
        torch.cuda.synchronize()
        for _ in range(W):
            g.replay()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        cur = torch.cuda.current_stream()
        for i in range(K):
            ev[i][0].record(cur)
            g.replay()
            ev[i][1].record(cur)
        torch.cuda.synchronize()
        lat = np.array([a.elapsed_time(z) for a, z in ev])
        info = bt.info[:512].cpu().numpy()
        assert np.all(info == 0), np.nonzero(info)
        res[prec] = {"ms_per_batch": round(float(lat.mean()), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
                     "solves_per_s": round(512 / (lat.mean() * 1e-3), 1), "b": choice["b"], "tile": choice["tile"]}
        outs[prec] = [(bt.U[i].cpu().numpy(), bt.sigma[i].cpu().numpy(), bt.VT[i].cpu().numpy())
                      for i in range(0, 512, 32)]
        del g
        bt.close()
        print(f"[bench] c4 {prec}: {res[prec]}", file=sys.stderr, flush=True)
    # truncation errors of 16 matrices against the FP64 oracle (untimed)
    import oracle
    ratios = {"mixed": [], "fp64": []}
    for j, i in enumerate(range(0, 512, 32)):
        A = batch[i][0]
        ref = oracle.tuxv(A, k, res["mixed"]["b"], p, seed=seeds[i])
        nrm = np.linalg.norm(A)
        e_ref = np.linalg.norm(A - (ref["U"] * ref["s"]) @ ref["VT"]) / nrm
        for prec in ("mixed", "fp64"):
            U, sg, VT = outs[prec][j]
            ratios[prec].append(float(np.linalg.norm(A - (U * sg) @ VT) / nrm / e_ref))
    sums = sum(A.shape[0] * A.shape[1] for A in mats)
    line = {
        "metric": METRIC, "value": res["mixed"]["solves_per_s"],
        "unit": "batched TUXV solves/s (512 uneven matrices, k=32, FP32 products)", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": res["mixed"]["ms_per_batch"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": "tuxv_batched_c4", "matrices": 512, "k": k, "p": p, "sum_mn": sums,
                   "inputs": "U diag(10^(-6 j/n)) V^T, m log-uniform [64, 2048], n uniform [64, m]"},
        "mixed": res["mixed"], "fp64": res["fp64"],
        "mixed_over_fp64": round(res["mixed"]["solves_per_s"] / res["fp64"]["solves_per_s"], 3),
        "error_over_oracle_max": {pr: round(max(v), 5) for pr, v in ratios.items()},
        "hbm_gbs_a_reads": round(3 * 8 * sums / (res["mixed"]["ms_per_batch"] * 1e-3) / 1e9, 1),
    }
    print(json.dumps(line), flush=True)


def run_c5(args):
    """The served request stream: requests with m, n log-uniform on
    [256, 8192] (m >= n), k in {16, 32, 64, 128, 256}, sigma_i = 0.95^i,
    half FP64 and half mixed precision, Poisson arrivals; the server admits
    them by HBM footprint and runs them with continuous batching.  First a
    saturated FP64 pass (all arrivals at 0) measures the plain throughput;
    the timed pass offers the mixed stream at 0.7 of it.  value: solves/s of
    the timed pass; p50/p99 latency (arrival -> completion)."""
    import torch
    from paper_1509_06820_amd import binding, inputs, serve
    n_req = args.requests
    specs = inputs.serving_c5(n_req, smax=args.serve_max)
    t_gen = time.perf_counter()
    mats = [serve.serving_matrix_device(r["i"], r["m"], r["n"]) for r in specs]
    torch.cuda.synchronize()
    print(f"[bench] c5: {n_req} request matrices made on the GPU in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)
    budget = args.hbm_budget_gb * 1e9

    def reqs(precisions, gaps):
        out, t = [], 0.0
        for r, A, prec, gap in zip(specs, mats, precisions, gaps):
            out.append(serve.Request(r["i"], A, r["k"], prec, seed=50_000 + r["i"], arrival=t))
            t += gap
        return out

    # warm-up: every distinct (k, precision) once
    warm = reqs([binding.RQ_FP64] * n_req, [0.0] * n_req)[:min(n_req, 12)]
    serve.TuxvServer(budget, streams=args.serve_streams).serve(warm)
    sat = serve.TuxvServer(budget, streams=args.serve_streams).serve(reqs([binding.RQ_FP64] * n_req, [0.0] * n_req))
    mu = sat["solves_per_s"]
    lam = 0.7 * mu
    precs = [binding.RQ_MIXED if r["mixed"] else binding.RQ_FP64 for r in specs]
    timed_reqs = reqs(precs, [r["gap"] / lam for r in specs])
    srv = serve.TuxvServer(budget, streams=args.serve_streams)
    st = srv.serve(timed_reqs)
    bad = [r.id for r in timed_reqs if int(r.info.item()) != 0]
    assert not bad, bad
    line = {
        "metric": METRIC, "value": round(st["solves_per_s"], 2),
        "unit": "served TUXV solves/s (Poisson arrivals at 0.7x saturated FP64 throughput)", "n_gpus": 1,
        "steps": n_req, "warmup": len(warm), "ms_per_step": round(1e3 / st["solves_per_s"], 3),
        "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 and f32/f64", "data": "synthetic",
        "config": {"workload": "tuxv_served_c5", "requests": n_req, "size_range": [256, args.serve_max],
                   "k_choices": [16, 32, 64, 128, 256], "hbm_budget_gb": args.hbm_budget_gb,
                   "streams": args.serve_streams, "arrival_rate_per_s": round(lam, 2)},
        "saturated_fp64": {k_: (round(v, 3) if isinstance(v, float) else v) for k_, v in sat.items()},
        "served": {k_: (round(v, 3) if isinstance(v, float) else v) for k_, v in st.items()},
    }
    print(json.dumps(line), flush=True)


def c1_latency(K, W):
    """RQRCP of the 512 x 512 configuration (b = 32, 16 blocks): microseconds
    per factorization and per block (HIP events, mean of K after W warm-ups;
    each call factors its own copy made before the timed region)."""
    import torch
    from paper_1509_06820_amd import binding, inputs
    A_host, prm = inputs.config_matrix("c1")
    A = torch.from_numpy(A_host).cuda()
    b, p, seed = prm["b"], prm["p"], prm["seed"]
    m, n = A.shape
    L = binding.load()
    stream = torch.cuda.current_stream()
    work = binding.workspace(binding.RQ_OP_RQRCP, m, n, n, b, p, A.device)
    jp = torch.empty(n, dtype=torch.int64, device=A.device)
    tau = torch.empty(n, dtype=torch.float64, device=A.device)
    inf = torch.zeros(1, dtype=torch.int32, device=A.device)
    copies = [A.clone() for _ in range(W + K)]
    torch.cuda.synchronize()
    pairs = []
    for i in range(W + K):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rc = L.rq_rqrcp(stream.cuda_stream, m, n, copies[i].data_ptr(), m, b, p, seed, binding.RQ_FP64,
                        jp.data_ptr(), tau.data_ptr(), work.data_ptr(), work.numel(), inf.data_ptr())
        e1.record(stream)
        assert rc == 0, rc
        pairs.append((e0, e1))
    torch.cuda.synchronize()
    assert int(inf.item()) == 0
    t = np.array([a.elapsed_time(z) for a, z in pairs[W:]]) * 1e3
    blocks = (n + b - 1) // b
    return {"us_per_factorization": round(float(t.mean()), 1), "us_per_block": round(float(t.mean()) / blocks, 2),
            "p99_us": round(float(np.percentile(t, 99)), 1), "blocks": blocks, "m": m, "n": n, "b": b, "p": p}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2_iid",
                    choices=["c2_iid", "c2_lr", "c1", "c3", "c4", "c5", "rsrqrcp_c2", "select_expect"])
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (c4; default: the user cache)")
    ap.add_argument("--requests", type=int, default=200, help="c5: number of requests")
    ap.add_argument("--serve-max", type=int, default=8192, help="c5: largest matrix dimension")
    ap.add_argument("--serve-streams", type=int, default=4, help="c5: streams of the server")
    ap.add_argument("--hbm-budget-gb", type=float, default=64.0, help="c5: HBM admission budget")
    ap.add_argument("--jmax", type=int, default=1, help="TUXV steps (Alg. 7 j_max) for --workload c3")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "mixed_bf16"],
                    help="arithmetic of the products with A (RQ_FP64, RQ_MIXED, RQ_MIXED_BF16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the 512 x 512 latency and the TUXV (20000 x 10000) part")
    ap.add_argument("--cpu-blocks", type=int, default=3)
    ap.add_argument("--check", action="store_true", help="residual of the last factorization (untimed)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    ap.add_argument("--no-lookahead", action="store_true",
                    help="run each block's trailing update right after its R12 instead of in the next sample "
                         "QRCP's launch (the sample QRCP's own counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (requested --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import torch
    from paper_1509_06820_amd import binding, inputs

    torch.cuda.set_device(0)
    if args.no_lookahead:
        binding.rq_set_lookahead(False)
    if args.workload == "c3":
        run_c3(args)
        return
    if args.workload == "select_expect":
        run_select_expect(args)
        return
    if args.workload == "c4":
        if args.tune_cache is None:
            from paper_1509_06820_amd import autotune
            args.tune_cache = autotune.DEFAULT_CACHE
        run_c4(args)
        return
    if args.workload == "c5":
        run_c5(args)
        return
    resample = args.workload == "rsrqrcp_c2"
    A_host, prm = inputs.config_matrix("c2_iid" if resample else args.workload)
    b, p, seed = prm["b"], prm["p"], prm["seed"]
    m, n = A_host.shape
    k = min(m, n)
    A = torch.from_numpy(A_host).cuda()
    W, K = args.warmup, args.steps
    print(f"[bench] workload {args.workload} {m}x{n} b={b} p={p}: {W} warmup + {K} timed steps", file=sys.stderr,
          flush=True)

    L = binding.load()
    stream = torch.cuda.current_stream()
    s_ptr = binding._stream(stream)
    work_rq = binding.workspace(binding.RQ_OP_RQRCP, m, n, k, b, p, A.device, args.precision)
    work_qr = binding.workspace(binding.RQ_OP_QR, m, n, k, b, 0, A.device)
    jpvt = torch.empty(n, dtype=torch.int64, device=A.device)
    tau = torch.empty(k, dtype=torch.float64, device=A.device)
    tau_qr = torch.empty(k, dtype=torch.float64, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)

    # fresh copies of A for every step, made before any timed region: W
    # warmup, K steps with HIP events around every stage (the breakdown),
    # then the K timed steps
    copies = [A.clone() for _ in range(W + 2 * K)]
    copies_qr = [A.clone() for _ in range(W + K)]
    torch.cuda.synchronize()

    def rqrcp(F):
        rc = L.rq_rqrcp(s_ptr, m, n, binding._ptr(F), m, b, p, seed, binding.PRECISIONS[args.precision],
                        binding._ptr(jpvt), binding._ptr(tau),
                        binding._ptr(work_rq), work_rq.numel(), binding._ptr(info))
        assert rc == 0, rc

    def rsrqrcp(F):
        rc = L.rq_rsrqrcp(s_ptr, m, n, binding._ptr(F), m, b, p, seed, binding._ptr(jpvt), binding._ptr(tau),
                          binding._ptr(work_rq), work_rq.numel(), binding._ptr(info))
        assert rc == 0, rc

    # the method the line reports (Alg. 4, or Alg. 5 for rsrqrcp_c2)
    method, method_name = (rsrqrcp, "rsrqrcp") if resample else (rqrcp, "rqrcp")

    def qr(F):
        rc = L.rq_unpivoted_qr(s_ptr, m, n, binding._ptr(F), m, b, binding._ptr(tau_qr), binding._ptr(work_qr),
                               work_qr.numel(), binding._ptr(info))
        assert rc == 0, rc

    copies_rq = [A.clone() for _ in range(W + K)] if resample else []
    for i in range(W):
        method(copies[i])
        qr(copies_qr[i])
        if resample:
            rqrcp(copies_rq[i])
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # pass 1: HIP events around every stage (on the kernels' stream) give the
    # stage breakdown and the dominant stage
    binding.rq_profile_start()
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(K):
        method(copies[W + i])
    e1.record(stream)
    torch.cuda.synchronize()
    stages = binding.rq_profile_stop()
    ms_prof = e0.elapsed_time(e1) / K
    assert int(info.item()) == 0, f"info = {int(info.item())}"
    dom = max(stages, key=lambda nm: stages[nm]["ms"])
    # pass 2, the timed steps: only the dominant stage keeps its events, so
    # its launches are timed live inside the timed region at little cost
    binding.rq_profile_start([dom])
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    for i in range(K):
        method(copies[W + K + i])
    e1.record(stream)
    torch.cuda.synchronize()
    wall_rq = time.perf_counter() - t_wall
    dom_timed = binding.rq_profile_stop()[dom]
    L.rq_profile_select(0xFFFFFFFF)
    ms_rq = e0.elapsed_time(e1) / K
    assert int(info.item()) == 0, f"info = {int(info.item())}"
    print(f"[bench] {method_name} {ms_rq:.3f} ms/factorization", file=sys.stderr, flush=True)
    ms_rq4 = None
    if resample:
        # Alg. 4 on the same matrix, for the cost of repeated sampling
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(K):
            rqrcp(copies_rq[W + i])
        e1.record(stream)
        torch.cuda.synchronize()
        ms_rq4 = e0.elapsed_time(e1) / K
        print(f"[bench] rqrcp {ms_rq4:.3f} ms/factorization", file=sys.stderr, flush=True)

    # timed unpivoted QR
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(K):
        qr(copies_qr[W + i])
    e1.record(stream)
    torch.cuda.synchronize()
    ms_qr = e0.elapsed_time(e1) / K
    print(f"[bench] unpivoted qr {ms_qr:.3f} ms/factorization", file=sys.stderr, flush=True)

    flops = qr_flops(m, n)
    value = flops / (ms_rq * 1e-3) / 1e9

    # dominant stage and its roofline position
    per_step = {name: dict(ms=v["ms"] / K, launches=v["count"] / K, bytes=v["bytes"] / K, flops=v["flops"] / K)
                for name, v in stages.items()}
    # the dominant stage as timed in the timed region
    d = dict(ms=dom_timed["ms"] / K, launches=dom_timed["count"] / K, bytes=dom_timed["bytes"] / K,
             flops=dom_timed["flops"] / K)
    intensity = d["flops"] / d["bytes"] if d["bytes"] else float("inf")
    ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if dom in ALU_STAGES:
        achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s"}
    elif intensity < ridge:
        achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = None if resample else measured_traffic(dom, args.workload)
    roof["kernel"] = dom
    roof["avg_launch_us"] = round(d["ms"] / d["launches"] * 1e3, 2) if d["launches"] else None

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s (QR-equivalent, RSRQRCP)" if resample else "GFLOP/s (QR-equivalent, RQRCP)",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_rq, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rsrqrcp_c2_iid" if resample else f"rqrcp_{args.workload}", "m": m, "n": n, "b": b,
                   "p": p, "seed": seed,
                   "inputs": "i.i.d. N(0,1)" if args.workload in ("c2_iid", "rsrqrcp_c2") else args.workload},
        f"{method_name}_ms": round(ms_rq, 3),
        "unpivoted_qr_ms": round(ms_qr, 3),
        f"{method_name}_over_qr": round(ms_rq / ms_qr, 4),
        f"{method_name}_wall_ms": round(wall_rq * 1e3 / K, 3),
        "stages_ms_per_step": {nm: round(v["ms"], 3) for nm, v in sorted(per_step.items(), key=lambda kv: -kv[1]["ms"])},
        "profiled_ms_per_step": round(ms_prof, 3),
        "roofline": roof,
    }
    if args.check:
        F = copies[W + 2 * K - 1]
        Q = torch.linalg.householder_product(F, tau)
        res = (torch.linalg.norm(A[:, jpvt] - Q @ torch.triu(F)) / torch.linalg.norm(A)).item()
        line["residual"] = res
    if resample:
        line["rqrcp_ms"] = round(ms_rq4, 3)
        line["rsrqrcp_over_rqrcp"] = round(ms_rq / ms_rq4, 4)
    if not args.no_cpu_baseline and not resample:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(A_host, b, p, seed, args.cpu_blocks)
    if args.workload == "c2_iid" and not args.no_extras:
        # the rest of the metric: TUXV solves/s and p99 at its error (20000 x
        # 10000, k = 256; FP64 and both mixed levels), and the latency of the
        # 512 x 512 configuration
        del copies, copies_qr, copies_rq, work_rq, work_qr, A
        torch.cuda.empty_cache()
        print("[bench] 512x512 latency ...", file=sys.stderr, flush=True)
        line["c1_rqrcp"] = c1_latency(max(K, 10), max(W, 3))
        print("[bench] tuxv 20000x10000 k=256 ...", file=sys.stderr, flush=True)
        A3_host, prm3 = inputs.config_matrix("c3")
        A3 = torch.from_numpy(A3_host).cuda()
        del A3_host
        k3 = max(K // 2, 5)
        line["tuxv_c3"] = c3_measure(A3, prm3, k3, min(W, 2), "fp64")
        for lvl in ("mixed", "mixed_bf16"):
            line[f"tuxv_c3_{lvl}"] = c3_measure(A3, prm3, k3, min(W, 2), lvl)
            line[f"tuxv_c3_{lvl}"]["speedup_over_fp64"] = round(
                line[f"tuxv_c3_{lvl}"]["solves_per_s"] / line["tuxv_c3"]["solves_per_s"], 3)
        print(f"[bench] tuxv fp64 {line['tuxv_c3']['ms']:.3f} ms, mixed {line['tuxv_c3_mixed']['ms']:.3f} ms, "
              f"mixed_bf16 {line['tuxv_c3_mixed_bf16']['ms']:.3f} ms", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
