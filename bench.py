"""Benchmark: Y = K~ W on one MI355X for the headline workload (N = 65536
points in d = 8 from a 16-component Gaussian mixture, Gaussian kernel h = 1,
leaf 128, tol 1e-5, rank <= 128, distance admissibility tau = 2, W: N x 256).

One step = one full evaluation (permute-in, up pass, far reduction + down
pass, near field + leaf far part, permute-out) on inputs resident in HBM.
Prints one JSON line.  Throughput counts algorithmic flops only:
2 Q (2 E_V + 2 E_T + E_B + E_D), never the dense 2 N^2 Q.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (vector = matrix)
PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32
PEAK_HBM_GBPS = 8000.0
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 MFMA


def kernel_source_hash() -> str:
    """Hash of every source that decides what the timed launch executes: the
    kernels, the store layout and segments, the queue order, and the types."""
    h = hashlib.sha256()
    for f in ("hm_kernels.hip", "hm_build.hip", "hm_sched.hip", "hm_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1812_07152_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(name: str, launches_bytes_fallback=None):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{name}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def measured_counters(name: str):
    """MFMA utilisation of the dominant kernel from the committed counter
    summary, if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{name}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return {"mfma_busy_frac": d["mfma_busy_frac"],
            "mfma_executed_tflop_per_launch": d["mfma_executed_tflop_per_launch"],
            "source": f"profiles/{name}.json (rocprofv3 SQ_VALU_MFMA_BUSY_CYCLES, SQ_INSTS_VALU_MFMA_MOPS_F64)"}


def time_variant(hmx, torch, M, W, steps, warmup, flags=0, prec=None):
    """Times `steps` evaluations Y = K~ W on torch's current stream after
    `warmup` untimed ones; returns (ms per step by the host clock, per-phase
    launch milliseconds and counts from HIP events, Y)."""
    Y = torch.empty_like(W)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        hmx.hm_eval(M, W, Y, flags=flags, stream=stream, prec=prec)
    torch.cuda.synchronize()
    hmx.hm_profile_reset(M)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hmx.hm_eval(M, W, Y, flags=flags | hmx.HM_PROFILE, stream=stream, prec=prec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, n = hmx.hm_profile_read(M)
    hmx.hm_check(M)  # raises if a bounded dependency wait expired (the results would be invalid)
    return (t1 - t0) * 1e3 / steps, ms, n, Y


def host_description() -> dict:
    """The host the CPU baseline ran on: model name and usable cores."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "affinity_cores": len(os.sched_getaffinity(0))}


def cpu_baseline(w, X, W, budget_s: float = 15.0, eps_rows: int = 256):
    """The oracle (plain C, FP64, OpenMP over nodes) on a bounded column sample
    of the same workload: its own compression (untimed), then the timed tree
    walk, as the paper times (median of 5 runs), on all usable host cores and
    on one core.  The sample's width is chosen so that the five runs take about
    budget_s.  Also returns the oracle's Y on the sampled columns (the first
    qs columns of W) and the exact rows (K W)[rows, :qs] of eps_rows seeded rows
    (the direct definition), for the accuracy figures."""
    import numpy as np

    from oracle import oracle as orc
    H = orc.OracleH2.from_workload(w, X)
    st = H.stats()
    cores = orc.max_threads()
    # two probes fit time = fixed + per_col * columns (the tree walk's fixed
    # part is large next to a few columns, so one probe overestimates)
    probe = []
    for q in (4, 16):
        Wp = np.ascontiguousarray(W[:, :q])
        t = time.perf_counter()
        H.eval(Wp)
        probe.append(time.perf_counter() - t)
    per_col = max((probe[1] - probe[0]) / 12, 1e-9)
    fixed = max(probe[0] - 4 * per_col, 0.0)
    qs = int(max(4, min(w.Q, (budget_s / 5 - fixed) / per_col)))
    Ws = np.ascontiguousarray(W[:, :qs])
    times = []
    for _ in range(5):
        t = time.perf_counter()
        Yo = H.eval(Ws)
        times.append(time.perf_counter() - t)
    dt = float(np.median(times))
    # one core, on a narrower sample (the fixed part grows with it too)
    q1 = 4
    orc.set_threads(1)
    try:
        W1 = np.ascontiguousarray(W[:, :q1])
        t = time.perf_counter()
        H.eval(W1)
        dt1 = time.perf_counter() - t
    finally:
        orc.set_threads(cores)
    rows = np.random.default_rng(12345).choice(w.N, eps_rows, replace=False)
    exact = H.exact_rows(rows, Ws)
    eps_f = float(np.linalg.norm(Yo[rows] - exact) / np.linalg.norm(exact))
    base = {"value": st["flops_per_col"] * qs / dt / 1e9, "unit": "GFLOP/s",
            "cores": cores, "kind": "oracle",
            "sample": f"same compressed workload, {qs} of the {w.Q} columns of W; median of 5 timed "
                      f"tree walks ({dt:.2f} s each)",
            "seconds_median": dt, "seconds_all": times, **host_description(),
            "one_core": {"value": st["flops_per_col"] * q1 / dt1 / 1e9, "unit": "GFLOP/s", "columns": q1,
                         "seconds": dt1},
            "eps_f_sampled_oracle": eps_f}
    return base, {"cols": qs, "Y": Yo, "rows": rows, "exact": exact}


def errors_vs_oracle(Ygpu, ref) -> dict:
    """A GPU result against the oracle on the oracle's sampled columns: the
    relative Frobenius difference to the oracle's own evaluation (same
    compression) and the sampled-row eps_f against the exact (K W) rows."""
    import numpy as np
    Y = np.asarray(Ygpu, dtype=np.float64)[:, :ref["cols"]]
    return {"rel_err_vs_oracle": float(np.linalg.norm(Y - ref["Y"]) / np.linalg.norm(ref["Y"])),
            "eps_f_sampled": float(np.linalg.norm(Y[ref["rows"]] - ref["exact"]) / np.linalg.norm(ref["exact"]))}


def bench_batched(args) -> dict:
    """Batched form: 64 compressed matrices of uneven size (N in [2048, 32768],
    d in {3, 8}, leaf 64..128, tol 1e-6) and width (Q in [8, 512]), FP32, in
    one persistent launch with an autotuned column tile, against the plain
    path (one hm_eval per matrix) on the same inputs."""
    import torch

    import paper_1812_07152_amd as hmx
    import workloads as wl
    specs = wl.batched_workloads(64)
    t = time.perf_counter()
    mats = []
    for w in specs:
        R = hmx.hm_compress(wl.gen_points(w), kernel=w.kernel, h=w.h, leaf_size=w.m, tol=w.tol,
                            max_rank=w.rmax, admissibility=w.adm, tau=w.tau,
                            sample_rows=w.sample_rows, seed=w.sample_seed)
        mats.append(hmx.hm_load_compressed_mem(R, 0, hmx.precbit(hmx.HM_PREC_FP32)))
        del R
    t_build = time.perf_counter() - t
    Qs = [w.Q for w in specs]
    flops = sum(hmx.hm_info(m)["flops_per_col"] * q for m, q in zip(mats, Qs))
    Ws = [torch.from_numpy(wl.gen_w(w)).to("cuda", torch.float32) for w in specs]
    Ys = [torch.empty_like(W) for W in Ws]
    Yb = [torch.empty_like(W) for W in Ws]

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    def plain():
        for m, W, Y in zip(mats, Ws, Ys):
            hmx.hm_eval(m, W, Y)

    ms_plain = timed(plain)
    t = time.perf_counter()
    B = hmx.hm_batch_create(mats, Qs, dtype=hmx.HM_F32, flags=hmx.HM_BATCH_AUTOTUNE)
    t_tune = time.perf_counter() - t
    ms_batch = timed(lambda: hmx.hm_batch_eval(B, Ws, Yb))
    hmx.hm_batch_check(B)
    err = max(float((a - b).norm() / b.norm()) for a, b in zip(Yb, Ys))
    info = hmx.hm_batch_info(B)
    # the oracle beside it: the three smallest matrices, their first columns
    small = sorted(range(len(specs)), key=lambda i: specs[i].N)[:3]
    cpu = cpu_baseline_batched([specs[i] for i in small], [Ws[i][:, :8].double().cpu().numpy() for i in small],
                               [Yb[i][:, :8].double().cpu().numpy() for i in small])
    return {
        "metric": "batched K~W GFLOP/s (algorithmic), 64 matrices, one persistent launch",
        "value": flops / (ms_batch * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batch,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c3_64_matrices_n2048_32768", "matrices": len(specs),
                   "Q_range": [min(Qs), max(Qs)], "N_range": [min(w.N for w in specs), max(w.N for w in specs)],
                   "gflop_per_step": flops / 1e9},
        "plain_per_matrix": {"ms_per_step": ms_plain, "value": flops / (ms_plain * 1e-3) / 1e9},
        "speedup_vs_plain": ms_plain / ms_batch,
        "max_rel_diff_vs_plain": err,
        "frac_of_fp32_peak": flops / (ms_batch * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
        "autotune": {"column_tile": info["column_tile"], "tuned_ms": info["tuned_ms"], "seconds": t_tune},
        "tasks": info["n_tasks"], "workgroups": info["workgroups"], "setup_s": {"compress_and_load": t_build},
        "cpu_baseline": cpu,
    }


def cpu_baseline_batched(specs, Ws, Ys) -> dict:
    """The oracle on a few of the batched matrices (its own compression,
    untimed; the tree walk timed): GFLOP/s over them, and the batched FP32
    results' largest relative error against it (the bar of the plain FP32
    path is 5e-6: FP32 rounding of the blocks and W)."""
    import numpy as np

    import workloads as wl
    from oracle import oracle as orc
    flops, secs, errs = 0.0, 0.0, []
    for w, W, Y in zip(specs, Ws, Ys):
        H = orc.OracleH2.from_workload(w, wl.gen_points(w))
        Wr = np.ascontiguousarray(W.astype(np.float32).astype(np.float64))
        t = time.perf_counter()
        ref = H.eval(Wr)
        secs += time.perf_counter() - t
        flops += H.stats()["flops_per_col"] * W.shape[1]
        errs.append(float(np.linalg.norm(Y - ref) / np.linalg.norm(ref)))
    return {"value": flops / secs / 1e9, "unit": "GFLOP/s", "cores": orc.max_threads(), "kind": "oracle",
            "sample": f"{len(specs)} smallest matrices (N {[w.N for w in specs]}), 8 columns each",
            "max_rel_err_batched_fp32_vs_oracle": max(errs)}


def bench_serving(args) -> dict:
    """Serving form: 8 resident matrices (N 16384..524288, d in {3, 8, 28},
    H^2 and HSS, tol 1e-5), FP32, requests with Q ~ U{1..256} on a uniformly
    chosen matrix.  Measures the served saturation throughput (a burst of
    requests drained by the server) against the plain path (the same requests
    one at a time with hm_eval), then p50/p99 latency under open-loop Poisson
    arrivals at 25 / 50 / 80 % of the served saturation rate."""
    import threading

    import numpy as np
    import torch

    import paper_1812_07152_amd as hmx
    import workloads as wl
    specs = wl.serving_workloads()
    t = time.perf_counter()
    mats = []
    for w in specs:
        R = hmx.hm_compress(wl.gen_points(w), kernel=w.kernel, h=w.h, leaf_size=w.m, tol=w.tol,
                            max_rank=w.rmax, admissibility=w.adm, tau=w.tau,
                            sample_rows=w.sample_rows, seed=w.sample_seed)
        mats.append(hmx.hm_load_compressed_mem(R, 0, hmx.precbit(hmx.HM_PREC_FP32)
                                               | (hmx.HM_LOAD_SYMMETRIC if args.serving_symmetric else 0)))
        del R
        print(f"[serving] built {w.name} ({time.perf_counter() - t:.0f} s)", file=sys.stderr, flush=True)
    t_build = time.perf_counter() - t
    infos = [hmx.hm_info(m) for m in mats]
    Wsrc = [torch.randn(w.N, 256, device="cuda", dtype=torch.float32,
                        generator=torch.Generator(device="cuda").manual_seed(w.w_seed)) for w in specs]
    rng = np.random.default_rng(args.serving_seed)

    def draw(n):
        return [(int(rng.integers(0, len(specs))), int(rng.integers(1, 257))) for _ in range(n)]

    def flops(reqs):
        return sum(infos[m]["flops_per_col"] * q for m, q in reqs)

    # plain path: one request at a time
    burst = draw(args.burst)
    for m, q in burst[:8]:
        hmx.hm_eval(mats[m], Wsrc[m][:, :q], torch.empty(specs[m].N, q, device="cuda"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for m, q in burst:
        hmx.hm_eval(mats[m], Wsrc[m][:, :q], torch.empty(specs[m].N, q, device="cuda"))
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0

    S = hmx.hm_server_create(0, hbm_budget=24 << 30, max_slots=args.serving_slots, dtype=hmx.HM_F32)
    ids = [hmx.hm_server_add(S, mt) for mt in mats]

    def run(reqs, gaps):
        """Submit reqs (after the given inter-arrival gaps, seconds) and poll
        until all are done; returns (latencies in ms, wall seconds)."""
        out = {}
        pending = {}
        lock = threading.Lock()

        def producer():
            t_next = time.perf_counter()
            for (m, q), gap in zip(reqs, gaps):
                t_next += gap
                while time.perf_counter() < t_next:
                    time.sleep(0.0001)
                Y = torch.empty(specs[m].N, q, device="cuda")
                tk = hmx.hm_submit(S, ids[m], Wsrc[m][:, :q], Y)
                with lock:
                    pending[tk] = Y
        start = time.perf_counter()
        th = threading.Thread(target=producer)
        th.start()
        deadline = start + 300
        while len(out) < len(reqs):
            assert time.perf_counter() < deadline, "serving run did not drain"
            with lock:
                tks = list(pending)
            for tk in tks:
                done, lat = hmx.hm_poll(S, tk)
                if done:
                    out[tk] = lat / 1e3
                    with lock:
                        del pending[tk]
            time.sleep(0.0002)
        th.join()
        return list(out.values()), time.perf_counter() - start

    run(draw(16), [0.0] * 16)                      # warm-up
    lat, wall = run(burst, [0.0] * len(burst))    # saturation: everything at once
    sat_rps = len(burst) / wall
    levels = []
    for frac in (0.25, 0.5, 0.8):
        rate = frac * sat_rps
        n = max(16, int(rate * args.serving_seconds))
        reqs = draw(n)
        gaps = list(rng.exponential(1.0 / rate, n))
        lat, wall = run(reqs, gaps)
        levels.append({"offered_rps": rate, "fraction_of_saturation": frac, "requests": n,
                       "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                       "achieved_rps": n / wall, "gflops": flops(reqs) / wall / 1e9})
    # one more served request on the smallest matrix, checked against the oracle
    Wc = Wsrc[0][:, :16].contiguous()
    Yc = torch.full_like(Wc, float("nan"))
    tk = hmx.hm_submit(S, ids[0], Wc, Yc)
    t_end = time.perf_counter() + 60
    while not hmx.hm_poll(S, tk)[0]:
        assert time.perf_counter() < t_end, "check request did not complete"
        time.sleep(0.0005)
    st = hmx.hm_server_stats(S)
    hmx.hm_server_destroy(S)
    cpu = cpu_baseline_served(specs[0], Wc.double().cpu().numpy(), Yc.double().cpu().numpy())
    return {
        "metric": "served K~W throughput (GFLOP/s, algorithmic) and p50/p99 latency",
        "value": flops(burst) / (len(burst) / sat_rps) / 1e9, "unit": "GFLOP/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c5_8_resident_n16384_524288", "matrices": [w.name for w in specs],
                   "Q": "U{1..256}", "burst_requests": len(burst), "slots": args.serving_slots, "hbm_budget_gib": 24,
                   "symmetric_store": bool(args.serving_symmetric),
                   "store_gb_fp32": sum(i["bytes_fp32"] for i in infos) / 1e9},
        "saturation_rps": sat_rps,
        "plain_per_request": {"rps": len(burst) / plain_s, "gflops": flops(burst) / plain_s / 1e9},
        "speedup_vs_plain": (len(burst) / plain_s) and sat_rps / (len(burst) / plain_s),
        "levels": levels,
        "server": {"sweeps": st["sweeps"], "completed": st["completed"], "failed": st["failed"],
                   "requests_per_sweep": st["completed"] / max(st["sweeps"], 1),
                   "peak_inflight_sweeps": st["peak_inflight"], "peak_working_set_gib": st["peak_bytes"] / 2**30},
        "setup_s": {"compress_and_load": t_build},
        "cpu_baseline": cpu,
    }


def cpu_baseline_served(w, W, Y) -> dict:
    """The oracle on one served request (the smallest resident matrix, its
    own compression untimed, the tree walk timed); the served FP32 result's
    relative error against it (FP32 bar 5e-6, as the plain FP32 path)."""
    import numpy as np

    import workloads as wl
    from oracle import oracle as orc
    H = orc.OracleH2.from_workload(w, wl.gen_points(w))
    Wr = np.ascontiguousarray(W.astype(np.float32).astype(np.float64))
    t = time.perf_counter()
    ref = H.eval(Wr)
    dt = time.perf_counter() - t
    return {"value": H.stats()["flops_per_col"] * W.shape[1] / dt / 1e9, "unit": "GFLOP/s",
            "cores": orc.max_threads(), "kind": "oracle",
            "sample": f"one request of {W.shape[1]} columns on {w.name}",
            "rel_err_served_fp32_vs_oracle": float(np.linalg.norm(Y - ref) / np.linalg.norm(ref))}


def _mixed_one(args, w, adm_name: str, kernel_name: str, keep_cols: int = 0) -> dict:
    """Times one workload in FP64, split BF16 and FP32 on the same compressed
    matrix; errors are relative Frobenius norms against the FP64 result.
    keep_cols: also return W's and each result's first columns (host)."""
    import torch

    import paper_1812_07152_amd as hmx
    import workloads as wl
    t = time.perf_counter()
    R = hmx.hm_compress(wl.gen_points(w), kernel=w.kernel, h=w.h, leaf_size=w.m, tol=w.tol,
                        max_rank=w.rmax, admissibility=w.adm, tau=w.tau, sample_rows=w.sample_rows,
                        seed=w.sample_seed)
    t_compress = time.perf_counter() - t
    print(f"[mixed] {w.name}: compressed in {t_compress:.0f} s", file=sys.stderr, flush=True)
    mask = hmx.precbit(hmx.HM_PREC_FP64) | hmx.precbit(hmx.HM_PREC_BF16X3) | hmx.precbit(hmx.HM_PREC_FP32)
    M = hmx.hm_load_compressed_mem(R, 0, mask)
    del R
    info = hmx.hm_info(M)
    flops = info["flops_per_col"] * w.Q
    W = torch.from_numpy(wl.gen_w(w)).cuda()
    out, results = {}, {}
    for name, Wx, prec in (("fp64", W, hmx.HM_PREC_FP64), ("bf16x3", W, hmx.HM_PREC_BF16X3),
                           ("fp32", W.float(), hmx.HM_PREC_FP32)):
        Y = torch.empty_like(Wx)
        for _ in range(args.warmup):
            hmx.hm_eval(M, Wx, Y, prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            hmx.hm_eval(M, Wx, Y, prec=prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        hmx.hm_check(M)
        results[name] = Y.double()
        out[name] = {"ms_per_step": ms, "gflops": flops / (ms * 1e-3) / 1e9}
        print(f"[mixed] {w.name} {name}: {ms:.2f} ms", file=sys.stderr, flush=True)
    ref = results["fp64"]
    for name in ("bf16x3", "fp32"):
        out[name]["rel_err_vs_fp64"] = float((results[name] - ref).norm() / ref.norm())
    kept = None
    if keep_cols:
        kept = {"W": W[:, :keep_cols].cpu().numpy(),
                **{k: v[:, :keep_cols].cpu().numpy() for k, v in results.items()}}
    del results, ref, W, M
    return {
        "_cols": kept,
        "config": {"workload": w.name, "N": w.N, "d": w.d, "Q": w.Q, "kernel": kernel_name, "h": w.h,
                   "leaf": w.m, "tol": w.tol, "max_rank": w.rmax, "admissibility": adm_name,
                   "gflop_per_step": flops / 1e9, "E_V": info["E_V"], "E_T": info["E_T"],
                   "E_B": info["E_B"], "E_D": info["E_D"],
                   "fp64_transfer_share": 4 * info["E_T"] / info["flops_per_col"]},
        "paths": out,
        "speedup_vs_fp64": out["fp64"]["ms_per_step"] / out["bf16x3"]["ms_per_step"],
        "setup_s": {"compress": t_compress},
    }


def bench_mixed_c4(args) -> dict:
    """The mixed-precision form on its own workload: N = 262144 points in
    d = 28 (i.i.d. normal), kernel exp(-r/4), leaf 256, tol 1e-4, rank <= 256,
    HSS, W: N x 1024; split BF16 against the plain FP64 and FP32 paths on the
    same matrix.  Accuracy: against the GPU FP64 result (which the parity
    tests hold to the oracle's tree walk at this size), and against the exact
    (K W) rows of 256 seeded rows on 16 columns (the oracle's direct
    definition), for FP64 and split BF16."""
    import workloads as wl
    r = _mixed_one(args, wl.C4, "HSS", "exp(-r/h)", keep_cols=16)
    cols = r.pop("_cols")
    cpu = cpu_baseline_exact_rows(wl.C4, wl.gen_points(wl.C4), cols)
    m = r["paths"]["bf16x3"]
    return {"metric": "mixed-precision K~W GFLOP/s (algorithmic) vs the plain FP64 path",
            "value": m["gflops"], "unit": "GFLOP/s", "ms_per_step": m["ms_per_step"], "dtype": "bf16x3+f64",
            **r, "cpu_baseline": cpu}


def cpu_baseline_exact_rows(w, X, cols, n_rows: int = 256) -> dict:
    """Exact rows (K W)[rows, :q] from the oracle's direct definition (no
    compression), timed, and the sampled-row eps_f of each GPU result."""
    import numpy as np

    from oracle import oracle as orc
    rows = np.random.default_rng(54321).choice(w.N, n_rows, replace=False)
    Wq = np.ascontiguousarray(cols["W"])
    t = time.perf_counter()
    exact = orc.exact_rows(X, w.kernel, w.h, rows, Wq)
    dt = time.perf_counter() - t
    out = {"kind": "oracle", "cores": orc.max_threads(), "sample": f"exact rows: {n_rows} rows x {Wq.shape[1]} columns",
           "seconds": dt, "value": 2.0 * n_rows * w.N * Wq.shape[1] / dt / 1e9, "unit": "GFLOP/s (direct K W rows)"}
    for k, Y in cols.items():
        if k != "W":
            out[f"eps_f_sampled_{k}"] = float(np.linalg.norm(Y[rows] - exact) / np.linalg.norm(exact))
    return out


def bench_points(args) -> dict:
    """Blocks computed from the points (FP64): the N = 65536, d = 8, Q = 256
    workload (reported) and the N = 262144, d = 28, Q = 1024 HSS one beside it,
    each timed with stored blocks and with the near and far blocks computed
    from the points and skeletons on a store loaded without them."""
    import torch

    import paper_1812_07152_amd as hmx
    import workloads as wl

    both = hmx.HM_NEAR_FROM_POINTS | hmx.HM_FAR_FROM_POINTS
    fp64 = hmx.precbit(hmx.HM_PREC_FP64)
    runs = {}
    for w in (wl.C2, wl.C4):
        X = wl.gen_points(w)
        R = hmx.hm_compress(X, kernel=w.kernel, h=w.h, leaf_size=w.m, tol=w.tol, max_rank=w.rmax,
                            admissibility=w.adm, tau=w.tau, sample_rows=w.sample_rows, seed=w.sample_seed)
        M = hmx.hm_load_compressed_mem(R, 0, fp64)
        Mp = hmx.hm_load_compressed_mem(R, 0, fp64 | hmx.HM_LOAD_NO_NEAR_BLOCKS | hmx.HM_LOAD_NO_FAR_BLOCKS)
        del R
        hmx.hm_set_points(Mp, X, w.kernel, w.h)
        info = hmx.hm_info(M)
        flops = info["flops_per_col"] * w.Q
        Wd = torch.from_numpy(wl.gen_w(w)).to("cuda", torch.float64)
        ms0, _, _, Ys = time_variant(hmx, torch, M, Wd, args.steps, args.warmup)
        msp, php, npp, Yp = time_variant(hmx, torch, Mp, Wd, args.steps, args.warmup, flags=both)
        runs[w.name] = {
            "N": w.N, "d": w.d, "Q": w.Q, "ms_stored": ms0, "ms_from_points": msp,
            "launch_ms_from_points": php[3] / max(npp[3], 1),
            "gflops_from_points": flops / (msp * 1e-3) / 1e9,
            "store_gb": info["bytes_fp64"] / 1e9, "store_gb_without_near_and_far": hmx.hm_info(Mp)["bytes_fp64"] / 1e9,
            "rel_diff_vs_stored": float(torch.linalg.norm(Yp - Ys) / torch.linalg.norm(Ys))}
        print(f"[points] {w.name}: stored {ms0:.2f} ms, from points {msp:.2f} ms", file=sys.stderr, flush=True)
        del M, Mp, Wd, Ys, Yp
    main = runs[wl.C2.name]
    return {
        "metric": "K~W GFLOP/s (algorithmic), near and far blocks computed from the points",
        "value": main["gflops_from_points"], "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main["ms_from_points"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded points and normal W; no dataset)",
        "config": {"workload": wl.C2.name, "flags": "HM_NEAR_FROM_POINTS|HM_FAR_FROM_POINTS",
                   "load": "HM_LOAD_NO_NEAR_BLOCKS|HM_LOAD_NO_FAR_BLOCKS"},
        "runs": runs,
    }


def bench_mixed(args) -> dict:
    """Mixed-precision form: N = 262144 points in d = 28 (i.i.d. normal),
    kernel exp(-r/4), leaf 256, tol 1e-4, rank <= 256, HSS, W: N x 1024 FP64
    (the reported line), and the N = 65536, d = 8, Q = 256 distance-admissible
    workload beside it.  Split BF16 against the plain FP64 and FP32 paths on
    the same matrix, with its error against the FP64 result."""
    import workloads as wl
    if args.mixed_c2_only:  # the N = 65536 workload alone (for the profiles of its launch)
        main_run, also = _mixed_one(args, wl.C2, f"distance tau={wl.C2.tau}", "gaussian"), None
    else:
        main_run = _mixed_one(args, wl.C4, "HSS", "exp(-r/h)")
        also = _mixed_one(args, wl.C2, f"distance tau={wl.C2.tau}", "gaussian") if args.mixed_both else None
    main_run.pop("_cols", None)
    if also:
        also.pop("_cols", None)
    m = main_run["paths"]["bf16x3"]
    return {
        "metric": "mixed-precision K~W GFLOP/s (algorithmic) vs the plain FP64 path",
        "value": m["gflops"], "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["ms_per_step"], "higher_is_better": True,
        "dtype": "bf16x3+f64", "data": "synthetic", **main_run,
        "also": also,
    }


def bench_h2b(args) -> dict:
    """The headline points (N = 65536, d = 8, Q = 256) under the paper's
    structure for high-dimensional data: two-means tree (Section 3.1) and
    budget admissibility 0.03, "H^2-b" (Section 4.1).  Built by inspector-p1
    (host) and inspector-p2 on the GPU; FP64 and split BF16, with eps_f on
    256 sampled rows against the exact product."""
    import numpy as np
    import torch

    import paper_1812_07152_amd as hmx
    import workloads as wl
    from oracle.oracle import exact_rows

    w = wl.C2B
    X = wl.gen_points(w)
    t = time.perf_counter()
    S = hmx.hm_inspect_p1(X, leaf_size=w.m, admissibility=w.adm, tau=w.tau, sample_rows=w.sample_rows,
                          seed=w.sample_seed, partitioner=w.part, budget=w.budget)
    t_p1 = time.perf_counter() - t
    t = time.perf_counter()
    M = hmx.hm_inspect_p2_load(S, 0, kernel=w.kernel, h=w.h, tol=w.tol, max_rank=w.rmax,
                               prec_mask=hmx.precbit(hmx.HM_PREC_FP64) | hmx.precbit(hmx.HM_PREC_BF16X3))
    torch.cuda.synchronize()
    t_p2 = time.perf_counter() - t
    info = hmx.hm_info(M)
    flops = info["flops_per_col"] * w.Q
    W = torch.from_numpy(wl.gen_w(w)).cuda()
    ms64, ph64, n64, Y64 = time_variant(hmx, torch, M, W, args.steps, args.warmup)
    msm, phm, nm, Ym = time_variant(hmx, torch, M, W, args.steps, args.warmup, prec=hmx.HM_PREC_BF16X3)
    graph_ms = ph64[3] / max(n64[3], 1)
    rows = np.random.default_rng(12).choice(w.N, 256, replace=False)
    cols = np.arange(16)
    Yex = exact_rows(X, w.kernel, w.h, rows, W[:, cols].cpu().numpy())

    def eps(Y):
        Ys = Y[:, :16].cpu().numpy()[rows]
        return float(np.linalg.norm(Ys - Yex) / np.linalg.norm(Yex))

    return {
        "metric": "K~W GFLOP/s (algorithmic), H^2-b structure", "value": flops / (ms64 * 1e-3) / 1e9,
        "unit": "GFLOP/s", "ms_per_step": ms64, "dtype": "f64",
        "config": {"workload": w.name, "N": w.N, "d": w.d, "Q": w.Q, "partitioner": "two-means",
                   "admissibility": f"budget {w.budget}", "leaf": w.m, "tol": w.tol, "max_rank": w.rmax,
                   "n_near_pairs": info["n_near"], "n_far_pairs": info["n_far"], "gflop_per_step": flops / 1e9,
                   "E_V": info["E_V"], "E_T": info["E_T"], "E_B": info["E_B"], "E_D": info["E_D"]},
        "roofline": {"bound": "mfma", "kernel": "k_persistent<double,...> (task-graph launch)",
                     "achieved": flops / (graph_ms * 1e-3) / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": flops / (graph_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, "launch_ms": graph_ms},
        "mixed_bf16x3": {"ms_per_step": msm, "value": flops / (msm * 1e-3) / 1e9, "speedup_vs_fp64": ms64 / msm,
                         "rel_err_vs_gpu_fp64": float(torch.linalg.norm(Ym - Y64) / torch.linalg.norm(Y64))},
        "eps_f_sampled": {"fp64": eps(Y64), "mixed_bf16x3": eps(Ym), "rows": 256, "columns": 16},
        "setup_s": {"p1_host": t_p1, "p2_gpu_and_store": t_p2},
    }


def bench_compression(args) -> dict:
    """Reusing inspection (paper Section 5, its Fig. 10 scenario): the headline
    workload (N = 65536, d = 8) compressed for five accuracies 1e-1 ... 1e-5.
    Without reuse every change reruns the whole compression; with reuse
    inspector-p1 (tree, interaction lists, row samples; host) runs once and
    only inspector-p2 (IDs on the GPU, blocks generated in the device store)
    runs per accuracy.  Beside it, the host inspector (the same readings, all
    host cores) followed by the upload, per accuracy.  Every time includes
    building the device matrix that the evaluation uses."""
    import numpy as np
    import torch

    import paper_1812_07152_amd as hmx
    import workloads as wl
    from oracle.oracle import exact_rows

    w = wl.C2
    X = wl.gen_points(w)
    tols = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5)
    mask = hmx.precbit(hmx.HM_PREC_FP64)
    t = time.perf_counter()
    S = hmx.hm_inspect_p1(X, leaf_size=w.m, admissibility=w.adm, tau=w.tau, sample_rows=w.sample_rows,
                          seed=w.sample_seed)
    t_p1 = time.perf_counter() - t
    W = torch.from_numpy(wl.gen_w(w, Q=8)).cuda()
    rows = np.random.default_rng(11).choice(w.N, 256, replace=False)
    Yex = exact_rows(X, w.kernel, w.h, rows, W.cpu().numpy())
    per = []
    for tol in tols:
        torch.cuda.synchronize()
        t = time.perf_counter()
        M = hmx.hm_inspect_p2_load(S, 0, kernel=w.kernel, h=w.h, tol=tol, max_rank=w.rmax, prec_mask=mask)
        torch.cuda.synchronize()
        t_p2 = time.perf_counter() - t
        # the IDs alone (no blocks in the store)
        t = time.perf_counter()
        M0 = hmx.hm_inspect_p2_load(S, 0, kernel=w.kernel, h=w.h, tol=tol, max_rank=w.rmax,
                                    prec_mask=mask | hmx.HM_LOAD_NO_NEAR_BLOCKS | hmx.HM_LOAD_NO_FAR_BLOCKS)
        torch.cuda.synchronize()
        t_ids = time.perf_counter() - t
        del M0
        Y = torch.empty_like(W)
        hmx.hm_eval(M, W, Y)
        hmx.hm_check(M)
        e = float(np.linalg.norm(Y.cpu().numpy()[rows] - Yex) / np.linalg.norm(Yex))
        info = hmx.hm_info(M)
        del M
        t = time.perf_counter()
        R = hmx.hm_compress(X, kernel=w.kernel, h=w.h, leaf_size=w.m, tol=tol, max_rank=w.rmax,
                            admissibility=w.adm, tau=w.tau, sample_rows=w.sample_rows, seed=w.sample_seed)
        t_host = time.perf_counter() - t
        t = time.perf_counter()
        Mh = hmx.hm_load_compressed_mem(R, 0, mask)
        torch.cuda.synchronize()
        t_load = time.perf_counter() - t
        del Mh, R
        per.append({"tol": tol, "p2_gpu_s": t_p2, "p2_ids_only_s": t_ids, "host_compress_s": t_host,
                    "host_upload_s": t_load, "eps_f_sampled": e, "gflop_per_column": info["flops_per_col"] / 1e9})
        print(f"[compression] tol={tol:g}: p2 {t_p2:.2f} s (IDs {t_ids:.2f} s), host {t_host:.2f} + "
              f"{t_load:.2f} s, eps_f {e:.2e}", file=sys.stderr, flush=True)
    reuse = t_p1 + sum(p["p2_gpu_s"] for p in per)
    no_reuse = sum(t_p1 + p["p2_gpu_s"] for p in per)
    host = sum(p["host_compress_s"] + p["host_upload_s"] for p in per)
    return {
        "metric": "compression time over five accuracy changes (s), inspector-p1 reused",
        "value": reuse, "unit": "s", "higher_is_better": False, "dtype": "f64",
        "config": {"workload": w.name, "N": w.N, "d": w.d, "tols": list(tols), "leaf": w.m,
                   "max_rank": w.rmax, "sample_rows": w.sample_rows},
        "p1_host_s": t_p1, "per_accuracy": per,
        "total_s": {"gpu_p2_with_p1_reuse": reuse, "gpu_without_reuse": no_reuse,
                    "host_inspector_and_upload": host},
        "speedup_reuse_vs_host": host / reuse,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the split-BF16 step on the headline workload")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched, served and N=262144 mixed-precision forms after the headline")
    ap.add_argument("--no-c4", action="store_true", help="skip the N=262144 mixed-precision form")
    ap.add_argument("--no-symmetric", dest="symmetric", action="store_false",
                    help="skip the symmetric-store variant of the headline step")
    ap.add_argument("--no-near-from-points", dest="near_from_points", action="store_false",
                    help="skip the matrix-free near-field variant of the FP64 step")
    ap.add_argument("--mixed-c4-only", dest="mixed_both", action="store_false",
                    help="mixed form: skip the N=65536 workload reported beside the main one")
    ap.add_argument("--mixed-c2-only", action="store_true",
                    help="mixed form: run the N=65536 workload alone")
    ap.add_argument("--form", choices=("plain", "batched", "serving", "mixed", "points", "compression", "h2b"),
                    default="plain",
                    help="plain: the headline workload; batched: 64 uneven matrices in one launch; "
                         "serving: 8 resident matrices under a request stream; mixed: split BF16; "
                         "points: near and far blocks computed from the points; compression: "
                         "inspector-p1 reuse over five accuracy changes")
    ap.add_argument("--burst", type=int, default=128, help="serving: requests in the saturation burst")
    ap.add_argument("--serving-seconds", type=float, default=3.0, help="serving: seconds per load level")
    ap.add_argument("--serving-seed", type=int, default=4)
    ap.add_argument("--serving-slots", type=int, default=4, help="serving: concurrent sweeps (slots)")
    ap.add_argument("--serving-symmetric", action="store_true", help="serving: symmetric stores")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (a kernel of "
                         "known traffic for calibrating HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(on several GPUs the path would shard by columns of W, with no exchange between them)",
              file=sys.stderr)
        return 2

    if args.form == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return 0
    if args.form == "serving":
        print(json.dumps(bench_serving(args)), flush=True)
        return 0
    if args.form == "mixed":
        print(json.dumps(bench_mixed(args)), flush=True)
        return 0
    if args.form == "points":
        print(json.dumps(bench_points(args)), flush=True)
        return 0
    if args.form == "compression":
        print(json.dumps(bench_compression(args)), flush=True)
        return 0
    if args.form == "h2b":
        print(json.dumps(bench_h2b(args)), flush=True)
        return 0

    import numpy as np
    import torch

    import paper_1812_07152_amd as hmx
    import workloads as wl

    w = wl.C2
    X = wl.gen_points(w)
    Wn = wl.gen_w(w)
    t = time.perf_counter()
    R = hmx.hm_compress(X, kernel=w.kernel, h=w.h, leaf_size=w.m, tol=w.tol, max_rank=w.rmax,
                        admissibility=w.adm, tau=w.tau, sample_rows=w.sample_rows, seed=w.sample_seed)
    t_compress = time.perf_counter() - t
    precs = (hmx.precbit(hmx.HM_PREC_FP64) | (0 if args.no_fp32 else hmx.precbit(hmx.HM_PREC_FP32))
             | (0 if args.no_mixed else hmx.precbit(hmx.HM_PREC_BF16X3)))
    t = time.perf_counter()
    M = hmx.hm_load_compressed_mem(R, 0, precs)
    t_load = time.perf_counter() - t
    info = hmx.hm_info(M)
    if not (args.near_from_points or args.symmetric):
        del R
    flops = info["flops_per_col"] * w.Q
    W64 = torch.from_numpy(Wn).to("cuda", torch.float64)
    results = {}  # GPU results on the host, compared with the oracle at the end

    ms64, ph64, n64, Y = time_variant(hmx, torch, M, W64, args.steps, args.warmup)
    results["fp64"] = Y.cpu().numpy()
    # the dominant kernel: the persistent task-graph launch, which runs every
    # block product of the step (everything but the two permutes)
    graph_ms = ph64[3] / max(n64[3], 1)
    achieved = flops / (graph_ms * 1e-3) / 1e12
    traffic = measured_traffic("task_graph_c2_fp64")

    out = {
        "metric": "K~W GFLOP/s (algorithmic) and % of FP64 roofline",
        "value": flops / (ms64 * 1e-3) / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Gaussian-mixture points and normal W; no dataset)",
        "config": {"workload": w.name, "N": w.N, "d": w.d, "Q": w.Q, "kernel": "gaussian",
                   "h": w.h, "leaf": w.m, "tol": w.tol, "max_rank": w.rmax,
                   "admissibility": f"distance tau={w.tau}", "n_near_pairs": info["n_near"],
                   "n_far_pairs": info["n_far"], "gflop_per_step": flops / 1e9},
        "roofline": {"bound": "mfma", "kernel": "k_persistent<double,256> (task-graph launch: up, down, "
                                                  "near field, leaf far part)",
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "launch_ms": graph_ms, "algorithmic_gflop_per_launch": flops / 1e9,
                     "counters": measured_counters("task_graph_counters_c2_fp64")},
        "whole_step_frac_of_fp64_peak": flops / (ms64 * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
        "phase_ms": {k: ph64[i] / max(n64[i], 1) for i, k in
                     enumerate(("permute_in", "up", "down", "graph", "permute_out")) if n64[i]},
        "setup_s": {"compress": t_compress, "load": t_load},
        "store_gb_fp64": info["bytes_fp64"] / 1e9,
    }
    if not args.no_fp32:
        ms32, ph32, n32, Y = time_variant(hmx, torch, M, W64.float(), args.steps, args.warmup)
        results["fp32"] = Y.double().cpu().numpy()
        out["fp32"] = {"ms_per_step": ms32, "value": flops / (ms32 * 1e-3) / 1e9, "unit": "GFLOP/s",
                       "frac_of_fp32_peak": flops / (ms32 * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}
    if not args.no_mixed:
        # the mixed-precision form on the same matrix: split-BF16 near, far
        # and leaf-basis products, FP64 transfers and final sum
        msm, phm, nm, Y = time_variant(hmx, torch, M, W64, args.steps, args.warmup, prec=hmx.HM_PREC_BF16X3)
        results["mixed_bf16x3"] = Y.cpu().numpy()
        launch_m = phm[3] / max(nm[3], 1)
        out["mixed_bf16x3"] = {
            "ms_per_step": msm, "value": flops / (msm * 1e-3) / 1e9, "unit": "GFLOP/s",
            "launch_ms": launch_m, "speedup_vs_fp64": ms64 / msm,
            "rel_err_vs_gpu_fp64": float(np.linalg.norm(results["mixed_bf16x3"] - results["fp64"])
                                         / np.linalg.norm(results["fp64"]))}
        # the split-BF16 launch against both of its ceilings: its profiled
        # memory-fabric bytes (HBM and Infinity Cache reads, the committed
        # counter summary of the current kernel source) over the launch
        # time, and its BF16 MFMA work (three products per stored product)
        traffic_m = measured_traffic("task_graph_c2_mixed")
        bf16_tflops = 3 * flops / (launch_m * 1e-3) / 1e12
        out["mixed_bf16x3"]["roofline"] = {
            "bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBPS, "traffic": traffic_m,
            "achieved": traffic_m / (launch_m * 1e-3) / 1e9 if traffic_m else None,
            "frac": traffic_m / (launch_m * 1e-3) / 1e9 / PEAK_HBM_GBPS if traffic_m else None,
            "mfma_bf16": {"achieved": bf16_tflops, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                          "frac": bf16_tflops / PEAK_BF16_TFLOPS}}
    if args.symmetric:
        # symmetric store: each far and near block of a pair stored once, the
        # mirror product reading it transposed (same results bitwise)
        t = time.perf_counter()
        Ms = hmx.hm_load_compressed_mem(R, 0, precs | hmx.HM_LOAD_SYMMETRIC)
        t_sload = time.perf_counter() - t
        sinfo = hmx.hm_info(Ms)
        sym = {"store_gb_fp64": sinfo["bytes_fp64"] / 1e9, "store_gb_fp32": sinfo["bytes_fp32"] / 1e9,
               "load_s": t_sload}
        mss, phs, nss, Ys = time_variant(hmx, torch, Ms, W64, args.steps, args.warmup)
        sym["fp64"] = {"ms_per_step": mss, "value": flops / (mss * 1e-3) / 1e9, "launch_ms": phs[3] / max(nss[3], 1),
                       "speedup_vs_full_store": ms64 / mss,
                       "bitwise_equal_to_full_store": bool(np.array_equal(Ys.cpu().numpy(), results["fp64"]))}
        if not args.no_fp32:
            ms32s, _, _, _ = time_variant(hmx, torch, Ms, W64.float(), args.steps, args.warmup)
            sym["fp32"] = {"ms_per_step": ms32s, "speedup_vs_full_store": out["fp32"]["ms_per_step"] / ms32s}
        if not args.no_mixed:
            msms, _, _, _ = time_variant(hmx, torch, Ms, W64, args.steps, args.warmup, prec=hmx.HM_PREC_BF16X3)
            sym["mixed_bf16x3"] = {"ms_per_step": msms,
                                   "speedup_vs_full_store": out["mixed_bf16x3"]["ms_per_step"] / msms}
        out["symmetric_store"] = sym
        del Ms
    if args.near_from_points:
        # matrix-free near field: the same FP64 step with every near block
        # computed from the points in the product tiles (stored blocks unread)
        hmx.hm_set_points(M, X, w.kernel, w.h)
        msp, php, npp, Yp = time_variant(hmx, torch, M, W64, args.steps, args.warmup,
                                         flags=hmx.HM_NEAR_FROM_POINTS)
        results["near_from_points"] = Yp.cpu().numpy()
        out["near_from_points"] = {
            "ms_per_step": msp, "value": flops / (msp * 1e-3) / 1e9, "unit": "GFLOP/s",
            "launch_ms": php[3] / max(npp[3], 1),
            "near_block_bytes_not_read": info["E_D"] * 8,
            "rel_diff_vs_stored": float(np.linalg.norm(results["near_from_points"] - results["fp64"])
                                        / np.linalg.norm(results["fp64"]))}
        del M
        # the same matrix loaded without its near and far blocks (both
        # computed from the points and the skeletons): the store's HBM
        M3 = hmx.hm_load_compressed_mem(R, 0, hmx.precbit(hmx.HM_PREC_FP64) | hmx.HM_LOAD_NO_NEAR_BLOCKS
                                        | hmx.HM_LOAD_NO_FAR_BLOCKS)
        del R
        both = hmx.HM_NEAR_FROM_POINTS | hmx.HM_FAR_FROM_POINTS
        hmx.hm_set_points(M3, X, w.kernel, w.h)
        ms3, ph3, n3, Y3 = time_variant(hmx, torch, M3, W64, args.steps, args.warmup, flags=both)
        results["near_and_far_from_points"] = Y3.cpu().numpy()
        out["near_from_points"]["far_too"] = {
            "ms_per_step": ms3, "value": flops / (ms3 * 1e-3) / 1e9, "unit": "GFLOP/s",
            "launch_ms": ph3[3] / max(n3[3], 1),
            "far_block_bytes_not_read": info["E_B"] * 8,
            "store_gb_without_near_and_far_blocks": hmx.hm_info(M3)["bytes_fp64"] / 1e9,
            "rel_diff_vs_stored": float(np.linalg.norm(results["near_and_far_from_points"] - results["fp64"])
                                        / np.linalg.norm(results["fp64"]))}
        del M3, Y3, Yp
    else:
        del M
    del Y, W64
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8}
        del src, dst
    if not args.no_cpu_baseline:
        base, ref = cpu_baseline(w, X, Wn)
        out["cpu_baseline"] = base
        # every GPU result of this workload against the oracle, on the
        # oracle's sampled columns and rows
        out["accuracy_vs_oracle"] = {"columns": ref["cols"], "rows_for_eps_f": len(ref["rows"]),
                                     "eps_f_sampled_oracle": base["eps_f_sampled_oracle"],
                                     **{k: errors_vs_oracle(v, ref) for k, v in results.items()}}
        out["eps_f_sampled"] = out["accuracy_vs_oracle"]["fp64"]["eps_f_sampled"]
    del results
    if not args.no_forms:
        # the three forms beside the plain kernel, each on its own workload
        out["forms"] = {}
        t = time.perf_counter()
        out["forms"]["batched"] = compact(bench_batched(args))
        print(f"[bench] batched form done ({time.perf_counter() - t:.0f} s)", file=sys.stderr, flush=True)
        t = time.perf_counter()
        out["forms"]["served"] = compact(bench_serving(args))
        print(f"[bench] served form done ({time.perf_counter() - t:.0f} s)", file=sys.stderr, flush=True)
        if not args.no_c4:
            t = time.perf_counter()
            out["forms"]["mixed_c4"] = compact(bench_mixed_c4(args))
            print(f"[bench] mixed C4 form done ({time.perf_counter() - t:.0f} s)", file=sys.stderr, flush=True)
        t = time.perf_counter()
        out["forms"]["h2b_structure"] = compact(bench_h2b(args))
        print(f"[bench] H^2-b structure done ({time.perf_counter() - t:.0f} s)", file=sys.stderr, flush=True)
        t = time.perf_counter()
        out["forms"]["compression_reuse"] = compact(bench_compression(args))
        print(f"[bench] compression reuse done ({time.perf_counter() - t:.0f} s)", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)
    return 0


def compact(d: dict) -> dict:
    """A form's JSON line without the keys the headline line already has."""
    drop = ("n_gpus", "steps", "warmup", "higher_is_better", "data", "scaling", "vs_baseline")
    return {k: v for k, v in d.items() if k not in drop}


if __name__ == "__main__":
    sys.exit(main())
