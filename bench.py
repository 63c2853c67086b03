#!/usr/bin/env python3
"""Benchmark of the randomized SVD hot path on one MI355X.

One step = one rsvd_factor call: Gaussian test matrix, sketch, q power steps
with CholeskyQR2 re-orthonormalisation, projection, FP64 small SVD, lift
(Figure 5 of Martinsson's "Randomized methods for matrix computations" plus
Stage B of Section 3), on the 50000 x 20000 float32 workload (rank 2000,
sigma_j = j^-0.5, noise 1e-3 sigma_1/sqrt(n), k=100, p=10, q=2) resident in
HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-ε and TFLOP/s for rank-k RSVD; BF16/FP8+learned vs plain FP32"
MI355X_PEAK = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "fp8": 5000.0}   # dense MFMA TFLOP/s
HBM_PEAK_GBS = 8000.0
ELT_BYTES = {"f32": 4, "f64": 8, "bf16": 2, "fp8": 1}
# HBM traffic of the dominant product kernel, per launch, from rocprofv3 FETCH_SIZE / WRITE_SIZE passes scaled by a
# plain copy kernel (see traffic_summary); used only while the kernel source is the one the counters were taken on
TRAFFIC_FILES = {("bf16", "slowdecay_50000x20000"): "profiles/traffic_lp_nn_bf16_slowdecay_50000x20000.md",
                 ("fp8", "expdecay_65536"): "profiles/traffic_lp_nn_fp8_expdecay_65536.md"}
TRAFFIC_SOURCE = "paper_1607_01649_amd/csrc/lpgemm.hip"
# time-to-eps target per workload: eps = factor * sigma_{k+1} (spectral norm of the residual)
EPS_FACTOR = {"slowdecay_50000x20000": 1.15, "expdecay_65536": 1.10, "plain_f64_2000": 1.15}


def _sha256(path):
    import hashlib
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_per_launch(sketch, workload):
    """HBM bytes per launch of the product kernel from the committed counter summary, or None when there is none
    or the kernel source changed since it was taken."""
    rel = TRAFFIC_FILES.get((sketch, workload))
    if not rel or not os.path.exists(os.path.join(ROOT, rel)):
        return None
    with open(os.path.join(ROOT, rel)) as f:
        for line in f:
            if line.startswith("traffic-json: "):
                d = json.loads(line[len("traffic-json: "):])
                if d.get("source_sha256") == _sha256(TRAFFIC_SOURCE):
                    return d["bytes_per_launch"]
    return None


def traffic_summary(fetch_dir, write_dir, calib_bytes, sketch, workload, kernel_prefix="rsvd::lp_nn_kernel"):
    """Summarise two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of the `sketch` path
    on `workload` into its file under profiles/.  Each counter is scaled by calib_bytes / counter of the first
    dispatch that moves a sizeable share of them: --copy-calibration issues, before anything else, a fill (writes
    calib_bytes) and an elementwise copy (reads and writes them)."""
    import csv
    from workloads import gen

    def load(d, counter):
        path = os.path.join(d, "run_counter_collection.csv")
        vals = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            key = (r["Kernel_Name"], int(r["Dispatch_Id"]))
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"]) * 1024.0
        return vals

    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        vals = load(d, counter)
        first = sorted((disp, v) for (name, disp), v in vals.items() if v > calib_bytes / 16)
        if not first:
            raise SystemExit(f"no calibration dispatch among the {counter} dispatches")
        scale = calib_bytes / first[0][1]
        mine = [v for (name, _), v in vals.items() if name.startswith("void " + kernel_prefix) or
                name.startswith(kernel_prefix)]
        out[counter] = {"scale": scale, "launches": len(mine), "raw_bytes_per_launch": sum(mine) / len(mine),
                        "bytes_per_launch": scale * sum(mine) / len(mine)}
    tot = out["FETCH_SIZE"]["bytes_per_launch"] + out["WRITE_SIZE"]["bytes_per_launch"]
    cfg = gen.config(workload)
    alg = cfg.m * cfg.n * ELT_BYTES[sketch] + (cfg.m + cfg.n) * (cfg.k + cfg.p) * 4
    rec = {"kernel": kernel_prefix, "source_sha256": _sha256(TRAFFIC_SOURCE), "bytes_per_launch": tot,
           "fetch": out["FETCH_SIZE"], "write": out["WRITE_SIZE"], "calibration_copy_bytes": calib_bytes}
    run = (f"python -u bench.py --workload {workload} --paths {sketch} --steps 1 --warmup 0 --no-cpu --also '' "
           f"--copy-calibration {calib_bytes}" + (" --matrix randn" if workload != "slowdecay_50000x20000" else ""))
    lines = [f"# HBM traffic of `{kernel_prefix}` ({sketch} products), {cfg.m} x {cfg.n} workload ({workload})", "",
             "Two rocprofv3 counter passes over the same bench command (repository root, MI355X), each counter",
             "scaled by what it reads for a plain copy of a known size (an elementwise torch kernel, `--copy-calibration`):",
             "", "    rocprofv3 --pmc FETCH_SIZE --kernel-include-regex 'lp_nn|Functor' -d gpurun_out/pmc_fetch -o run "
             "--output-format csv -- " + run,
             "    rocprofv3 --pmc WRITE_SIZE --kernel-include-regex 'lp_nn|Functor' -d gpurun_out/pmc_write -o run "
             "--output-format csv -- " + run,
             f"    python bench.py --summarize-traffic gpurun_out/pmc_fetch gpurun_out/pmc_write {calib_bytes} "
             f"--traffic-key {sketch}:{workload}", "",
             "| counter | copy scale | launches | bytes per launch (scaled) |", "|---|---|---|---|"]
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        lines.append(f"| {c} | {out[c]['scale']:.4f} | {out[c]['launches']} | {out[c]['bytes_per_launch'] / 1e9:.3f} GB |")
    lines += ["", f"Total per launch: {tot / 1e9:.3f} GB (algorithmic: {alg / 1e9:.3f} GB; A in {sketch} once, the "
              f"FP32 thin operand and result; ratio {tot / alg:.2f}).",
              "bench.py reports it as `roofline.traffic` while the kernel source hash matches.", "",
              "traffic-json: " + json.dumps(rec)]
    out_path = os.path.join(ROOT, TRAFFIC_FILES[(sketch, workload)])
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[-6:]))


def spectral_residual(A, U, S, V, iters=40, seed=0):
    """||A - U diag(S) V^T||_2 by power iteration (harness-side torch, untimed)."""
    import torch
    g = torch.Generator(device=A.device)
    g.manual_seed(seed)
    x = torch.randn(A.shape[1], 1, generator=g, device=A.device, dtype=torch.float64)
    Ad = A
    Ud, Sd, Vd = U.double(), S.double(), V.double()

    def fwd(v):
        return (Ad @ v.float()).double() - Ud @ (Sd[:, None] * (Vd.T @ v))

    def adj(w):
        return (Ad.T @ w.float()).double() - Vd @ (Sd[:, None] * (Ud.T @ w))
    est = 0.0
    for _ in range(iters):
        x = x / torch.linalg.norm(x)
        y = fwd(x)
        x = adj(y)
        est = math.sqrt(float(torch.linalg.norm(x)))
    return est


def host_cpu():
    """CPU model, physical cores (distinct (package, core) pairs) and the CPUs this process may run on."""
    model, cores = "unknown", set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model == "unknown":
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except Exception:
        allowed = os.cpu_count() or 1
    return {"cpu_model": model, "physical_cores": len(cores) or None, "cpus_allowed": allowed}


def cpu_baseline(A_gpu, k, p, q, rows, seed, min_seconds=10.0, max_runs=20):
    """The FP64 numpy oracle (Figure 5 + Stage B, untuned) on a bounded row
    sample of the same matrix with the same Omega, repeated until about
    min_seconds of CPU work.  Returns the baseline record and the oracle's
    rank-k result (for the per-path comparison when the sample is all rows)."""
    from oracle import rsvd as orc
    from oracle import philox
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    rows = min(rows, A_gpu.shape[0])
    A = A_gpu[:rows].double().cpu().numpy()
    n = A.shape[1]
    G = philox.gaussian(n, k + p, seed, philox.STREAM_OMEGA)
    runs, tot = 0, 0.0
    res = None
    while runs < max_runs and (runs == 0 or tot < min_seconds):
        t0 = time.perf_counter()
        res = orc.rsvd(A, G, q).truncate(k)
        tot += time.perf_counter() - t0
        runs += 1
    dt = tot / runs
    flops = 2.0 * rows * n * (k + p) * (2 * q + 2)
    rec = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
           "sample": f"oracle (numpy float64, Figure 5 + Stage B) on the first {rows} of {A_gpu.shape[0]} rows, "
                     f"same n, k, p, q and Omega; {runs} run(s), {tot:.1f} s in total, {dt:.2f} s per run; "
                     f"flops counted as 2*rows*n*l*(2q+2)"}
    rec.update(host_cpu())
    return rec, (res if rows == A_gpu.shape[0] else None)


def vs_oracle(ref, S, U):
    """Error of one path's rank-k result against the FP64 oracle's on the same A and Omega: largest relative
    singular-value error, and the sine of the largest principal angle between the left subspaces."""
    Sg = np.asarray(S, dtype=np.float64)
    rel = np.abs(Sg - ref.D) / ref.D
    M = ref.U.T @ np.asarray(U, dtype=np.float64)
    cmin = float(np.linalg.svd(M, compute_uv=False).min())
    return {"sigma_rel_err_max": float(rel.max()), "sigma_rel_err_at_k": float(rel[-1]),
            "sin_theta_U": math.sqrt(max(0.0, 1.0 - min(cmin, 1.0) ** 2))}


def vs_planted(sig, S):
    """Singular values of a noise-free planted matrix against the planted ones (their exact values up to the
    float32 rounding of A): largest error relative to sigma_j and to sigma_1."""
    Sg = np.asarray(S, dtype=np.float64)
    s = np.asarray(sig[:len(Sg)], dtype=np.float64)
    return {"sigma_rel_err_max": float((np.abs(Sg - s) / s).max()),
            "sigma_err_max_over_sigma1": float(np.abs(Sg - s).max() / s[0])}


def run_path(A, cfg, sketch, proj, steps, warmup, seed, keep_u=True, flags=0):
    """Time `steps` factorisations with the given operand precisions; returns
    the measurements and the last factors."""
    import torch
    from paper_1607_01649_amd import RSVD, RSVD_TIMING
    m, n, k, p, q = cfg.m, cfg.n, cfg.k, cfg.p, cfg.q
    l = k + p
    solver = RSVD(m, n, k, p, q, dtype=cfg.dtype, device=A.device, seed=seed, flags=RSVD_TIMING | flags,
                  sketch_dtype=sketch, proj_dtype=proj)
    for _ in range(warmup):
        U, S, V, info = solver(A)
    torch.cuda.synchronize()
    nn_ms = tn_ms = 0.0
    nn_n = tn_n = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        U, S, V, info = solver(A)
        nn_ms += info.nn_ms
        tn_ms += info.tn_ms
        nn_n += info.nn_launches
        tn_n += info.tn_launches
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    if info.status != 0:
        raise SystemExit(f"rsvd_factor status {info.status}")
    flops_pass = 2.0 * m * n * l
    passes = 2 * q + 2
    avg_nn = nn_ms / max(nn_n, 1) * 1e-3
    avg_tn = tn_ms / max(tn_n, 1) * 1e-3
    # column tiles of 16 per workgroup of the low-precision product: bf16 at most 7; FP8 an even count <= 12,
    # the fewest column groups first
    nt = (l + 15) // 16
    if sketch == "bf16":
        lp_nb = min(7, nt)
    else:
        groups = (nt + 11) // 12
        lp_nb = ((nt + groups - 1) // groups + 1) // 2 * 2
    names = {"f32": ("nn_pipe_kernel (Y = A X, FP32 MFMA)", "tn_pipe_kernel (Z = A^T Q, FP32 MFMA)"),
             "f64": ("nn_kernel (Y = A X, FP64 MFMA)", "tn_kernel (Z = A^T Q, FP64 MFMA)"),
             "bf16": ("lp_nn_kernel<0,%d,4,1,true> (Y = bf16(A) X)" % lp_nb, "lp_nn_kernel<0,%d,4,1,true> (Z = bf16(A)^T Q)" % lp_nb),
             "fp8": ("lp_nn_kernel<1,%d,4,1,true> (Y = fp8(A) X)" % lp_nb, "lp_nn_kernel<1,%d,4,1,true> (Z = fp8(A)^T Q)" % lp_nb)}[sketch]
    dom_nn = nn_ms >= tn_ms
    avg = avg_nn if dom_nn else avg_tn
    # algorithmic bytes of one product: A once in its operand format, the thin FP32 operand and result
    bytes_launch = m * n * ELT_BYTES[sketch] + (m + n) * l * 4
    intensity = flops_pass / bytes_launch
    ridge = MI355X_PEAK[sketch] * 1e12 / (HBM_PEAK_GBS * 1e9)
    if intensity >= ridge:
        achieved = flops_pass / avg / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": MI355X_PEAK[sketch], "unit": "TFLOP/s",
                "frac": achieved / MI355X_PEAK[sketch], "achieved_gbs": bytes_launch / avg / 1e9}
    else:
        achieved = bytes_launch / avg / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "achieved_tflops": flops_pass / avg / 1e12}
    roof.update({"algorithmic_bytes_per_launch": bytes_launch, "flops_per_launch": flops_pass,
                 "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge})
    roof.update({"traffic": traffic_per_launch(sketch, cfg.name), "kernel": names[0] if dom_nn else names[1],
                 "avg_launch_ms": avg * 1e3,
                 "launches_per_step": (nn_n + tn_n) / steps,
                 "other_kernel": None if min(nn_n, tn_n) == 0 else
                 {"name": names[1] if dom_nn else names[0], "avg_launch_ms": (avg_tn if dom_nn else avg_nn) * 1e3,
                  "achieved_tflops": flops_pass / (avg_tn if dom_nn else avg_nn) / 1e12}})
    sig = cfg.sigma()
    fac = EPS_FACTOR.get(cfg.name, 1.15)
    eps_abs = fac * sig[k]
    err = spectral_residual(A, U, S, V)
    tte = {"eps": f"{fac}*sigma_{{k+1}}", "eps_abs": eps_abs, "achieved_err": err, "reached": bool(err <= eps_abs),
           "time_ms": dt * 1e3 if err <= eps_abs else None}
    S_host = S.double().cpu().numpy()
    U_host = U.double().cpu().numpy() if keep_u else None
    del solver, U, S, V
    torch.cuda.empty_cache()
    return {"_S": S_host, "_U": U_host, "sketch_dtype": sketch, "proj_dtype": proj, "ms_per_step": dt * 1e3,
            "tflops": flops_pass * passes / dt / 1e12, "stage_ms": [round(x, 4) for x in info.stage_ms],
            "jacobi_sweeps": info.jacobi_sweeps, "time_to_eps": tte, "roofline": roof}


def run_id_leg(A, cfg, kind, steps, warmup, seed):
    """Randomized row ID (Section 10.4) or CUR (Section 11) on the workload's matrix: time per call (HIP events
    on the plan's stream bracket the timed calls), the pivoted-QR share (RSVD_TIMING stage events) and the
    untimed spectral error of the result against sigma_{k+1}."""
    import torch
    from paper_1607_01649_amd import RSVD, RSVD_ID_CUR, RSVD_TIMING
    m, n, k, p, q = cfg.m, cfg.n, cfg.k, cfg.p, cfg.q
    solver = RSVD(m, n, k, p, q, dtype=cfg.dtype, device=A.device, seed=seed, flags=RSVD_ID_CUR | RSVD_TIMING)
    call = (lambda: solver.row_id(A)) if kind == "rowid" else (lambda: solver.cur(A))
    for _ in range(warmup):
        out = call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stage = np.zeros(8)
    for _ in range(steps):
        out = call()
        stage += np.array(out[-1].stage_ms)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    stage /= steps
    g = torch.Generator(device=A.device)
    g.manual_seed(0)
    x = torch.randn(n, 1, generator=g, device=A.device, dtype=torch.float64)
    if kind == "rowid":
        Is, X, _ = out
        R = A[Is.long()].double()
        fwd = lambda v: (A @ v.float()).double() - X.double() @ (R @ v)
        adj = lambda w: (A.T @ w.float()).double() - R.T @ (X.double().T @ w)
    else:
        Js, U, Is, _ = out
        C = A[:, Js.long()].double()
        R = A[Is.long()].double()
        fwd = lambda v: (A @ v.float()).double() - C @ (U @ (R @ v))
        adj = lambda w: (A.T @ w.float()).double() - R.T @ (U.T @ (C.T @ w))
    est = 0.0
    for _ in range(40):
        x = x / torch.linalg.norm(x)
        x = adj(fwd(x))
        est = math.sqrt(float(torch.linalg.norm(x)))
    sig = cfg.sigma()
    label = "randomized row ID (Section 10.4)" if kind == "rowid" else "randomized CUR (Section 11)"
    return {"method": label, "ms_per_step": dt * 1e3, "stage_ms": [round(float(v), 4) for v in stage],
            "stages": "sample (Stage A products), pivoted QR, solve / second pivoted QR, U, -, -, -, total",
            "spectral_error": est, "sigma_k+1": float(sig[k]), "error_over_sigma_k+1": est / float(sig[k]),
            "workload": cfg.name, "m": m, "n": n, "k": k, "p": p, "q": q, "steps": steps, "warmup": warmup}


def srht_roofline(A, l, seed, reps=10):
    """The structured sketch (Section 6) on its own: the library's kernel-level entry (draw and one-pass
    transform) timed with HIP events on the current stream; HBM-bound, algorithmic bytes = A once + Y."""
    import torch
    from paper_1607_01649_amd import rsvd_k_srht_sketch
    for _ in range(2):
        rsvd_k_srht_sketch(A, l, seed)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rsvd_k_srht_sketch(A, l, seed)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    m, n = A.shape
    nbytes = m * n * A.element_size() + m * l * A.element_size()
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": None, "kernel": "srht_sketch_kernel (Y = A D H S / sqrt(N), one pass)", "avg_launch_ms": ms,
            "algorithmic_bytes_per_launch": nbytes}


def run_batched(args):
    """Batched compression of 4096 kernel blocks (rows and columns uniform in
    [64, 512], K_ij = log|x_i - y_j|, boxes three units apart) to relative
    tolerance 1e-6 in one persistent launch replayed from a HIP graph."""
    import torch
    from paper_1607_01649_amd import Batched
    from workloads import gen
    dev = torch.device("cuda:0")
    nblk, eps = 4096, 1e-6
    ms, ns = gen.batched_blocks(nblk, args.seed)
    _, blocks = gen.kernel_blocks_device(ms, ns, args.seed, str(dev))
    torch.cuda.synchronize()
    bat = Batched(blocks, eps=eps, rank_cap=64, seed=args.seed, n_workgroups=args.batched_wg)
    s = torch.cuda.Stream(device=dev)
    bat.stream = s
    tiles, tune_ms = bat.autotune()      # untimed: per size class, the fastest MFMA tile shape
    print(f"autotuned tiles {tiles}: ms per class/variant {[[round(x, 3) for x in r] for r in tune_ms]}",
          file=sys.stderr, flush=True)
    bat.capture(s)
    for _ in range(args.warmup):
        bat.replay(s)
    s.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(args.steps):
        bat.replay(s)
    e1.record(s)
    s.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    ms_rep = e0.elapsed_time(e1) / args.steps
    elems = float((ms.astype(np.float64) * ns).sum())
    # algorithmic work of the fixed 16-column basis: Y = K [Omega | G_c] (26 columns) and
    # B^T = K^T Q (16 columns), FP64 arithmetic; two reads of every block
    flops = 2.0 * elems * (26 + 16)
    bytes_alg = 2.0 * elems * 4
    st = bat.status.cpu().numpy()
    rk = bat.rank.cpu().numpy()
    # untimed check: true relative spectral error of a sample of blocks
    g = np.random.default_rng(args.seed)
    sample = g.choice(nblk, size=min(64, nblk), replace=False)
    worst = 0.0
    for b in sample:
        U, S, V = bat.factors(int(b))
        K = blocks[b].double()
        R = K - (U.double() * S) @ V.double().T
        s1 = torch.linalg.matrix_norm(K, ord=2)
        worst = max(worst, float(torch.linalg.matrix_norm(R, ord=2) / s1))
    achieved = flops / (ms_rep * 1e-3) / 1e12
    out = {"metric": "batched compression to relative tolerance 1e-6 (blocks/s)", "value": nblk / (ms_rep * 1e-3),
           "unit": "blocks/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_rep,
           "wall_ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 data, f64 arithmetic", "data": "synthetic",
           "config": {"workload": "kernel_blocks_4096", "nblk": nblk, "rows_cols": "uniform [64, 512]", "eps": eps,
                      "elements": elems, "n_workgroups": args.batched_wg or "default (resident slots)",
                      "tiles": tiles},
           "roofline": {"bound": "alu", "achieved": achieved, "peak": MI355X_PEAK["f64"], "unit": "TFLOP/s",
                        "frac": achieved / MI355X_PEAK["f64"], "traffic": None, "kernel": "batched_kernel",
                        "hbm_gbs_algorithmic": bytes_alg / (ms_rep * 1e-3) / 1e9},
           "certified_frac": float((st == 0).mean()), "status_counts": {int(k): int(v) for k, v in
                                                                        zip(*np.unique(st, return_counts=True))},
           "rank_max": int(rk.max()), "rank_mean": float(rk.mean()), "true_rel_err_max_of_64": worst}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="slowdecay_50000x20000")
    ap.add_argument("--paths", default="bf16,f32,f32+srht",
                    help="comma list of operand formats, '+srht' for the structured first sketch; the first one is "
                         "the headline")
    ap.add_argument("--cpu-rows", type=int, default=1 << 30, help="row sample of the CPU oracle (default: all rows)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--also", default="expdecay_65536:fp8,psd_20000:f32+nystrom,slowdecay_50000x20000:bf16+singlepass,"
                                      "slowdecay_50000x20000:f32+rowid,slowdecay_50000x20000:f32+cur",
                    help="comma list of workload:sketch[/proj][+srht|+nystrom] legs timed after the headline "
                         "('' for none)")
    ap.add_argument("--leg-steps", type=int, default=5)
    ap.add_argument("--leg-warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--batched-wg", type=int, default=0, help="workgroups of the batched launch (0 = library default)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="bytes of one plain device copy issued first (scale of the traffic counters)")
    ap.add_argument("--summarize-traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "CALIB_BYTES"),
                    help="write the traffic summary of two rocprofv3 --pmc passes to profiles/ and exit")
    ap.add_argument("--traffic-key", default="bf16:slowdecay_50000x20000",
                    help="sketch:workload of the traffic summary")
    ap.add_argument("--matrix", choices=("planted", "randn"), default="planted",
                    help="randn: a seeded standard normal matrix of the workload's shape instead of its planted "
                         "spectrum (for counter runs: the product kernels' traffic depends on the shapes only)")
    args = ap.parse_args()
    if args.summarize_traffic:
        fd, wd, cb = args.summarize_traffic
        sk, _, wl = args.traffic_key.partition(":")
        traffic_summary(fd, wd, int(cb), sk, wl)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the factorisation runs on one GPU (its multi-GPU sharding is not implemented); "
                                   "--gpus must be 1"}))
        sys.exit(2)
    if args.workload == "kernel_blocks_4096":
        run_batched(args)
        return

    import torch
    from workloads import gen

    dev = torch.device("cuda:0")
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)   # an elementwise kernel that reads and writes calibration bytes once
        torch.cuda.synchronize()
        del src, dst
    cfg = gen.config(args.workload)
    if args.matrix == "randn":
        g = torch.Generator(device=dev)
        g.manual_seed(args.seed)
        A = torch.randn(cfg.m, cfg.n, generator=g, device=dev,
                        dtype=torch.float32 if cfg.dtype == "f32" else torch.float64)
    else:
        A = cfg.matrix(seed=args.seed, device=str(dev))
        A = A.to(torch.float32) if cfg.dtype == "f32" else A
    torch.cuda.synchronize()
    paths = [p for p in args.paths.split(",") if p]
    res = {}
    print(f"[bench] {args.workload}: matrix ready", file=sys.stderr, flush=True)
    from paper_1607_01649_amd import RSVD_NYSTROM, RSVD_SINGLE_PASS, RSVD_SINGLE_PASS_SYM, RSVD_SKETCH_SRHT
    variant_flags = {"": 0, "srht": RSVD_SKETCH_SRHT, "nystrom": RSVD_NYSTROM, "singlepass": RSVD_SINGLE_PASS,
                     "singlepass_sym": RSVD_SINGLE_PASS_SYM}
    for pth in paths:
        fmt, _, var = pth.partition("+")
        if var not in variant_flags:
            raise SystemExit(f"unknown path variant '{var}' (row ID and CUR run as --also legs)")
        cfg_p = dataclasses.replace(cfg, q=0) if var.startswith("singlepass") else cfg
        res[pth] = run_path(A, cfg_p, fmt, fmt, args.steps, args.warmup, args.seed, keep_u=not args.no_cpu,
                            flags=variant_flags[var])
        if var == "srht":
            res[pth]["sketch"] = "structured (Section 6: random signs, Walsh-Hadamard, subsampled columns)"
            res[pth]["srht_roofline"] = srht_roofline(A, cfg.k + cfg.p, args.seed)
        print(f"[bench] path {pth}: {res[pth]['ms_per_step']:.2f} ms per step", file=sys.stderr, flush=True)
    head = res[paths[0]]
    out = {"metric": METRIC, "value": head["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": paths[0], "data": "synthetic",
           "config": {"workload": args.workload, "m": cfg.m, "n": cfg.n, "k": cfg.k, "p": cfg.p, "q": cfg.q,
                      "sketch_dtype": paths[0], "proj_dtype": paths[0], "a_dtype": cfg.dtype},
           "time_to_eps": head["time_to_eps"], "roofline": head["roofline"], "paths": res}
    if not args.no_cpu:
        out["cpu_baseline"], ref = cpu_baseline(A, cfg.k, cfg.p, cfg.q, args.cpu_rows, args.seed)
        print("[bench] cpu oracle done", file=sys.stderr, flush=True)
        if ref is not None:
            for pth in paths:
                if "+" not in pth:
                    res[pth]["vs_fp64_oracle"] = vs_oracle(ref, res[pth]["_S"], res[pth]["_U"])
                elif pth.endswith("+srht"):
                    res[pth]["vs_fp64_oracle_gaussian_omega"] = vs_oracle(ref, res[pth]["_S"], res[pth]["_U"])
    if cfg.noise_std == 0.0 and args.matrix == "planted":
        for pth in paths:
            res[pth]["vs_planted_sigma"] = vs_planted(cfg.sigma(), res[pth]["_S"])
    for pth in paths:
        res[pth].pop("_S")
        res[pth].pop("_U")
    torch.cuda.empty_cache()

    def leg_matrix(c2):
        """The leg's matrix: the headline's when the workload is the same (no second generation)."""
        if c2.name == args.workload:
            return A
        M = c2.matrix(seed=args.seed, device=str(dev))
        return M.to(torch.float32) if c2.dtype == "f32" else M
    # further legs: other workloads and operand formats, each with its own roofline (not part of `value`)
    legs = {}
    for leg in [x for x in args.also.split(",") if x]:
        wl, _, fmt = leg.partition(":")
        fmt, _, var = fmt.partition("+")
        sk, _, pj = fmt.partition("/")
        pj = pj or sk
        c2 = gen.config(wl)
        if var.startswith("singlepass"):
            c2 = dataclasses.replace(c2, q=0)   # one pass over A: no power steps
        if var in ("rowid", "cur"):
            A2 = leg_matrix(c2)
            torch.cuda.synchronize()
            legs[leg] = run_id_leg(A2, c2, var, args.leg_steps, args.leg_warmup, args.seed)
            print(f"[bench] leg {leg}: {legs[leg]['ms_per_step']:.2f} ms per step", file=sys.stderr, flush=True)
            del A2
            torch.cuda.empty_cache()
            continue
        A2 = leg_matrix(c2)
        torch.cuda.synchronize()
        print(f"[bench] {wl}: matrix ready", file=sys.stderr, flush=True)
        r = run_path(A2, c2, sk, pj, args.leg_steps, args.leg_warmup, args.seed, keep_u=False,
                     flags=variant_flags[var])
        if var == "nystrom":
            r["method"] = "Nystrom eigendecomposition (Section 9): A ~= U diag(S) U^T"
        elif var == "singlepass":
            r["method"] = "single-pass SVD (Section 5.2): Y_c = A G_c, Y_r = A^T G_r, least-squares core"
        if c2.noise_std == 0.0:
            r["vs_planted_sigma"] = vs_planted(c2.sigma(), r["_S"])
        r.pop("_S")
        r.pop("_U")
        r.update({"workload": wl, "m": c2.m, "n": c2.n, "k": c2.k, "p": c2.p, "q": c2.q,
                  "steps": args.leg_steps, "warmup": args.leg_warmup})
        legs[leg] = r
        print(f"[bench] leg {leg}: {r['ms_per_step']:.2f} ms per step", file=sys.stderr, flush=True)
        del A2
        torch.cuda.empty_cache()
    del A
    if legs:
        out["legs"] = legs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
