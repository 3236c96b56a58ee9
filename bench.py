#!/usr/bin/env python3
"""SP2 density-matrix throughput on one MI355X.

One "step" is one complete SP2 solve of a synthetic tight-binding Hamiltonian
through the C ABI: Gershgorin bounds, X_0, every trace-steered squaring until
||X^2 - X||_F <= tol, and the copy of D.  Inputs are resident in HBM before
the timed region starts.

Default workload: n = 4096 (1024 atoms x 4 orbitals), n_occ = 2048, HOMO-LUMO
gap opened to 0.5 eV, H stored in FP32, tol 1e-10, mixed precision (FP64
prefix, split-operand FP16 x2 squarings on the 16-bit matrix cores, FP64
refinement).  The same run also times the plain FP64 solve, which is both the
accuracy reference of the metric ("vs FP64 SP2") and the speed-up baseline.

Printed (one JSON line on stdout): density matrices per second, algorithmic
TFLOP/s (n^2 (n+1) per symmetric squaring), accuracy against the FP64 GPU
solve and against an FP64 eigendecomposition of the same stored H, the
roofline position of the dominant squaring kernel from HIP events taken
around each of its launches inside the timed region, the roofline fraction of
the whole mixed solve (sum over squarings of executed flops / peak of their
precision, over the wall time), and the FP64 CPU oracle timed on a bounded
sample on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SP2 density matrices/s + MFMA TFLOP/s at ‖D−D_ref‖_F/√n ≤ 1e-6 vs FP64 SP2"
PEAKS_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0, "fp8": 5000.0}
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Sources a step's kernels are compiled from (step kernel, step end, headers).
STEP_SOURCES = {
    "syrk_f64.hip": ["syrk_f64.hip", "syrk_f64_core.h", "sk_finish.h", "step_end.hip", "sp2_device.h",
                     "sp2_internal.h"],
    "syrk_lp.hip": ["syrk_lp.hip", "syrk_f64_core.h", "sk_finish.h", "step_end.hip", "sp2_device.h",
                    "sp2_internal.h"],
}


def kernel_sha(name):
    """sha256 prefix over the sources of a step's kernels, in a fixed order."""
    h = hashlib.sha256()
    for src in STEP_SOURCES.get(name, [name]):
        with open(os.path.join(ROOT, "paper_2401_13772_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_file, workload):
    """HBM bytes per launch from a committed counter summary, if it is current.

    The summary's lines `source_sha:`, `workload:`, `fetch_bytes_per_launch:` and
    `write_bytes_per_launch:` are used only when source_sha matches the kernel
    source as it is now.
    """
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip().strip("-* `")] = v.strip().strip("` ")
    if vals.get("source_sha") != kernel_sha(kernel_file):
        return None
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(H64, n_occ, iterations, steps):
    """The FP64 oracle's SP2 loop on this host: `steps` squarings of the same
    workload (a bounded sample), scaled to density matrices per second with
    the FP64 solve's iteration count.  Also times the oracle's Jacobi
    eigendecomposition route to D on a 256-orbital matrix of the same model
    (one thread), for scale."""
    import oracle
    from tbgen import make_tb_hamiltonian
    threads = len(os.sched_getaffinity(0))
    threads = min(threads, oracle.max_threads()) if oracle.max_threads() > 0 else threads
    t0 = time.perf_counter()
    r = oracle.sp2(H64, n_occ, tol=1e-10, max_iter=steps, nthreads=threads)
    dt = time.perf_counter() - t0
    per_step = dt / max(r.iterations, 1)
    small = make_tb_hamiltonian(256, seed=0, gap=0.5)
    t1 = time.perf_counter()
    oracle.jacobi_dm(small.H, small.n_occ)
    dj = time.perf_counter() - t1
    return {
        "value": 1.0 / (per_step * iterations),
        "unit": "DM/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"oracle_sp2 (plain C triple loops, FP64, OpenMP over rows, {threads} threads) ran "
                   f"the first {r.iterations} of the {iterations} squarings of the same n={H64.shape[0]} "
                   f"FP64 solve in {dt:.2f} s; value = 1/({per_step:.3f} s x {iterations})"),
        "jacobi_dm_n256_1thread_s": round(dj, 3),
    }


def copy_calibration(nbytes):
    """A plain device-to-device copy of known size, for scaling HBM counters."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 3}), flush=True)


PRODUCTS = {"f64": 1, "f16x2": 3, "bf16x3": 6, "bf16x2": 3, "fp8": 3}


def timed_solves(sp2, H, D, ws, n_occ, args, compute, steps, warmup, stream):
    """warmup + `steps` timed solves; per-kernel HIP-event sums of the squarings."""
    import torch

    def solve():
        _, info = sp2.sp2_density(H, n_occ, tol=args.tol, max_iter=sp2.MAX_ITER, compute=compute,
                                  fp64_prefix_iters=args.prefix, D=D, workspace=ws, stream=stream)
        if info.status < 0:
            raise RuntimeError(f"sp2_density: {info.status_str}")
        return info

    for _ in range(warmup):
        solve()
    torch.cuda.synchronize()
    sp2.sp2_profile_enable(True)
    kern = {"f64": [0.0, 0], "split": [0.0, 0]}
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(solve())
        (fm, fk), (lm, lk) = sp2.sp2_profile_read_split()
        kern["f64"][0] += fm
        kern["f64"][1] += fk
        kern["split"][0] += lm
        kern["split"][1] += lk
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sp2.sp2_profile_enable(False)
    return elapsed, infos, kern


def kernel_lines(kern, n, elapsed, compute):
    """Per step kind: the step kernel plus the step end (split-tile finish and
    steering) that follows it, timed together by the library's HIP events."""
    flops_per_sq = float(n) * n * (n + 1)
    f64_step = "k_syrk_f64_hyb + k_step_finish + k_step_steer" if n > 2048 else "k_syrk_f64"
    kinds = {"f64": (f64_step, PEAKS_TFLOPS["f64"], 1),
             "split": ("k_syrk_lp + k_step_finish + k_step_steer", PEAKS_TFLOPS["fp8" if compute == "fp8" else "f16"],
                       PRODUCTS[compute])}
    lines = {}
    for key, (ms_tot, launches) in kern.items():
        if launches == 0:
            continue
        name, peak, mult = kinds[key]
        avg_s = ms_tot / 1e3 / launches
        ach = flops_per_sq / avg_s / 1e12
        lines[key] = {
            "kernel": name,
            "bound": "mfma",
            "achieved": round(ach, 3),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(ach / peak, 4),
            "executed_tflops": round(ach * mult, 3),
            "frac_executed": round(ach * mult / peak, 4),
            "per_launch_flops": flops_per_sq,
            "avg_launch_ms": round(1e3 * avg_s, 4),
            "launches_timed": launches,
            "share_of_solve": round(ms_tot / (1e3 * elapsed), 4),
        }
    return lines


def _learned_sample(args):
    """One generated Hamiltonian of the learned workload: (H, ascending
    spectrum, Gershgorin bounds, n_occ).  Worker of a process pool."""
    n, seed, gap, keep_h = args
    import numpy as np
    from threadpoolctl import threadpool_limits
    from tbgen import make_tb_hamiltonian
    with threadpool_limits(1):     # one BLAS thread per pool worker
        inst = make_tb_hamiltonian(n, seed=seed, gap=gap, dtype=np.float32)
    H = inst.H.astype(np.float64)
    R = np.abs(H).sum(1) - np.abs(np.diag(H))
    lo, hi = float((np.diag(H) - R).min()), float((np.diag(H) + R).max())
    # the spectrum the generator built H from (FP64; the FP32 storage moves
    # it by ~1e-6 eV, far below what the layers resolve)
    w = np.sort(inst.eigvals)
    return (inst.H if keep_h else None), w, (lo, hi), inst.n_occ


def bench_learned(args):
    """The learned recursive expansion: 16 trace-steered quadratic layers
    trained on the spectra of 20,000 generated n = 512 Hamiltonians (gaps
    U(0.3, 2) eV, seeds 100000 + s), then inference on 256 held-out ones (seeds
    200000 + b) against the plain SP2 plan on the same 256.  A step is one
    solve of the 256; value = density matrices per second of the learned path."""
    import multiprocessing as mp
    import numpy as np
    import torch

    n, L = 512, args.layers
    rng = np.random.default_rng(args.seed)
    gaps_tr = rng.uniform(0.3, 2.0, args.train)
    gaps_te = rng.uniform(0.3, 2.0, args.batch_learned)
    workers = min(16, len(os.sched_getaffinity(0)))
    log(f"generating {args.train} training spectra and {args.batch_learned} held-out H (n={n}, {workers} procs)")
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        tr = []
        for s in pool.imap(_learned_sample, [(n, 100000 + s, float(gaps_tr[s]), False)
                                             for s in range(args.train)], chunksize=64):
            tr.append(s)
            if len(tr) % 2000 == 0:
                log(f"  {len(tr)} / {args.train} training spectra ({time.perf_counter() - t0:.0f} s)")
        te = pool.map(_learned_sample, [(n, 200000 + b, float(gaps_te[b]), True)
                                        for b in range(args.batch_learned)], chunksize=8)
    log(f"  generated in {time.perf_counter() - t0:.1f} s")
    import paper_2401_13772_amd as sp2
    t0 = time.perf_counter()
    model = sp2.Learned.fit(L, [s[1] for s in tr], [s[3] for s in tr], [s[2] for s in tr],
                            epochs=args.epochs, seed=args.seed)
    fit_s = time.perf_counter() - t0
    coef, loss = model.coefficients()
    log(f"  trained {L} layers, {args.epochs} epochs in {fit_s:.1f} s, loss {loss:.2f}")
    Hs = [torch.from_numpy(s[0]).cuda() for s in te]
    nocc = [s[3] for s in te]
    Ds = [torch.empty_like(H) for H in Hs]
    for _ in range(args.warmup):
        model.density(Hs, nocc, Ds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, infos = model.density(Hs, nocc, Ds)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    plan = sp2.Plan([n] * len(Hs), nocc, dtype="f32", tol=1e-10, max_iter=60)
    D2 = [torch.empty_like(H) for H in Hs]
    plan.run(Hs, D2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, pinfos = plan.run(Hs, D2)
    torch.cuda.synchronize()
    el2 = (time.perf_counter() - t0) / args.steps
    errs = []
    for k, s in enumerate(te):
        w, V = np.linalg.eigh(s[0].astype(np.float64))
        Dref = V[:, :s[3]] @ V[:, :s[3]].T
        errs.append(float(np.linalg.norm(Ds[k].cpu().numpy().astype(np.float64) - Dref)) / np.sqrt(n))
    errs = np.array(errs)
    st = np.array([i.status for i in infos])
    layers_its = np.array([i.iterations for i in infos])
    sp2_its = np.array([i.iterations for i in pinfos])
    flops = sum(float(n) * n * (n + 1) * i.iterations for i in infos)
    out = {
        "metric": METRIC, "value": round(len(Hs) / el, 2), "unit": "DM/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * el, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"sp2_learned{L}_n512_batch{len(Hs)}_f32storage", "layers": L, "train": args.train,
                   "epochs": args.epochs},
        "fit_seconds": round(fit_s, 2), "fit_loss": loss,
        "plain_sp2_plan": {"value": round(len(Hs) / el2, 2), "unit": "DM/s", "mean_iterations": float(sp2_its.mean())},
        "speedup_vs_plain_sp2": round(el2 / el, 3),
        "mean_squarings": float(layers_its.mean()),
        "status_counts": {"ok": int((st == 0).sum()), "fallback": int((st == 3).sum()),
                          "other": int(((st != 0) & (st != 3)).sum())},
        "err_rms_vs_eigh": {"median": float(np.median(errs)), "max": float(errs.max())},
        "meets_1e-6": bool(errs.max() <= 1e-6),
        "tflops_algorithmic": round(flops / el / 1e12, 3),
        "roofline": {"bound": "mfma", "achieved": round(flops / el / 1e12, 3), "peak": PEAKS_TFLOPS["f64"],
                     "unit": "TFLOP/s", "frac": round(flops / el / 1e12 / PEAKS_TFLOPS["f64"], 4),
                     "traffic": None,
                     "note": "whole batched learned solve (all kernels) against the FP64 matrix peak"},
        "coefficients": coef.tolist(),
    }
    model.close()
    plan.close()
    print(json.dumps(out), flush=True)


def bench_graph(args):
    """The graph-partitioned solver on the local gapped model: n = 16384 (4096
    atoms), 64 core parts of 256 orbitals, threshold 0.03 eV on H, FP32
    storage, FP64 squarings, mu = 0 (mid-gap by construction).  A step is one
    sp2_graph_density call (gather, batched mu-steered SP2 of the 64 parts,
    map-back); value = full density matrices per second.  The dense FP64 SP2
    solve of the same H is timed beside it and is the error reference."""
    import numpy as np
    import torch

    import paper_2401_13772_amd as sp2
    from tbgen import make_local_hamiltonian
    n, parts, tau = args.graph_n, args.graph_parts, args.graph_tau
    log(f"generating the local gapped model n={n}")
    t0 = time.perf_counter()
    inst = make_local_hamiltonian(n, seed=args.seed, dtype=np.float32)
    log(f"  generated in {time.perf_counter() - t0:.1f} s")
    H = torch.from_numpy(inst.H).cuda()
    del inst.H
    t0 = time.perf_counter()
    g = sp2.Graph(H, tau, parts, tol=args.tol)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    sizes, cores = g.sizes()
    log(f"  {parts} parts, core {min(cores)}..{max(cores)}, core+halo {min(sizes)}..{max(sizes)} "
        f"(created in {create_s:.2f} s)")
    D = torch.empty_like(H)
    for _ in range(args.warmup):
        g.density(H, inst.mu, D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, infos = g.density(H, inst.mu, D)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    bad = [(k, i.status_str, i.iterations, i.idempotency) for k, i in enumerate(infos) if i.status != 0]
    assert not bad, f"parts that did not converge: {bad[:4]}"
    flops = sum(float(s) * s * (s + 1) * i.iterations for s, i in zip(sizes, infos))
    log(f"  graph solve {1e3 * el:.2f} ms, {flops / el / 1e12:.2f} TFLOP/s algorithmic")
    # dense FP64 SP2 of the same H (one warm-up, then timed)
    ws = sp2.alloc_workspace(n, "f32", "f64")
    Dd = torch.empty_like(H)
    sp2.sp2_density(H, n // 2, tol=args.tol, D=Dd, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dense_steps = max(1, min(args.steps, 2))
    for _ in range(dense_steps):
        _, idense = sp2.sp2_density(H, n // 2, tol=args.tol, D=Dd, workspace=ws)
    torch.cuda.synchronize()
    el_dense = (time.perf_counter() - t0) / dense_steps
    del ws
    diff = (D.double() - Dd.double())
    err = float(torch.linalg.norm(diff)) / np.sqrt(n)
    err_avg = float(torch.linalg.norm(diff)) / n
    asym = float(torch.linalg.norm(D.double() - D.double().T)) / np.sqrt(n)
    tr_err = abs(float(torch.trace(D.double())) - n / 2)
    log(f"  dense FP64 SP2 {1e3 * el_dense:.1f} ms ({idense.iterations} squarings); "
        f"rms|D_graph - D_dense| = {err:.3e}, ||.||_F/n = {err_avg:.3e}, trace error {tr_err:.3e}")
    tf = flops / el / 1e12
    out = {
        "metric": METRIC, "value": round(1.0 / el, 4), "unit": "DM/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * el, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"sp2_graph_local_n{n}_parts{parts}_tau{tau:g}_f32storage_f64", "n": n,
                   "parts": parts, "tau_eV": tau, "mu_eV": inst.mu, "tol": args.tol},
        "parts": {"core_min": min(cores), "core_max": max(cores), "size_min": min(sizes),
                  "size_max": max(sizes), "size_mean": round(float(np.mean(sizes)), 1),
                  "iterations_max": max(i.iterations for i in infos), "create_s": round(create_s, 3)},
        "dense_fp64_sp2": {"value": round(1.0 / el_dense, 4), "unit": "DM/s", "ms": round(1e3 * el_dense, 2),
                           "iterations": idense.iterations},
        "speedup_vs_dense_fp64": round(el_dense / el, 2),
        "err_rms_vs_dense": err, "err_fro_over_n_vs_dense": err_avg, "asymmetry_rms": asym,
        "trace_error": tr_err,
        "tflops_algorithmic": round(tf, 3),
        "roofline": {"bound": "mfma", "achieved": round(tf, 3), "peak": PEAKS_TFLOPS["f64"], "unit": "TFLOP/s",
                     "frac": round(tf / PEAKS_TFLOPS["f64"], 4), "traffic": None,
                     "note": "whole graph solve (gather, batched steps, map-back) against the FP64 matrix peak"},
    }
    g.close()
    print(json.dumps(out), flush=True)


def bench_sparse(args):
    """Thresholded SP2 with tile skipping on the local gapped model: n = 16384,
    tau = 1e-5, FP32 storage, FP64 arithmetic.  A step is one
    sp2_density_sparse solve; the dense FP64 SP2 of the same H is timed beside
    it and is the error reference."""
    import numpy as np
    import torch

    import paper_2401_13772_amd as sp2
    from tbgen import make_local_hamiltonian
    n, tau = args.sparse_n, args.sparse_tau
    log(f"generating the local gapped model n={n}")
    inst = make_local_hamiltonian(n, seed=args.seed, dtype=np.float32)
    H = torch.from_numpy(inst.H).cuda()
    del inst.H
    nbytes = sp2.sp2_sparse_workspace_size(n)
    wraw = torch.empty(nbytes + sp2.WORKSPACE_ALIGN, dtype=torch.uint8, device="cuda")
    off = (-wraw.data_ptr()) % sp2.WORKSPACE_ALIGN
    ws = wraw[off:off + nbytes]
    D = torch.empty_like(H)
    for _ in range(args.warmup):
        sp2.sp2_density_sparse(H, inst.n_occ, tau, tol=args.tol, D=D, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = sp2.sp2_density_sparse(H, inst.n_occ, tau, tol=args.tol, D=D, workspace=ws)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    flops_exec, tile_steps = sp2.sp2_sparse_stats(ws)
    T = (n + 127) // 128
    dense_eq = float(n) * n * (n + 1) * info.iterations
    log(f"  sparse solve {1e3 * el:.1f} ms, {info.iterations} steps, status {info.status_str}, "
        f"executed {flops_exec / dense_eq:.3f} of the dense work, {flops_exec / el / 1e12:.2f} TFLOP/s executed")
    del ws, wraw
    wsd = sp2.alloc_workspace(n, "f32", "f64")
    Dd = torch.empty_like(H)
    sp2.sp2_density(H, inst.n_occ, tol=1e-10, D=Dd, workspace=wsd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, idense = sp2.sp2_density(H, inst.n_occ, tol=1e-10, D=Dd, workspace=wsd)
    torch.cuda.synchronize()
    el_dense = time.perf_counter() - t0
    del wsd
    diff = D.double() - Dd.double()
    err = float(torch.linalg.norm(diff)) / np.sqrt(n)
    zero_frac = float((D == 0).double().mean())
    log(f"  dense FP64 SP2 {1e3 * el_dense:.1f} ms; rms|D_sparse - D_dense| = {err:.3e}; "
        f"zero entries {zero_frac:.3f}")
    tf = flops_exec / el / 1e12
    out = {
        "metric": METRIC, "value": round(1.0 / el, 4), "unit": "DM/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * el, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"sp2_sparse_local_n{n}_tau{tau:g}_f32storage_f64", "n": n, "tau": tau,
                   "tol": args.tol},
        "status": info.status_str, "iterations": info.iterations, "idempotency": info.idempotency,
        "trace_error": info.trace_error,
        "executed_fraction_of_dense": round(flops_exec / dense_eq, 4),
        "tile_fraction": round(tile_steps / (info.iterations * T * (T + 1) / 2), 4),
        "dense_fp64_sp2": {"value": round(1.0 / el_dense, 4), "unit": "DM/s", "ms": round(1e3 * el_dense, 2),
                           "iterations": idense.iterations},
        "speedup_vs_dense_fp64": round(el_dense / el, 3),
        "err_rms_vs_dense": err, "zero_entry_fraction": round(zero_frac, 4),
        "roofline": {"bound": "mfma", "achieved": round(tf, 3), "peak": PEAKS_TFLOPS["f64"], "unit": "TFLOP/s",
                     "frac": round(tf / PEAKS_TFLOPS["f64"], 4), "traffic": None,
                     "note": "executed FP64 MFMA work of the tile-skipping solve over its wall time"},
    }
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """512 problems with sizes uniform on {64, 68, ..., 512} (n_occ = n/2, gap
    0.5 eV, FP32 storage, FP64 squarings): one graph replay of the batched plan
    vs the same problems as 512 separate sp2_density calls.  A step is one
    solve of the whole batch; value = density matrices per second."""
    import numpy as np
    import torch

    import paper_2401_13772_amd as sp2
    from tbgen import batch_sizes, make_tb_hamiltonian
    sizes = [int(v) for v in batch_sizes(args.batch, seed=args.seed)]
    log(f"generating {len(sizes)} tight-binding Hamiltonians (n 64..512)")
    t0 = time.perf_counter()
    Hs, nocc = [], []
    for k, n in enumerate(sizes):
        inst = make_tb_hamiltonian(n, seed=10_000 + k, gap=args.gap, dtype=np.float32)
        Hs.append(torch.from_numpy(inst.H).cuda())
        nocc.append(inst.n_occ)
    log(f"  generated in {time.perf_counter() - t0:.1f} s")
    cache = args.autotune_cache or None
    plan = sp2.Plan(sizes, nocc, dtype="f32", tol=args.tol, max_iter=args.batch_max_iter,
                    autotune_cache=cache)
    Ds = [torch.empty_like(H) for H in Hs]
    for _ in range(args.warmup):
        plan.run(Hs, Ds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, infos = plan.run(Hs, Ds)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert all(i.status == 0 for i in infos), "a batched solve did not converge"
    # baseline: 512 plain launches of the single-matrix solve
    ws = sp2.alloc_workspace(max(sizes), "f32", "f64")
    D1 = [torch.empty_like(H) for H in Hs]
    for k in range(len(sizes)):
        sp2.sp2_density(Hs[k], nocc[k], tol=args.tol, D=D1[k], workspace=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    iters = 0
    for k in range(len(sizes)):
        _, i1 = sp2.sp2_density(Hs[k], nocc[k], tol=args.tol, D=D1[k], workspace=ws)
        iters += i1.iterations
    torch.cuda.synchronize()
    el1 = time.perf_counter() - t1
    same = all(torch.equal(a, b) for a, b in zip(Ds, D1)) if cache is None else None
    flops = sum(float(n) * n * (n + 1) * i.iterations for n, i in zip(sizes, infos))
    per_batch = el / args.steps
    out = {
        "metric": METRIC, "value": round(len(sizes) / per_batch, 2), "unit": "DM/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * per_batch, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"sp2_tb_batch{len(sizes)}_n64to512_f32storage_f64", "batch": len(sizes),
                   "gap_eV": args.gap, "tol": args.tol, "tile_shape": plan.config},
        "tflops_algorithmic": round(flops / per_batch / 1e12, 3),
        "roofline": {"bound": "mfma", "achieved": round(flops / per_batch / 1e12, 3),
                     "peak": PEAKS_TFLOPS["f64"], "unit": "TFLOP/s",
                     "frac": round(flops / per_batch / 1e12 / PEAKS_TFLOPS["f64"], 4),
                     "note": "whole batched solve (all kernels) against the FP64 matrix peak"},
        "plain_launches": {"value": round(len(sizes) / el1, 2), "unit": "DM/s", "ms": round(1e3 * el1, 3),
                           "iterations_total": iters},
        "speedup_vs_plain_launches": round(el1 / per_batch, 3),
        "bitwise_equal_to_plain": same,
        "max_idempotency": max(i.idempotency for i in infos),
        "max_trace_error": max(i.trace_error for i in infos),
    }
    plan.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--gap", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--compute", default="f16x2", choices=["f64", "f16x2", "bf16x3", "bf16x2", "fp8"])
    ap.add_argument("--prefix", type=int, default=-1,
                    help="FP64 steps before the split-operand phase (-1 = library default)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f64"])
    ap.add_argument("--fp64-steps", type=int, default=5,
                    help="timed plain-FP64 solves (accuracy reference and speed-up baseline; 0 = skip)")
    ap.add_argument("--cpu-steps", type=int, default=6,
                    help="oracle squarings in the CPU-baseline sample (0 = skip)")
    ap.add_argument("--no-reference", action="store_true",
                    help="skip the FP64 eigendecomposition accuracy check (profiling runs)")
    ap.add_argument("--workload", default="single", choices=["single", "batch", "learned", "graph", "sparse"],
                    help="single: one n x n solve (default); batch: the batched plan (512 problems)")
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--graph-n", type=int, default=16384, help="graph workload: matrix size")
    ap.add_argument("--graph-parts", type=int, default=64, help="graph workload: core parts")
    ap.add_argument("--graph-tau", type=float, default=0.03, help="graph workload: adjacency threshold (eV)")
    ap.add_argument("--sparse-n", type=int, default=16384, help="sparse workload: matrix size")
    ap.add_argument("--sparse-tau", type=float, default=1e-5, help="sparse workload: drop threshold")
    ap.add_argument("--layers", type=int, default=16, help="learned workload: quadratic layers")
    ap.add_argument("--train", type=int, default=20000, help="learned workload: training Hamiltonians")
    ap.add_argument("--epochs", type=int, default=600, help="learned workload: passes over the training set")
    ap.add_argument("--batch-learned", type=int, default=256, help="learned workload: held-out batch")
    ap.add_argument("--batch-max-iter", type=int, default=60)
    ap.add_argument("--autotune-cache", default="",
                    help="batch: autotune the tile shape with this cache file (default: no autotune)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain copy of BYTES bytes (counter scaling) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "learned":
        bench_learned(args)
        return
    if args.workload == "graph":
        bench_graph(args)
        return
    if args.workload == "sparse":
        bench_sparse(args)
        return

    import paper_2401_13772_amd as sp2
    from tbgen import make_tb_hamiltonian

    n = args.n
    n_occ = n // 2
    storage = np.float32 if args.storage == "f32" else np.float64
    log(f"generating tight-binding H n={n} seed={args.seed} gap={args.gap} storage={args.storage}")
    t0 = time.perf_counter()
    inst = make_tb_hamiltonian(n, args.seed, gap=args.gap, dtype=storage,
                               eigh_device="cuda" if n > 8192 else None)
    log(f"  generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    H = torch.from_numpy(inst.H).to(dev)
    stream = torch.cuda.current_stream()
    flops_per_sq = float(n) * n * (n + 1)

    # plain FP64 SP2: the metric's accuracy reference and the speed-up baseline
    fp64 = None
    D64 = None
    if args.compute != "f64" and args.fp64_steps > 0:
        log(f"FP64 leg: warmup x1, timed x{args.fp64_steps}")
        D64 = torch.empty_like(H)
        ws64 = sp2.alloc_workspace(n, args.storage, "f64", device=dev)
        el64, inf64, kern64 = timed_solves(sp2, H, D64, ws64, n_occ, args, "f64", args.fp64_steps, 1, stream)
        l64 = kernel_lines(kern64, n, el64, "f64")["f64"]
        fp64 = {"value": round(args.fp64_steps / el64, 4), "unit": "DM/s",
                "ms_per_step": round(1e3 * el64 / args.fp64_steps, 4), "iterations": inf64[-1].iterations,
                "status": inf64[-1].status_str, "k_syrk_f64": l64}
        del ws64
        torch.cuda.empty_cache()
        log(f"  FP64: {fp64['ms_per_step']:.3f} ms/DM, {inf64[-1].iterations} squarings, "
            f"k_syrk_f64 {l64['avg_launch_ms']:.4f} ms = {l64['achieved']:.1f} TFLOP/s")

    D = torch.empty_like(H)
    ws = sp2.alloc_workspace(n, args.storage, args.compute, device=dev)
    log(f"main leg ({args.compute}): warmup x{args.warmup}, timed x{args.steps}")
    elapsed, infos, kern = timed_solves(sp2, H, D, ws, n_occ, args, args.compute, args.steps,
                                        args.warmup, stream)
    info = infos[-1]
    iters = info.iterations
    ms_per_step = 1e3 * elapsed / args.steps
    dms = args.steps / elapsed
    flops_per_dm = sum(i.iterations for i in infos) / len(infos) * flops_per_sq
    tflops = flops_per_dm * dms / 1e12
    lines = kernel_lines(kern, n, elapsed, args.compute)
    dominant = max(lines, key=lambda k: kern[k][0])
    # roofline fraction of the whole solve: sum over squarings of executed
    # flops / peak of their precision, over the wall time
    peak_time = 0.0
    for key, (ms_tot, launches) in kern.items():
        if launches:
            peak = PEAKS_TFLOPS["f64"] if key == "f64" else PEAKS_TFLOPS["fp8" if args.compute == "fp8" else "f16"]
            mult = 1 if key == "f64" else PRODUCTS[args.compute]
            peak_time += launches * flops_per_sq * mult / (peak * 1e12)
    solve_frac = peak_time / elapsed
    log(f"status={info.status_str} iterations={iters} (FP64 prefix {info.fp64_prefix_iters}, "
        f"refine {info.refine_steps}) {ms_per_step:.3f} ms/DM {dms:.2f} DM/s {tflops:.2f} TFLOP/s "
        f"solve roofline fraction {solve_frac:.3f}")
    for key, ln in lines.items():
        log(f"  {ln['kernel']}: {ln['launches_timed']} launches, {ln['avg_launch_ms']:.4f} ms avg, "
            f"{ln['achieved']:.1f} TFLOP/s algorithmic ({ln['executed_tflops']:.1f} executed), "
            f"{100 * ln['share_of_solve']:.1f}% of the solve")

    # accuracy of the last D
    Dg = D.double()
    Hd = H.double()
    idem = float(torch.linalg.norm(Dg @ Dg - Dg))
    comm = float(torch.linalg.norm(Hd @ Dg - Dg @ Hd)) / np.sqrt(n)
    tr_err = abs(float(torch.trace(Dg)) - n_occ)
    err_fp64 = None
    if D64 is not None:
        err_fp64 = float(torch.linalg.norm(Dg - D64.double())) / np.sqrt(n)
        log(f"  rms|D - D_fp64_sp2| = {err_fp64:.3e}")
    err_ref = None
    if not args.no_reference:
        log("FP64 eigendecomposition of the stored H (accuracy reference)")
        t0 = time.perf_counter()
        w, V = np.linalg.eigh(inst.H.astype(np.float64))
        Dref = torch.from_numpy(V[:, :n_occ] @ V[:, :n_occ].T).to(dev)
        err_ref = float(torch.linalg.norm(Dg - Dref)) / np.sqrt(n)
        log(f"  eigh {time.perf_counter() - t0:.1f} s; rms|D - D_ref| = {err_ref:.3e}")
        del Dref

    workload = f"sp2_tb_n{n}_{args.storage}storage_{args.compute}"
    roofline = dict(lines[dominant])
    kernel_file = "syrk_f64.hip" if dominant == "f64" else "syrk_lp.hip"
    tw = workload if dominant != "f64" else f"sp2_tb_n{n}_{args.storage}storage_f64"
    roofline["traffic"] = read_traffic(kernel_file, tw)
    others = [dict(v) for k, v in lines.items() if k != dominant]

    cpu = None
    if args.cpu_steps > 0:
        log(f"CPU oracle sample: {args.cpu_steps} squarings")
        it64 = fp64["iterations"] if fp64 else iters
        cpu = cpu_baseline(inst.H.astype(np.float64), n_occ, it64, args.cpu_steps)
        log(f"  {cpu['sample']}")

    out = {
        "metric": METRIC,
        "value": round(dms, 4),
        "unit": "DM/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.compute,
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "n_occ": n_occ, "gap_eV": args.gap,
                   "storage": args.storage, "compute": args.compute, "tol": args.tol,
                   "fp64_prefix": info.fp64_prefix_iters, "seed": args.seed},
        "tflops_algorithmic": round(tflops, 3),
        "iterations": iters,
        "fp64_prefix_iters": info.fp64_prefix_iters,
        "refine_steps": info.refine_steps,
        "status": info.status_str,
        "err_rms_vs_fp64_sp2": err_fp64,
        "err_rms_vs_fp64_eigh": err_ref,
        "meets_1e-6": None if err_fp64 is None and err_ref is None else
        bool(max(e for e in (err_fp64, err_ref) if e is not None) <= 1e-6),
        "idempotency_fro": idem,
        "trace_error": tr_err,
        "commutator_rms": comm,
        "fp64_sp2": fp64,
        "speedup_vs_fp64_sp2": None if fp64 is None else round(dms / fp64["value"], 3),
        "solve_roofline_frac": round(solve_frac, 4),
        "roofline": roofline,
        "roofline_other_kernels": others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
