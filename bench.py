#!/usr/bin/env python3
"""Benchmark of the FGFRFT online stage on one MI355X.

Workload (default): kNN graph (k=10, Gaussian weights) on 4096 points from a
5-component 3-D Gaussian mixture, combinatorial Laplacian, F = U^T (real
orthogonal), L = 32, 256 orders uniform in [-2, 2], 64 real N(0,1) signals per
order.  One step = operator update for all 256 orders (coefficients on the
GPU, one launch) followed by the apply of each operator to its 64 signals.
Inputs are resident in HBM before timing starts; the plan (offline stage) is
built once, outside the timed region, as in the paper's own timings.

Prints one JSON line.  ``--gpus N`` with N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 31          # plain device copy used as the counter and bandwidth reference

# HBM bytes per k_update launch on this workload, from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch), each scaled by the same counter's reading for the plain
# copy of COPY_BYTES that this script runs.  Valid only for the kernel sources with this digest:
# once update.hip or internal.h change, the figure is reported as null until re-measured.
UPDATE_TRAFFIC = {"fetch_bytes": 4362316720, "write_bytes": 34365347584,
                  "source_sha256": "80a71ad94fa4793f0a7b1bc340e59dc76448790d91f14ef1c112cc35e3974bb2"}
# The same for one k_direct_pair launch over 64 signal columns of the knn4096 plan (FP16X2 stack;
# direct.hip + internal.h).
DIRECT_TRAFFIC = {"fetch_bytes": 2225043155, "write_bytes": 67108864, "ncols": 64,
                  "source_sha256": "fd3bc293a225be9b1a52c6790e40e76d8b0ebd80473cefe1c6f3de21a336cf3c"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def update_algorithmic_bytes(N, L, n_alpha):
    # per order: 8 N^2 (complex64 Q written) + [(L+1) 4N^2 (M_0..M_L) + 4N^2 (P)] / n_alpha
    return n_alpha * 8.0 * N * N + (L + 2) * 4.0 * N * N


def apply_algorithmic_bytes(N, B, n_alpha):
    # per order: 8 N^2 (Q read) + 4 N B (x read) + 8 N B (y written)
    return n_alpha * (8.0 * N * N + 12.0 * N * B)


def source_digest(main):
    import hashlib
    h = hashlib.sha256()
    for f in (main, "internal.h"):
        with open(os.path.join(ROOT, "paper_2602_20870_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def update_source_digest():
    return source_digest("update.hip")


def update_traffic():
    t = UPDATE_TRAFFIC
    if t["source_sha256"] is None or t["source_sha256"] != update_source_digest():
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def copy_bandwidth(dev, reps=5):
    """Plain device-to-device copy of COPY_BYTES (read + write), GB/s over `reps` launches."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES, "ms": ms, "GBps": 2 * COPY_BYTES / (ms * 1e-3) / 1e9}


def write_bandwidth(dev, nbytes=1 << 33, reps=5):
    """Write-only streaming kernel (16-byte nontemporal stores, fgfrft_probe_write) over `nbytes`:
    the write bandwidth the device attains, the ceiling for the store-dominated update."""
    import torch
    from paper_2602_20870_amd import lib
    from paper_2602_20870_amd._lib import check
    import ctypes
    buf = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    s = ctypes.c_void_p(stream.cuda_stream)
    check(lib().fgfrft_probe_write(ctypes.c_void_p(buf.data_ptr()), nbytes, s), "fgfrft_probe_write")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        check(lib().fgfrft_probe_write(ctypes.c_void_p(buf.data_ptr()), nbytes, s), "fgfrft_probe_write")
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del buf
    torch.cuda.empty_cache()
    return {"bytes_written": nbytes, "ms": ms, "GBps": nbytes / (ms * 1e-3) / 1e9}


def update_traffic_reference(dev, N, L, na, reps=5):
    """The operator update's own HBM traffic with no arithmetic (fgfrft_probe_update_traffic): per
    strip of 4 x 64 positions, its 2L + 1 stack-shaped tiles staged in LDS with direct loads, then
    the strip's positions of every order written in the update's store pattern.  The attainable
    time for the update's mix of reads and writes on this device."""
    import torch
    from paper_2602_20870_amd import lib
    from paper_2602_20870_amd._lib import check
    import ctypes
    nt = min(2 * L + 1, 65)
    src = torch.zeros(nt * N * N * 4, dtype=torch.uint8, device=dev)
    dst = torch.empty(na * N * N * 8, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    s = ctypes.c_void_p(stream.cuda_stream)
    call = lambda: check(lib().fgfrft_probe_update_traffic(ctypes.c_void_p(src.data_ptr()), N, nt, na,
                                                           ctypes.c_void_p(dst.data_ptr()), s),
                         "fgfrft_probe_update_traffic")
    call()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        call()
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"kernel": "k_update_traffic: the update's staging reads and store pattern, no arithmetic",
            "tiles": nt, "orders": na, "bytes_read": nt * N * N * 4, "bytes_written": na * N * N * 8, "ms": ms}


def throughput_configs(reps=5):
    """Plain-method throughput on the 32x32 grid (N = 1024, weights U[0.5, 1.5], real F) and the
    directed 256-cycle (unitary DFT, complex F with a -1 eigenspace): L = 32, 256 orders in
    [-2, 2] in one update launch, then the apply to 64 complex Gaussian signals per order."""
    import torch
    import synth
    from paper_2602_20870_amd import Plan, apply_operator

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for name in ("grid1024", "dft256"):
        cfg = synth.make_config(name, seed=0)
        F, L, N, alphas = cfg["F"], cfg["L"], cfg["N"], cfg["alphas"]
        X = torch.from_numpy(cfg["X"].astype(np.complex64)).to(dev)
        na, B = X.shape[0], X.shape[2]
        plan = Plan(torch.from_numpy(F).to(dev), L)
        Q = torch.empty((na, N, N), dtype=torch.complex64, device=dev)
        Y = torch.empty((na, N, B), dtype=torch.complex64, device=dev)
        for _ in range(2):
            plan.update(alphas, out=Q)
            apply_operator(Q, X, out=Y)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1, e2 in ev:
            e0.record(stream)
            plan.update(alphas, out=Q)
            e1.record(stream)
            apply_operator(Q, X, out=Y)
            e2.record(stream)
        torch.cuda.synchronize()
        upd = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
        app = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
        es = 8 if plan.complex else 4
        upd_bytes = na * 8.0 * N * N + (L + 2) * es * N * N       # Q written + M_0..M_L and P read once
        app_bytes = na * (8.0 * N * N + 16.0 * N * B)             # Q read + complex x read, y written
        row = {"workload": name, "N": N, "L": L, "orders": na, "signals_per_order": B, "complex_F": plan.complex,
               "r_minus1": plan.r_minus1, "update_ms": upd, "apply_ms": app, "updates_per_s": na / ((upd + app) * 1e-3),
               "signals_per_s": na * B / ((upd + app) * 1e-3), "update_algorithmic_GBps": upd_bytes / (upd * 1e-3) / 1e9,
               "apply_algorithmic_GBps": app_bytes / (app * 1e-3) / 1e9}
        log(f"throughput {row}")
        rows.append(row)
        del plan, Q, Y, X
        torch.cuda.empty_cache()
    return {"workload": "grid1024 (32x32 grid, real F) and dft256 (directed cycle, unitary DFT): L=32, 256 orders, "
                        "64 complex signals per order; step = update + apply", "rows": rows}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(F, alphas, L, X, budget_s=12.0, chunk=16, one_thread_orders=8):
    """The oracle (FP64 NumPy) taking the GPU line's step on the host cores, over a bounded sample of
    the same workload's orders: Algorithm 1's online combination for a chunk of orders as one BLAS
    product [chunk x (2L+1)] . [(2L+1) x N^2] over the pre-transposed term matrix (P_c, M_1..M_L,
    M_1^H..M_L^H) plus e^{j pi alpha} P, then the apply (Definition 2) of each operator to that order's
    signal block X[a] (host float32 array [n_alpha, N, B]).  Timed once with every BLAS thread and once
    limited to one thread (threadpoolctl).  The offline stage (projector, powers, term matrix) is
    built first and not timed."""
    import oracle as O

    t0 = time.time()
    plan = O.Plan(F, L, route="symmetric")
    T = O.term_matrix(plan.M)
    P = plan.P
    del plan
    setup = time.time() - t0
    alphas = np.asarray(alphas, dtype=np.float64)

    def run(orders_max, budget):
        done, t_acc = 0, 0.0
        while done < min(orders_max, len(alphas)) and t_acc <= budget:
            a0 = done
            a1 = min(done + chunk, orders_max, len(alphas))
            xs = [X[a].astype(np.float64) for a in range(a0, a1)]      # host copies, not timed
            t1 = time.perf_counter()
            Q = O.fgfrft_combine_many(P, T, alphas[a0:a1])
            for i in range(a1 - a0):
                O.apply(Q[i], xs[i])
            t_acc += time.perf_counter() - t1
            del Q
            done = a1
        return done, t_acc

    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:             # threadpoolctl missing: the one-thread leg is skipped
        threadpool_limits, blas = None, None
    affinity = len(os.sched_getaffinity(0))
    done, t_acc = run(len(alphas), budget_s)
    out = dict(value=done / t_acc, unit="updates/s", cores=blas if blas else affinity, kind="oracle",
               sample=(f"{done} of {len(alphas)} orders of the same workload (N={F.shape[0]}, L={L}, "
                       f"{X.shape[-1]} real signals per order), in chunks of {chunk}: the FP64 combination as "
                       f"one BLAS product over the (2L+1) x N^2 term matrix plus the P term, and the complex128 "
                       f"apply to the order's signals; offline setup {setup:.1f}s untimed"),
               seconds=t_acc, affinity_cores=affinity, blas_threads=blas, cpu_model=cpu_model())
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            d1, t1 = run(one_thread_orders, budget_s)
        out["one_thread"] = dict(value=d1 / t1, unit="updates/s", orders=d1, seconds=t1)
    return out


def grad_bench(reps=3, stacktype="fp32"):
    """Order and signal gradients (Proposition 4) on the sphere workload: kNN (k=10) graph on 2048
    points of the unit sphere, L = 48, 64 orders (one per channel), 64 real signals per order."""
    import torch
    import synth
    from paper_2602_20870_amd import Plan

    cfg = synth.make_config("sphere2048", seed=0, with_signals=False)
    F, L, N = cfg["F"], cfg["L"], cfg["N"]
    na, B = 64, 64
    rng = np.random.default_rng(3)
    alphas = rng.uniform(-1.5, 1.5, na)
    dev = torch.device("cuda:0")
    X = torch.from_numpy(rng.standard_normal((na, N, B)).astype(np.float32)).to(dev)
    GY = torch.from_numpy((rng.standard_normal((na, N, B)) + 1j * rng.standard_normal((na, N, B)))
                          .astype(np.complex64)).to(dev)
    plan = Plan(torch.from_numpy(F).to(dev), L, stacktype=stacktype)
    plan.grad(alphas, X, GY, want_dX=True)       # warm-up (kernel attributes, workspace)
    torch.cuda.synchronize()
    out = {"workload": f"sphere2048: N={N}, L={L}, {na} orders, {B} real signals per order"}
    for want_dx in (False, True):
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.grad(alphas, X, GY, want_dX=want_dx)
        torch.cuda.synchronize()
        out["ms_with_dX" if want_dx else "ms_dalpha_only"] = (time.perf_counter() - t0) * 1e3 / reps
    del X, GY
    # the differentiable workload end to end: point-cloud denoiser (3 -> 64 channel lift, per-channel
    # order and mask, projection back), 64 noisy clouds of the same graph, one Adam step per iteration
    from paper_2602_20870_amd.learn import PointCloudDenoiser
    d = synth.point_cloud_denoising(seed=0, N=N, clouds=B)
    model = PointCloudDenoiser(plan, channels=na)
    Y = torch.from_numpy(d["noisy"].astype(np.float32)).to(dev)
    clean = torch.from_numpy(d["clean"].astype(np.float32)).to(dev)
    opt = torch.optim.Adam(model.parameters(), lr=0.01)

    def step():
        opt.zero_grad()
        loss = ((model(Y) - clean[None]) ** 2).mean()
        loss.backward()
        opt.step()
        return float(loss.detach())

    first = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        last = step()
    torch.cuda.synchronize()
    out["denoiser"] = {"workload": f"sphere2048 point-cloud denoiser: 3 -> {na} channel lift, per-channel order "
                                   f"and mask (L={L}), {B} noisy clouds (N(0, 0.05^2)), Adam lr 0.01",
                       "ms_per_training_step": (time.perf_counter() - t0) * 1e3 / reps,
                       "loss_first_step": first, "loss_after": last, "steps": reps + 1}
    del plan, model, Y, clean, opt
    torch.cuda.empty_cache()
    return out


def table4_bench(sizes=(1000, 2000, 3000, 4000, 5000, 6000, 7000, 8000), L=10, alpha=0.5, reps=5):
    """Online time of FGFRFT (operator update for one order) and of the exact GFRFT from a cached
    eigendecomposition (V diag(e^{j alpha theta}) V^H), both on the GPU, plus the accuracy of FGFRFT
    against the exact operator: Haar-random eigenvectors, uniform eigenphases, L = 10, alpha = 0.5."""
    import torch
    import synth
    from paper_2602_20870_amd import Plan, gfrft_exact

    dev = torch.device("cuda:0")
    ev = lambda: torch.cuda.Event(enable_timing=True)
    rows = []
    for N in sizes:
        t0 = time.time()
        rng = np.random.default_rng(N)
        V = torch.from_numpy(synth.haar_unitary(N, rng)).to(dev)
        theta = torch.from_numpy(rng.uniform(-np.pi, np.pi, N)).to(dev)
        Vh = V.conj().T.contiguous()
        F = gfrft_exact(V, Vh, theta, 1.0)            # F = V diag(e^{j theta}) V^H
        plan = Plan(F, L)
        Q = torch.empty((1, N, N), dtype=torch.complex64, device=dev)
        Fa = torch.empty((N, N), dtype=torch.complex128, device=dev)
        times = {}
        for name, fn in (("fgfrft", lambda: plan.update([alpha], out=Q)),
                         ("exact", lambda: gfrft_exact(V, Vh, theta, alpha, out=Fa))):
            fn()
            torch.cuda.synchronize()
            e0, e1 = ev(), ev()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            e1.synchronize()
            times[name] = e0.elapsed_time(e1) / reps
        E = Q[0].to(torch.complex128) - Fa
        f2 = float((E.abs() ** 2).sum())
        row = dict(N=N, fgfrft_ms=times["fgfrft"], exact_ms=times["exact"], speedup=times["exact"] / times["fgfrft"],
                   MSE=f2 / N ** 2, MAE=float(E.abs().sum()) / N ** 2, NMSE=f2 / N)
        log(f"table4 {row} ({time.time() - t0:.0f}s)")
        rows.append(row)
        del V, Vh, F, plan, Q, Fa, E, theta
        torch.cuda.empty_cache()
    return {"workload": f"Haar eigenvectors, uniform phases, L={L}, alpha={alpha}", "rows": rows}


def precision_form_bench(chunks=(32, 128), reps=3):
    """Precision-form workload (grid8192: 128x64 grid, lognormal weights, N = 8192, L = 64, 1024 orders):
    per stack storage form -- FP32, FP16X2 (its split operands stored), BF16 hi/lo pairs (all 4 bytes per
    real value) and the plain complex64 stack of F handed over as complex (8 bytes) -- one update launch
    per order chunk, the pass over all 1024 orders in launches of 128, the apply of a 32-order chunk to
    one shared block of 1024 real signals (real stacks) and the direct route (32 orders x 2 signals)."""
    import torch
    import synth
    from paper_2602_20870_amd import Plan, apply_operator

    dev = torch.device("cuda:0")
    t0 = time.time()
    cfg = synth.make_config("grid8192", seed=0, with_signals=False)
    F, L, N = cfg["F"], cfg["L"], cfg["N"]
    alphas = cfg["alphas"]
    log(f"grid8192 built in {time.time() - t0:.0f}s")
    rng = synth.streams(0, 3)[2]
    X = torch.from_numpy(synth.real_signals((N, 1024), rng).astype(np.float32)).to(dev)
    out = {"workload": "grid8192: 128x64 grid, lognormal(0, 0.5) weights, N=8192, L=64, 1024 orders in [-2, 2]",
           "forms": []}
    ev = lambda: torch.cuda.Event(enable_timing=True)
    for name in ("fp32", "fp16x2", "bf16x2", "complex64"):
        cplx = name == "complex64"
        st = "fp32" if cplx else name
        Ft = torch.from_numpy(F.astype(np.complex128) if cplx else F).to(dev)
        t0 = time.perf_counter()
        plan = Plan(Ft, L, stacktype=st)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        del Ft
        es = 8 if cplx else 4
        Q = torch.empty((max(chunks), N, N), dtype=torch.complex64, device=dev)
        for n in chunks:
            al = alphas[:n]
            plan.update(al, out=Q[:n])
            torch.cuda.synchronize()
            e0, e1 = ev(), ev()
            e0.record()
            for _ in range(reps):
                plan.update(al, out=Q[:n])
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            alg = n * 8.0 * N * N + (L + 2) * es * N * N
            row = {"stack": name, "orders": n, "update_ms": ms, "updates_per_s": n / (ms * 1e-3),
                   "algorithmic_GB": alg / 1e9, "algorithmic_GBps": alg / (ms * 1e-3) / 1e9, "plan_s": plan_s}
            if n == 32 and not cplx:
                Y = apply_operator(Q[:32], X)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(reps):
                    apply_operator(Q[:32], X, out=Y)
                e1.record()
                e1.synchronize()
                ams = e0.elapsed_time(e1) / reps
                flops = 32 * 4.0 * N * N * 1024      # complex Q times real X: 4 N^2 B flops per order
                row.update(apply_ms=ams, apply_signals=1024, apply_TFLOPs=flops / (ams * 1e-3) / 1e12)
                del Y
            log(f"precision form {row}")
            out["forms"].append(row)
        # all 1024 orders, launches of 128
        CH = 128
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        for c0 in range(0, alphas.size, CH):
            plan.update(alphas[c0: c0 + CH], out=Q[:CH])
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        nl = alphas.size // CH
        alg = alphas.size * 8.0 * N * N + nl * (L + 2) * es * N * N
        row = {"stack": name, "orders": int(alphas.size), "launches": nl, "pass_ms": ms,
               "updates_per_s": alphas.size / (ms * 1e-3), "algorithmic_GBps": alg / (ms * 1e-3) / 1e9}
        log(f"precision form {row}")
        out["forms"].append(row)
        del Q
        torch.cuda.empty_cache()
        if not cplx:   # the direct route on the same plan: 32 orders x 2 signals (64 columns, no operator formed)
            ms = direct_call_ms(plan, alphas[:32], 2, dev)
            alg = direct_algorithmic_bytes(N, L, 64)
            row = {"stack": name, "direct_orders": 32, "direct_columns": 64, "direct_ms": ms,
                   "direct_algorithmic_GBps": alg / (ms * 1e-3) / 1e9}
            log(f"precision form {row}")
            out["forms"].append(row)
        del plan
        torch.cuda.empty_cache()
    return out


SERVE_NS = (256, 512, 1024, 1024, 2048, 2048, 4096, 4096)


def realf_algorithmic_bytes(N, L, B, n_alpha):
    # update of R = Re Q: per order 4 N^2 written, plus (L+2) 4 N^2 of stack and projector read once
    # per call; apply: per order 4 N^2 of R read, 4 N B of x read and 8 N B of y written
    upd = n_alpha * 4.0 * N * N + (L + 2) * 4.0 * N * N
    app = n_alpha * (4.0 * N * N + 12.0 * N * B)
    return upd, app


def realf_bench(plan, alphas, X, reps=10):
    """The real-F route of the apply call on the main workload: one call forms R = Re Q for all
    orders (one update launch) and applies R X + j sin(pi alpha) W (W^T X) (one apply launch).
    Whole-call times from HIP events on the current stream, inputs resident."""
    import torch
    na, N, B = X.shape
    stream = torch.cuda.current_stream()
    Y = torch.empty((na, N, B), dtype=torch.complex64, device=X.device)
    ws = torch.empty(plan.apply_workspace_bytes(na, B, chunk=na), dtype=torch.uint8, device=X.device)
    for _ in range(2):
        plan.apply(alphas, X, chunk=na, out=Y, ws=ws)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.apply(alphas, X, chunk=na, out=Y, ws=ws)
        e1.record(stream)
        times.append((e0, e1))
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in times]))
    upd, app = realf_algorithmic_bytes(N, plan.L, B, na)
    del Y, ws
    torch.cuda.empty_cache()
    return {"workload": "the step's orders and signals through fgfrft_apply's real-F route (R = Re Q written as "
                        "float32, imaginary part sin(pi alpha) W (W^T X) from the rank-r_-1 basis)",
            "ms": ms, "updates_per_s": na / (ms * 1e-3), "signals_per_s": na * B / (ms * 1e-3),
            "algorithmic_GB": (upd + app) / 1e9, "algorithmic_GBps": (upd + app) / (ms * 1e-3) / 1e9,
            "hbm_frac": (upd + app) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def direct_algorithmic_bytes(N, L, ncols):
    # M_1..M_L and P read once, (L + 1) 4 N^2 (M_n^H is the same data), plus x read (4 N) and y
    # written (8 N) per column; wider calls stream the stack once per 64-column block
    return (L + 1) * 4.0 * N * N + 12.0 * N * ncols


def direct_bench(plan, alphas, dev, reps=10, sizes=((32, 2), (64, 1), (16, 16), (32, 64))):
    """Direct route (no operator formed) vs update + apply vs the apply call (fgfrft_apply: the real-F
    route when the signal count is a multiple of 64) for signal batches of one plan.

    Each case is (orders, signals per order); every route produces the same Y (complex64 [N, B] per
    order).  Times are per call, HIP events on the current stream, inputs resident."""
    import torch
    import synth
    from paper_2602_20870_amd import apply_operator

    N, L = plan.N, plan.L
    stream = torch.cuda.current_stream()
    rng = synth.streams(5, 1)[0]
    out = []
    for n, B in sizes:
        al = np.ascontiguousarray(alphas[:n])
        X = torch.from_numpy(synth.real_signals((n, N, B), rng).astype(np.float32)).to(dev)
        Xd = X.permute(1, 0, 2).reshape(N, n * B).contiguous()
        cols = torch.arange(n, dtype=torch.int32, device=dev).repeat_interleave(B)
        al_dev = torch.from_numpy(al).to(dev)
        Yd = torch.empty((N, n * B), dtype=torch.complex64, device=dev)
        ws = torch.empty(max(256, plan.direct_workspace_bytes(n * B, n * B)), dtype=torch.uint8, device=dev)
        Q = torch.empty((n, N, N), dtype=torch.complex64, device=dev)
        Ya = torch.empty((n, N, B), dtype=torch.complex64, device=dev)
        wsa = torch.empty(plan.apply_workspace_bytes(n, B, chunk=n), dtype=torch.uint8, device=dev)

        def apply_call():
            plan.apply(al, X, chunk=n, out=Ya, ws=wsa)

        def direct():
            plan.apply_direct(al_dev, cols, Xd, out=Yd, ws=ws)

        def two_step():
            plan.update(al, out=Q)
            return apply_operator(Q, X)

        res = {}
        for name, fn in (("direct", direct), ("update_apply", two_step), ("apply_call", apply_call)):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            res[name] = e0.elapsed_time(e1) / reps
        Y2 = two_step().permute(1, 0, 2).reshape(N, n * B)
        diff = float(torch.linalg.norm(Yd - Y2) / torch.linalg.norm(Y2))
        alg = direct_algorithmic_bytes(N, L, n * B)
        out.append({"orders": n, "signals_per_order": B, "ncols": n * B, "direct_ms": res["direct"],
                    "update_apply_ms": res["update_apply"], "speedup": res["update_apply"] / res["direct"],
                    "apply_call_ms": res["apply_call"], "apply_call_real_F_route": B % 64 == 0,
                    "direct_algorithmic_GB": alg / 1e9,
                    "direct_GBps": alg / (res["direct"] * 1e-3) / 1e9, "rel_diff_between_routes": diff})
        log(f"direct n={n} B={B}: {res['direct']:.3f} ms vs update+apply {res['update_apply']:.3f} ms, apply call "
            f"{res['apply_call']:.3f} ms "
            f"({alg / (res['direct'] * 1e-3) / 1e9:.0f} GB/s algorithmic, rel diff {diff:.1e})")
        del X, Xd, Yd, ws, Q, Y2, Ya, wsa
        torch.cuda.empty_cache()
    res = {"workload": f"knn4096 plan (N={N}, L={L}), real signals, orders from the main workload", "cases": out}
    # roofline of the direct route on the 64-column case: HIP events on this stream around the
    # whole call, i.e. k_direct plus its set-up kernels (column scales, coefficient table, signal
    # split) and the final reduction, about 50 us together; an upper bound on k_direct's time
    n, B = 32, 2
    ms = direct_call_ms(plan, alphas[:n], B, dev)
    ms_iso = direct_call_ms(plan, alphas[:n], B, dev, isolated=True)
    alg = direct_algorithmic_bytes(N, L, n * B)
    traffic = None
    if DIRECT_TRAFFIC["source_sha256"] == source_digest("direct.hip") and N == 4096 and L == 32:
        traffic = DIRECT_TRAFFIC["fetch_bytes"] + DIRECT_TRAFFIC["write_bytes"]
    res["roofline"] = {"bound": "hbm", "achieved": alg / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
                       "kernel": "k_direct (timed call includes its set-up and reduction kernels)",
                       "ms": ms, "isolated_call_ms": ms_iso, "ncols": n * B}
    log(f"direct call (64 columns): {ms:.3f} ms, {alg / (ms * 1e-3) / 1e9:.0f} GB/s algorithmic")
    return res


def direct_call_ms(plan, alphas, B, dev, reps=10, isolated=False):
    """Duration of one direct-route call (HIP events on the current stream): `reps` calls queued back to
    back between two events, so each call's kernels (column scales, coefficients, signal split, the
    paired kernel, the reduction) run without the host's launch gaps; isolated=True gives the median
    of single calls with a synchronisation after each instead."""
    import torch
    import synth
    N, n = plan.N, len(alphas)
    rng = synth.streams(6, 1)[0]
    Xd = torch.from_numpy(synth.real_signals((N, n * B), rng).astype(np.float32)).to(dev)
    cols = torch.arange(n, dtype=torch.int32, device=dev).repeat_interleave(B)
    al = torch.from_numpy(np.ascontiguousarray(alphas)).to(dev)
    Yd = torch.empty((N, n * B), dtype=torch.complex64, device=dev)
    ws = torch.empty(plan.direct_workspace_bytes(n * B, n * B), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        plan.apply_direct(al, cols, Xd, out=Yd, ws=ws)
    torch.cuda.synchronize()
    if not isolated:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            plan.apply_direct(al, cols, Xd, out=Yd, ws=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.apply_direct(al, cols, Xd, out=Yd, ws=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def serving_bench(n_requests=20000, warmup=2000, rate=5000.0, L=32, K=32, slot_sets=1, per_request=True,
                  warm_trace=4000, keep_every=16, route="auto", stacktype="fp32"):
    """p50/p99 latency of the continuous-batching server vs one launch per request.

    8 resident plans from kNN graphs (k=10, Gaussian weights) on 3-D GMM points with
    N in {256, 512, 1024, 1024, 2048, 2048, 4096, 4096}, L = 32; Poisson arrivals at
    `rate` requests/s; each request: graph uniform, order U[-2, 2], 1..64 real signals.
    After an untimed warm-up trace, `n_requests` are replayed and the first `warmup` of them
    are left out of the statistics.  The client keeps every `keep_every`-th result (compared
    between the two modes) and drops the rest as they complete.
    """
    import torch
    import synth
    from paper_2602_20870_amd import serve

    t0 = time.time()
    Fs = {g: synth.make_config("knn4096", seed=100 + g, N=N, with_signals=False)["F"]
          for g, N in enumerate(SERVE_NS)}
    rng = np.random.default_rng(7)
    sig = {g: rng.standard_normal((F.shape[0], 64)).astype(np.float32) for g, F in Fs.items()}
    srv = serve.Server(hbm_budget=120 << 30, K=K, bmax=64, slot_sets=slot_sets, use_graphs=True, route=route,
                       stacktype=stacktype)
    for g, F in Fs.items():
        srv.add_plan(g, F, L)
    torch.cuda.synchronize()
    log(f"serving: {len(Fs)} plans resident ({srv.used / 1e9:.1f} GB) in {time.time() - t0:.1f}s")
    if warm_trace:   # an untimed trace first: first-use costs of graphs, staging and caches
        serve.run_trace(srv, serve.poisson_trace(warm_trace, rate, list(Fs), 64, seed=10), sig, keep_every=keep_every)
    trace = serve.poisson_trace(n_requests, rate, list(Fs), 64, seed=11)
    batched = serve.run_trace(srv, trace, sig, warmup=warmup, keep_every=keep_every)
    out = {"batched": batched, "rate_req_s": rate, "requests": n_requests, "warmup": warmup,
           "plans_N": list(SERVE_NS), "L": L, "K": K, "slot_sets": slot_sets, "route": route}
    kept = batched.pop("kept")
    if per_request:
        # baseline: the same route choice for a batch of one, preallocated buffers and captured graphs,
        # one launch per request, nothing coalesced or overlapped; at the offered rate, then at 80% of
        # the rate it sustained (a load it can keep up with), where the batched server is run again
        one = serve.run_trace_one_launch(srv.plans, trace, sig, warmup=warmup, keep_every=keep_every)
        outs = one.pop("outputs")
        worst = 0.0
        for i, f in kept:
            r, y = f.result(), outs[i]
            worst = max(worst, float(np.linalg.norm(r - y) / max(np.linalg.norm(y), 1e-30)))
        out["one_launch_per_request"] = one
        out["max_rel_diff_between_modes"] = worst
        out["results_compared"] = len(kept)
        log(f"serve one launch per request at {rate:.0f} req/s: p50 {one['p50_ms']:.2f} ms p99 {one['p99_ms']:.2f} ms, "
            f"sustained {one['throughput_req_s']:.0f} req/s")
        low = 0.8 * min(one["throughput_req_s"], rate)
        n_low = int(min(n_requests, max(4000, 4 * low)))
        trace2 = serve.poisson_trace(n_low, low, list(Fs), 64, seed=12)
        b2 = serve.run_trace(srv, trace2, sig, warmup=min(warmup, n_low // 10), keep_every=keep_every)
        b2.pop("kept")
        o2 = serve.run_trace_one_launch(srv.plans, trace2, sig, warmup=min(warmup, n_low // 10), keep_every=n_low)
        o2.pop("outputs")
        out["at_sustainable_rate"] = {"rate_req_s": low, "requests": n_low, "batched": b2, "one_launch_per_request": o2}
        log(f"serve at {low:.0f} req/s: batched p50 {b2['p50_ms']:.2f} / p99 {b2['p99_ms']:.2f} ms, one launch per "
            f"request p50 {o2['p50_ms']:.2f} / p99 {o2['p99_ms']:.2f} ms")
    del srv
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-alpha", type=int, default=256)
    ap.add_argument("--signals", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stacktype", default="fp16x2", choices=["fp32", "fp16x2", "bf16x2"],
                    help="stack storage of the plans (fp16x2: the FP32 stack's split operands, bitwise the "
                         "FP32 results)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving p50/p99 measurement")
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient timing")
    ap.add_argument("--no-direct", action="store_true", help="skip the direct-route comparison")
    ap.add_argument("--no-configs", action="store_true", help="skip the grid1024 / dft256 throughput leg")
    ap.add_argument("--precision-form", action="store_true",
                    help="only the precision-form workload (grid8192, N = 8192, L = 64, FP32 and BF16X2 stacks)")
    ap.add_argument("--table4", action="store_true",
                    help="only the Table IV workload (FGFRFT vs exact GFRFT online time, N = 1000..8000)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    from paper_2602_20870_amd import Plan, apply_operator, lib

    lib()  # fail loudly if the HIP library is missing
    if args.table4:
        print(json.dumps({"table4": table4_bench()}), flush=True)
        return
    if args.precision_form:
        print(json.dumps({"precision_form": precision_form_bench()}), flush=True)
        return
    dev = torch.device("cuda:0")
    t0 = time.time()
    cfg = synth.make_config("knn4096", seed=0, n_alpha=args.n_alpha, with_signals=False)
    F, L, N = cfg["F"], cfg["L"], cfg["N"]
    alphas = cfg["alphas"]
    B, na = args.signals, args.n_alpha
    rng = synth.streams(0, 3)[2]
    X_host = synth.real_signals((na, N, B), rng).astype(np.float32)
    X = torch.from_numpy(X_host).to(dev)
    log(f"workload built in {time.time() - t0:.1f}s (N={N}, L={L}, n_alpha={na}, B={B})")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = Plan(torch.from_numpy(F).to(dev), L, stacktype=args.stacktype)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan.info()
    log(f"plan {plan_s:.2f}s {info}")

    Q = torch.empty((na, N, N), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(times=None):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(stream)
        plan.update(alphas, out=Q)
        e1.record(stream)
        Y = apply_operator(Q, X)
        e2.record(stream)
        if times is not None:
            times.append((e0, e1, e2))
        return Y

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(times)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    upd_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in times]))
    app_ms = float(np.mean([b.elapsed_time(c) for _, b, c in times]))
    ms_step = wall * 1e3 / args.steps
    log(f"update {upd_ms:.3f} ms, apply {app_ms:.3f} ms, step {ms_step:.3f} ms")

    upd_bytes = update_algorithmic_bytes(N, L, na)
    achieved = upd_bytes / (upd_ms * 1e-3) / 1e9
    app_gbs = apply_algorithmic_bytes(N, B, na) / (app_ms * 1e-3) / 1e9
    out = {
        "metric": "F^alpha updates/s (update + apply to 64 signals per order), N=4096, L=32; serve p50/p99",
        "value": na / (ms_step * 1e-3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32 (split fp16 MFMA operands, fp32 accumulate)",
                  "fp16x2": "f32 (stack stored as its split fp16 MFMA operands, fp32 accumulate)",
                  "bf16x2": "bf16x2"}[args.stacktype],
        "data": "synthetic",
        "config": {"workload": "knn4096: kNN k=10 on 5-GMM 3-D points, N=4096, L=32, 256 orders in [-2,2], "
                               "64 real N(0,1) signals per order", "n_alpha": na, "signals_per_order": B,
                   "stacktype": args.stacktype},
        "signals_per_s": na * B / (ms_step * 1e-3),
        "update": {"ms": upd_ms, "updates_per_s": na / (upd_ms * 1e-3), "algorithmic_GB": upd_bytes / 1e9},
        "apply": {"ms": app_ms, "algorithmic_GBps": app_gbs, "hbm_frac": app_gbs / HBM_PEAK_GBS},
        "plan_s": plan_s,
        "plan_info": info,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": update_traffic(), "kernel": "k_update"},
    }
    del Q
    torch.cuda.empty_cache()

    def leg(name, fn):
        """A secondary measurement: its failure is recorded in the line, never loses the line."""
        try:
            out[name] = fn()
        except Exception as e:          # noqa: BLE001
            import traceback
            traceback.print_exc()
            out[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.synchronize()
            torch.cuda.empty_cache()

    if plan.info()["r_minus1"] <= 32:
        leg("real_F_route", lambda: realf_bench(plan, alphas, X))
        if "ms" in out["real_F_route"]:
            r = out["real_F_route"]
            log(f"real-F route {r['ms']:.3f} ms per step ({r['signals_per_s'] / 1e6:.2f}M signals/s, "
                f"{r['algorithmic_GBps']:.0f} GB/s algorithmic)")
    del X
    torch.cuda.empty_cache()
    if not args.no_direct:
        leg("direct", lambda: direct_bench(plan, alphas, dev))
    leg("copy_reference", lambda: copy_bandwidth(dev))
    if "GBps" in out["copy_reference"]:
        log(f"plain copy {out['copy_reference']['GBps']:.0f} GB/s")
    leg("write_reference", lambda: write_bandwidth(dev))
    if "GBps" in out["write_reference"]:
        w = out["write_reference"]["GBps"]
        out["roofline"]["attainable_write_GBps"] = w
        out["roofline"]["frac_of_attainable_write"] = achieved / w
        log(f"write-only stream {w:.0f} GB/s; update at {achieved / w:.2f} of it")
    leg("update_traffic_reference", lambda: update_traffic_reference(dev, N, L, na))
    if "ms" in out["update_traffic_reference"]:
        t = out["update_traffic_reference"]["ms"]
        out["roofline"]["attainable_GBps"] = upd_bytes / (t * 1e-3) / 1e9
        out["roofline"]["frac_of_attainable"] = t / upd_ms
        log(f"update traffic alone {t:.3f} ms; update at {t / upd_ms:.2f} of it")
    if not args.no_configs:
        leg("throughput_configs", throughput_configs)
    if not args.no_grad:
        log("gradients ...")
        # the gradient takes FP32-class stacks (FP32 or FP16X2)
        leg("grad", lambda: grad_bench(stacktype="fp32" if args.stacktype == "bf16x2" else args.stacktype))
        log(f"grad {out['grad']}")
    del plan
    torch.cuda.empty_cache()
    if not args.no_serve:
        log("serving trace ...")
        leg("serve", lambda: serving_bench(stacktype=args.stacktype))
        if "batched" in out["serve"]:
            b, p = out["serve"]["batched"], out["serve"].get("one_launch_per_request")
            log(f"serve batched p50 {b['p50_ms']:.2f} ms p99 {b['p99_ms']:.2f} ms"
                + (f"; per-request p50 {p['p50_ms']:.2f} ms p99 {p['p99_ms']:.2f} ms" if p else ""))
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        leg("cpu_baseline", lambda: cpu_baseline(F, alphas, L, X_host))
        log(f"cpu baseline {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
