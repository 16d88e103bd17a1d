#!/usr/bin/env python3
"""Benchmark of the decoupled multicontinuum time step on one MI355X.

Workload (default): the two-continuum fractured medium on a 2048 x 2048 grid (lognormal
matrix permeability, 400 any-angle fracture segments, ~63k fracture cells), tau = 1e-3,
100 backward-Euler time layers, D-scheme with per-continuum PCG to 1e-10, FP64.

One "step" = one time layer of the whole hot path: transfer right-hand side assembly for
every continuum plus every PCG iteration of every continuum.  The timed region starts with
all inputs resident on the GPU and the state reset to the initial pressure, and covers
exactly `--steps` layers.  Printed: one JSON line (metric, value = cell-updates/s, ...)
with the roofline of the dominant kernel, the coupled-FP64 comparison on the same GPU,
p50/p99 step latency, accuracy against stored oracle values, and the CPU oracle baseline.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("cell-updates/s per decoupled time step vs coupled+FP64 at 1e-8 rel err; "
          "p50/p99 step latency")
HBM_PEAK_GBS = 8000.0

# HBM bytes per dispatch of the grid operator kernel, from two rocprofv3 counter passes
# (FETCH_SIZE, then WRITE_SIZE) of `bench.py --steps 2 --warmup 0 --no-cpu --no-coupled
# --calibrate-copy 4096`, each scaled by what the same counter reads for a 2 GiB sum (read
# factor 1.9999) and a 2 GiB fill (write factor 0.9999).  Valid only for the kernel sources
# they were taken on (hash of kernels.hpp + common.hpp); otherwise traffic is reported null.
MEASURED_TRAFFIC = {
    ("C2", "bic0"): {"sources": "7be7f8b36faa832f", "fetch_kib": 84047.2, "write_kib": 65600.4,
                     "read_factor": 1.9999, "write_factor": 0.9999},
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def grid_A_bytes_per_cell(precision, precond, has_t):
    """Algorithmic bytes the grid operator kernel (p_new = z + beta p_old, q = A p_new,
    partial (p,q)) must move per cell: read r (or z), p_old, diag [, tx, ty]; write p_new,
    q; Jacobi reads diag once for both z and the operator."""
    w = 8 if precision == "fp64" else 4
    reads = 3 + (2 if has_t else 0)
    writes = 2
    return (reads + writes) * w


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2209_01158_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precond):
    m = MEASURED_TRAFFIC.get((workload, precond))
    if m is None or m["sources"] != kernel_sources_hash():
        return None
    return (m["fetch_kib"] * m["read_factor"] + m["write_kib"] * m["write_factor"]) * 1024.0


def golden_check(g, name, steps, scheme):
    path = os.path.join(ROOT, "tests", "golden", f"{name.lower()}_oracle.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    if steps not in list(z[f"steps_{scheme}"]):
        return None
    num = den = 0.0
    maxrel = 0.0
    for a in range(g.n_cont):
        st = g.get_state(a)
        idx = z[f"idx{a}"]
        ref = z[f"{scheme}_s{steps}_c{a}"]
        d = st[idx] - ref
        num += float(d @ d)
        den += float(ref @ ref)
        maxrel = max(maxrel, float(np.max(np.abs(d)) / max(np.max(np.abs(ref)), 1e-300)))
    return dict(rel_l2_sampled=float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num)),
                max_abs_over_max=maxrel, reference=os.path.relpath(path, ROOT),
                sample=f"{len(z['idx0'])} seeded cells per continuum, step {steps}")


def cpu_baseline(n_cpu=1024, steps=5):
    """The CPU oracle (SuperLU, one core) on a bounded sample of the workload's recipe."""
    import media
    from oracle import schemes
    p = media.configs._c2(n=n_cpu, nseg=max(1, 400 * n_cpu // 2048))
    t0 = time.perf_counter()
    st = schemes.Stepper(p, None, "D")
    t1 = time.perf_counter()
    x = p.initial_state()
    for _ in range(steps):
        x = st.step(x)
    t2 = time.perf_counter()
    dof = p.dof()
    return {"value": dof * steps / (t2 - t1), "unit": "cell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"C2 recipe at {n_cpu}x{n_cpu} ({p.nf} fracture cells), D-scheme, "
                       f"{steps} steps after a one-time sparse LU factorization "
                       f"({t1 - t0:.1f} s, excluded; including it: "
                       f"{dof * steps / (t2 - t0):.3g} cell-updates/s); SuperLU is sequential"),
            "host_cpu": platform.processor() or platform.machine(),
            "host_cpu_count": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--precond", default="bic0")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--coupled-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-coupled", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB written by a fill and read by a sum (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import media
    from paper_2209_01158_amd import mcdec
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()

    t = time.time()
    p = media.config_problem(args.workload)
    log(f"workload {args.workload}: {p.nx}x{p.ny}, nf={p.nf}, dof={p.dof()} "
        f"(generated in {time.time() - t:.1f}s)")
    dof = p.dof()
    p0 = p.initial_state()

    with torch.cuda.stream(stream):
        t = time.time()
        g = mcdec.Problem(p, scheme="D", precision="fp64", precond=args.precond, tol=args.tol,
                          stream=stream.cuda_stream)
        inf = g.info()
        log(f"setup {time.time() - t:.2f}s, device memory {inf.device_bytes / 2**20:.0f} MiB")
        for k in range(args.warmup):
            rep = g.step(1)
            log(f"warmup step {k + 1}: iters {rep['iters']}, {rep['seconds'] * 1e3:.2f} ms")
        g.set_states(p0)
        g.profile(True)
        lat = []
        iters = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ts = time.perf_counter()
            rep = g.step(1)
            lat.append(time.perf_counter() - ts)
            iters.append(rep["iters"])
            if (k + 1) % 20 == 0:
                log(f"step {k + 1}/{args.steps}: iters {rep['iters']}")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        nA, msA = g.profile_read(0)
        nB, msB = g.profile_read(1)
        g.profile(False)
        elapsed = t1 - t0
        value = dof * args.steps / elapsed
        acc = golden_check(g, args.workload, args.steps, "D")
        log(f"decoupled: {value:.4g} cell-updates/s, {elapsed / args.steps * 1e3:.3f} ms/step")

        coupled = None
        if not args.no_coupled and args.coupled_steps > 0:
            g.set_options(scheme="coupled")
            g.set_states(p0)
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            citers = []
            for k in range(args.coupled_steps):
                rep = g.step(1)
                citers.append(rep["iters"][0])
                log(f"coupled step {k + 1}: iters {rep['iters'][0]}")
            torch.cuda.synchronize()
            c1 = time.perf_counter()
            cval = dof * args.coupled_steps / (c1 - c0)
            cacc = golden_check(g, args.workload, args.coupled_steps, "coupled")
            coupled = {"value": cval, "unit": "cell-updates/s", "steps": args.coupled_steps,
                       "ms_per_step": (c1 - c0) / args.coupled_steps * 1e3,
                       "pcg_iters_per_step": float(np.mean(citers)),
                       "decoupled_over_coupled": value / cval, "accuracy": cacc}
        g.close()
        if args.calibrate_copy:
            # known traffic for the HBM counters: a fill writes N bytes, a sum reads N bytes
            n = args.calibrate_copy * 2**20 // 8
            src = torch.full((n,), 1.0, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            tot = float(src.sum())
            torch.cuda.synchronize()
            log(f"calibration: filled and summed {args.calibrate_copy} MiB (sum {tot:.0f})")

    lat_ms = np.array(lat) * 1e3
    it = np.array(iters)
    ncell_grid = p.nx * p.ny * p.n_omega
    has_t = any(o.k is not None for o in p.omega)
    bpc = grid_A_bytes_per_cell("fp64", args.precond, has_t)
    avgA = msA / max(nA, 1) * 1e-3
    achieved = ncell_grid * bpc / avgA / 1e9 if nA else None
    pname = {"bic0": "BIC0", "jacobi": "JACOBI"}.get(args.precond, args.precond)
    traffic = measured_traffic(args.workload, args.precond)
    roof = {"bound": "hbm", "kernel": f"k_pcg_A<double,{pname},GRID> (p = z + beta p; q = A p; "
            "partial p.q), grid continuum", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic, "traffic_unit": "bytes per launch",
            "algorithmic_bytes_per_launch": ncell_grid * bpc,
            "bytes_per_cell": bpc, "cells_per_launch": ncell_grid, "launches": nA,
            "avg_launch_us": avgA * 1e6,
            "update_kernel_avg_us": msB / max(nB, 1) * 1e3, "update_kernel_launches": nB}
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: two-continuum {p.nx}x{p.ny} lognormal "
                   f"matrix + {p.nf} fracture cells, tau={p.tau}, D-scheme FP64, "
                   f"PCG {args.precond} tol {args.tol}", "dof": dof,
                   "precond": args.precond, "scheme": "D", "precision": "fp64"},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99)),
                       "max": float(lat_ms.max())},
        "pcg_iters_per_step": {"mean": it.mean(axis=0).tolist(), "max": it.max(axis=0).tolist()},
        "accuracy_vs_oracle": acc,
        "coupled_fp64": coupled,
        "roofline": roof,
    }
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
