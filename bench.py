#!/usr/bin/env python3
"""Benchmark of the decoupled multicontinuum time step on one MI355X.

Workloads (``--workload``):
  C2 (default)  two-continuum fractured medium on a 2048 x 2048 grid (lognormal matrix
                permeability, 400 any-angle fracture segments, ~63k fracture cells),
                tau = 1e-3, 100 backward-Euler layers, D-scheme, FP64 PCG to 1e-10 with the
                multigrid V-cycle on the grid and the exact fracture solve.
  C1            64 x 64 two-continuum medium, 20 layers, Jacobi PCG to 1e-12 (latency-bound).
  C3            three continua on a 4096 x 4096 grid (~150k fracture cells), 50 layers,
                FP32 inner PCG (V-cycle) inside FP64 refinement to 1e-10.
  C4            256 independent realizations of uneven size (128..1024 cells a side, two or
                three continua), 50 layers, all advanced by shared launches in FP32 inner PCG
                inside FP64 refinement.
  3D            the 3-D extension: two continua on a 256 x 256 x 256 grid of cubes (lognormal
                matrix permeability per plane, 40 fracture planes), 20 layers, D-scheme,
                FP64 block IC(0) PCG to 1e-10.
  NLMC          the coarse-grid NLMC schemes on the paper's 2C / 3C problems (200 x 200 with
                wells) on 20 x 20 and 40 x 40 coarse grids: basis set-up, coarse layers of
                every scheme, e_H against the fine coupled solution.
  C5            serving: a seeded Poisson trace of simulation requests (mean 40/s, sides
                64..2048, 10..500 layers each) replayed in real time against the server
                (admission by device-memory footprint, continuous batching); a "step" there is
                one server step (one layer of every resident request).

One "step" = one time layer of the whole hot path for the whole workload: transfer
right-hand-side assembly of every continuum plus every PCG iteration (and refinement pass)
of every continuum.  The timed region starts with all inputs resident on the GPU and the
state reset to the initial pressure, and covers exactly `--steps` layers.  Printed: one JSON
line (metric, value = cell-updates/s, ...) with the roofline of the dominant kernel (HIP
events bound to sampled dispatches inside the timed region), the coupled-FP64 comparison on
the same GPU, p50/p99 step latency, accuracy against stored oracle values, and the CPU
oracle baseline on a bounded sample.
"""
import argparse
import hashlib
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

DEFAULTS = {
    "C1": dict(precond="jacobi", precision="fp64", tol=1e-12, steps=20, coupled_steps=20,
               small_max=8192),
    "C2": dict(precond="mg", precision="fp64", tol=1e-10, steps=100, coupled_steps=5),
    # (C3: inner FP32 solves to 1e-3 relative take fewer iterations in all than to 1e-4, at
    # one more refinement pass: 13.4 against 14.7 ms per layer)
    "C3": dict(precond="mg", precision="mixed", tol=1e-10, steps=50, coupled_steps=1,
               sample_every=4, inner_tol=1e-3),
    "C4": dict(precond="mg", precision="mixed", tol=1e-10, steps=50, coupled_steps=2,
               sample_every=4, autotune=True),
    "C5": dict(precond="mg", precision="mixed", tol=1e-10, steps=0, coupled_steps=0),
    "3D": dict(precond="bic0", precision="fp64", tol=1e-10, steps=20, coupled_steps=2,
               sample_every=2),
    "NLMC": dict(precond="mg", precision="fp64", tol=1e-12, steps=50, coupled_steps=0),
}

# HBM bytes per dispatch of the grid PCG kernels, from two rocprofv3 counter passes
# (FETCH_SIZE, then WRITE_SIZE) of `bench.py --steps 2 --warmup 0 --no-cpu --no-coupled
# --calibrate-copy 4096`, each scaled by what the same counter reads for a 2 GiB sum (read
# factor 1.9999) and a 2 GiB fill (write factor 1.0).  Valid only for the kernel sources
# they were taken on (hash of kernels.hpp + common.hpp); otherwise traffic is reported null.
MEASURED_TRAFFIC = {
    ("C2", "mg", "A"): {"sources": "92bffb5b6cc8c44b", "fetch_kib": 83653.5,
                        "write_kib": 65552.7, "read_factor": 1.9999, "write_factor": 1.0},
    ("C2", "mg", "B"): {"sources": "92bffb5b6cc8c44b", "fetch_kib": 110852.7,
                        "write_kib": 107788.8, "read_factor": 1.9999, "write_factor": 1.0},
    ("C2", "mg", "P"): {"sources": "92bffb5b6cc8c44b", "fetch_kib": 81977.1,
                        "write_kib": 32848.1, "read_factor": 1.9999, "write_factor": 1.0},
}

def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in ("kernels.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2209_01158_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precond, kernel):
    m = MEASURED_TRAFFIC.get((workload, precond, kernel))
    if m is None or m["sources"] != kernel_sources_hash():
        return None
    return (m["fetch_kib"] * m["read_factor"] + m["write_kib"] * m["write_factor"]) * 1024.0


def grid_bytes_per_cell(kernel, precision, precond, has_t, dim=2, fused=False):
    """Algorithmic bytes a grid PCG kernel must move per cell (w = 4 or 8 byte words).

    A (operator): read z (Jacobi: r), p_old, diag [, tx, ty] [3-D: tz]; write p_new, q.
    B (update):   read x, p, r, q; write x, r; Jacobi also reads diag (z = r / diag is
                  recomputed where needed, never stored); block IC(0) reads the FP32 copies
                  of the inverse pivots and of tx, ty (4 bytes each) and writes z (under mg
                  the same sweep is the finest pre-smoothing and writes z_p).  Fused with the
                  restriction into level 1 (mg, level 1 above the tail) it also reads the
                  FP32 diagonal and writes the in-block part of r_c (one word per 2 x 2
                  cells) and the block edges (two words and 4 B per 64 cells).
    P (mg: finest correction + post-smoothing): read z_p, r, the coarse correction e (one
                  word per 2 x 2 cells), the FP32 diagonal, the FP32 inverse pivots [and
                  FP32 tx, ty, shared by the residual and the sweep]; write z."""
    w = 4 if precision == "mixed" else 8
    if kernel == "A":
        return (3 + (2 if has_t else 0) + (1 if dim == 3 else 0) + 2) * w
    if kernel == "P":
        return 3 * w + w / 4 + (2 + (2 if has_t else 0)) * 4
    if precond in ("bic0", "mg"):
        return 7 * w + 3 * 4 + ((4 + w / 4 + (2 * w + 4) / 64) if fused else 0.0)
    return 7 * w


def mg_fused(nx, ny, nlev=None, dim=2, precision="fp64"):
    """The update kernel forms the finest level's in-block share of the restriction into
    level 1 (FP64 solves of 2-D V-cycles whose level 1 is above the tail; MCDEC_MG_FUSE=0
    turns it off)."""
    if dim != 2 or precision != "fp64" or os.environ.get("MCDEC_MG_FUSE", "1") == "0":
        return False
    lv = mg_levels(nx, ny)
    if len(lv) < 2 or (nlev is not None and nlev < 1):
        return False
    return lv[1][0] * lv[1][1] > MG_TAIL


MG_COARSE, MG_TAIL = 256, 1024   # coarsest level size; levels of at most MG_TAIL cells: tail


def mg_levels(nx, ny):
    """Grid shapes of the V-cycle levels: 2 x 2 aggregation until at most MG_COARSE cells."""
    out = [(nx, ny)]
    while nx * ny > MG_COARSE:
        nx, ny = (nx + 1) // 2, (ny + 1) // 2
        out.append((nx, ny))
    return out


def vcycle_bytes(nx, ny, precision, has_t, nlev=None, fused=False, once=False):
    """Algorithmic bytes of one V-cycle's coarse kernels (all levels), per timing slot.

    RS (restriction into coarse level l with its pre-smoothing, every level above the tail):
        per cell of level l-1 read r, z_p (2 words) and the FP32 diagonal [, tx, ty] (4 B
        each; level 0 without a conductance field: the diagonal only); per cell of level l
        write r_c, z_p (2 words) and read its FP32 inverse pivots, tx, ty (12 B).  Into a
        fused level 1 (the update kernel summed the in-block part of r_c): per cell of
        level 1 read and write r_c, write z_p (3 words), read its factor (12 B), plus the
        finest row next to a block edge (a word and 4 B per fine column, one fine row in 8)
        and the block edges (3 per 128 fine columns, a word and 4 B per fine row).
    PC (correction + post-smoothing at level l, levels above the tail except the finest):
        read z_p, r, e (one word per 2 x 2 cells), FP32 diagonal, pivots, tx, ty; write z:
        3 words + w / 4 + 16 B per cell.
    R  (restriction into the tail's first level): the finer level's r, z_p, FP32 diagonal,
        tx, ty read, r_c written.
    TAIL (levels of at most MG_TAIL cells in one workgroup): counted as R's output only;
        it is latency-bound.
    once: the last level of a truncated hierarchy is smoothed once (no PC launch there)."""
    w = 4 if precision == "mixed" else 8
    lv = mg_levels(nx, ny)
    if nlev is not None:               # a hierarchy truncated above the tail
        lv = lv[:nlev + 1]
    n = [a * b for a, b in lv]
    rs = pc = r = 0.0
    for l in range(1, len(lv)):
        fine_coef = (12 if (l > 1 or has_t) else 4)
        if n[l] > MG_TAIL and l == 1 and fused:
            rs += n[l] * (3 * w + 12 + (w + 4) / 2 + 24 * (w + 4) / 256)
            pc += n[l] * (3 * w + w / 4 + 16)
        elif n[l] > MG_TAIL:
            rs += n[l - 1] * (2 * w + fine_coef) + n[l] * (2 * w + 12)
            if not (once and l == len(lv) - 1):
                pc += n[l] * (3 * w + w / 4 + 16)
        elif n[l - 1] > MG_TAIL or l == 1:
            r += n[l - 1] * (2 * w + fine_coef) + n[l] * w
    return {"RS": rs, "PC": pc, "R": r, "TAIL": 0.0}


KERNEL_NAMES = {
    "A": "k_pcg_A<{tp},{pn},GRID> (p = z + beta p; q = A p; partial p.q)",
    "B": "k_pcg_B<{tp},{pn},GRID> (x += alpha p; r -= alpha q; z = M^-1 r; partial r.z, r.r)",
    "P": "k_mg_post<{tp},FINAL> (z = z_p + P e + M^-1 (r - A (z_p + P e)); partial r.z)",
    "RS": "k_mg_restrict_smooth<{tp}> / k_mg_fix_smooth<{tp}> (all coarse levels: r_c = P^T "
          "(r - A z_p); z_p = M^-1 r_c; level 1 of an FP64 solve completes the update kernel's "
          "in-block restriction)",
    "PC": "k_mg_post_c<{tp}> (all coarse levels: z = z_p + P e + M^-1 (r - A (z_p + P e)))",
    "TAIL": "k_mg_tail<{tp}> (levels of <= 1024 cells and the dense coarsest solve, one "
            "workgroup)",
    "R": "k_mg_restrict<{tp}> (restriction into the tail's first level)",
}


def roofline(kind_time, bytes_total, precision, precond, workload, working=None):
    """Roofline objects of every timed grid kernel: the operator (A), update (B) and, with
    the V-cycle, the finest post-smoothing (P) and the coarse kernels summed over their
    levels (RS, PC, TAIL, R); the one with the most total time is the dominant kernel.

    kind_time[k] = (sampled, summed ms, issued, working sampled, working summed ms), where the
    working samples are those of at least a quarter of the mean sample (the others are
    launches whose systems had all converged; they return at once and move no bytes).
    working[k]: launches that did work, counted from the iterations the timed layers took
    (a launch of the group's systems works while any of them still iterates); without it,
    issued x working share of the samples.  Total time = mean working sample x working
    launches; achieved = algorithmic bytes of the timed layers / total time; the average
    launch duration is the mean working sample."""
    out = {}
    for k, (sampled, ms, issued, wn, wms) in kind_time.items():
        if not sampled or not wn:
            continue
        avg_s = wms / wn * 1e-3
        work = working.get(k) if working else None
        working_k = work if work else issued * wn / sampled
        total_s = avg_s * working_k
        per_launch = bytes_total[k] / max(working_k, 1)
        achieved = bytes_total[k] / total_s / 1e9 if total_s > 0 else 0.0
        tp = "float" if precision == "mixed" else "double"
        pn = {"bic0": "BIC0", "mg": "BIC0", "jacobi": "JACOBI"}[precond]
        name = KERNEL_NAMES[k].format(tp=tp, pn=pn)
        bound = "latency" if k == "TAIL" else "hbm"
        out[k] = {"bound": bound, "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                  "traffic": measured_traffic(workload, precond, k),
                  "traffic_unit": "bytes per launch",
                  "algorithmic_bytes_per_launch": per_launch,
                  "avg_launch_us": avg_s * 1e6, "sampled_launches": sampled,
                  "sampled_working_launches": wn, "issued_launches": issued,
                  "working_launches": working_k,
                  "all_samples_avg_us": ms / sampled * 1e3,
                  "total_ms_est": total_s * 1e3}
    if not out:
        return None, None
    order = sorted(out, key=lambda k: -out[k]["total_ms_est"])
    return out[order[0]], [out[k] for k in order[1:]]


def golden_states(states_of, name, step, scheme):
    """Relative L2 error on the stored oracle sample: states_of(a) -> state of continuum a."""
    path = os.path.join(ROOT, "tests", "golden", f"{name.lower()}_oracle.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    if step not in list(z[f"steps_{scheme}"]):
        return None
    num = den = 0.0
    a = 0
    while f"idx{a}" in z:
        idx = z[f"idx{a}"]
        ref = z[f"{scheme}_s{step}_c{a}"]
        d = states_of(a)[idx] - ref
        num += float(d @ d)
        den += float(ref @ ref)
        a += 1
    return dict(rel_l2_sampled=float(np.sqrt(num / den)), step=step, scheme=scheme,
                reference=os.path.relpath(path, ROOT),
                sample=f"{len(z['idx0'])} seeded cells per continuum")


def golden_c4(handles, step, scheme):
    """Per-problem relative L2 error on the stored oracle samples of six realizations."""
    path = os.path.join(ROOT, "tests", "golden", "c4_oracle.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    if step not in list(z[f"steps_{scheme}"]):
        return None
    per = {}
    for i in z["problems"]:
        i = int(i)
        num = den = 0.0
        a = 0
        while f"p{i}_idx{a}" in z:
            ref = z[f"p{i}_{scheme}_s{step}_c{a}"]
            d = handles[i].get_state(a)[z[f"p{i}_idx{a}"]] - ref
            num += float(d @ d)
            den += float(ref @ ref)
            a += 1
        per[str(i)] = float(np.sqrt(num / den))
    return dict(rel_l2_sampled_max=max(per.values()), per_problem=per, step=step,
                scheme=scheme, reference=os.path.relpath(path, ROOT))


def cpu_baseline(workload):
    """The CPU oracle (SuperLU, one core) on a bounded sample of the workload's recipe;
    rate per layer excludes the one-time factorization (reported beside it)."""
    import media
    from oracle import schemes
    if workload == "C1":
        probs, steps, what = [media.config_problem("C1")], 20, "the full C1 workload"
    elif workload == "C2":
        probs, steps = [media.configs._c2(n=1024, nseg=200)], 5
        what = "C2 recipe at 1024x1024 (200 segments)"
    elif workload == "C3":
        probs, steps = [media.configs._c3(n=1024, min_cells=150_000 // 16)], 3
        what = "C3 recipe at 1024x1024 (three continua)"
    elif workload == "3D":
        probs, steps = [media.configs._3d(n=32, nz=32)], 20
        what = "3-D recipe at 32x32x32 (sparse LU of 3-D systems fills in fast)"
    else:
        probs, steps = media.configs.c4_problems(only=[55, 212]), 10
        what = "realizations 55 and 212 of the batched workload"
    tf = ts = 0.0
    dof = 0
    for p in probs:
        t0 = time.perf_counter()
        st = schemes.Stepper(p, None, "D")
        t1 = time.perf_counter()
        x = p.initial_state()
        for _ in range(steps):
            x = st.step(x)
        t2 = time.perf_counter()
        tf += t1 - t0
        ts += t2 - t1
        dof += p.dof()
    return {"value": dof * steps / ts, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": (f"{what}, D-scheme, {steps} layers after a one-time sparse LU "
                       f"factorization ({tf:.1f} s, excluded; including it: "
                       f"{dof * steps / (ts + tf):.3g} cell-updates/s); SuperLU is sequential"),
            "host_cpu": platform.processor() or platform.machine(),
            "host_cpu_count": os.cpu_count()}


def read_profile(h, kernels):
    """(sampled, ms, issued, working sampled, working ms) per timed kernel of handle h."""
    out = {}
    for i, k in enumerate(kernels):
        n, ms, iss = h.profile_read(i)
        wn, wms = h.profile_read_above(i, 0.25 * ms / n) if n else (0, 0.0)
        out[k] = (n, ms, iss, wn, wms)
    return out


def kernels_of(precond):
    """Timed grid kernels, in the library's profile order (0 = A, 1 = B, 2 = P, then the
    V-cycle's coarse kernels 3 = RS, 4 = PC, 5 = TAIL, 6 = R)."""
    return ("A", "B", "P", "RS", "PC", "TAIL", "R") if precond == "mg" else ("A", "B")


def step_bytes(p, rep, precision, precond, nlev=None, once=None):
    """Algorithmic bytes of every timed grid kernel for one layer of problem p (iterations
    x cells x bytes per cell; the V-cycle's coarse kernels per cycle from the level
    shapes; nlev[c]: coarse levels of continuum c's hierarchy, once[c]: its truncated last
    level smoothed once)."""
    out = {k: 0.0 for k in kernels_of(precond)}
    dim = getattr(p, "dim", 2)
    for c in range(p.n_omega):
        has_t = p.omega[c].k is not None or dim == 3
        it = rep["iters"][c]
        nl = None if nlev is None else nlev[c]
        fused = precond == "mg" and mg_fused(p.nx, p.ny, nl, dim, precision)
        for k in ("A", "B", "P"):
            if k in out:
                out[k] += it * p.ncell * grid_bytes_per_cell(k, precision, precond, has_t, dim,
                                                             fused)
        if precond == "mg":
            vb = vcycle_bytes(p.nx, p.ny, precision, has_t, nl, fused,
                              bool(once and once[c]))
            for k, b in vb.items():
                out[k] += it * b
    return out


def working_launches(iter_rows, precond, nlevs, shapes, onces=None):
    """Launches of each timed grid kernel that did work over the timed layers: one operator,
    update (and finest post-smoothing) launch per iteration while any grid system of the
    launch still iterates (iter_rows: per layer, the iterations of every grid system served
    by the launches), and per such iteration the V-cycle's coarse launches (levels above the
    tail: restriction + pre-smoothing and post-smoothing; the tail and the restriction into
    it once each when some hierarchy reaches the tail; a truncated last level smoothed once
    has no post-smoothing launch)."""
    its = float(sum(max(r) if len(r) else 0 for r in iter_rows))
    out = {"A": its, "B": its}
    if precond == "mg":
        out["P"] = its
        above = post = tail = 0
        for k, (nl, (nx, ny)) in enumerate(zip(nlevs, shapes)):
            lv = mg_levels(nx, ny)[:nl + 1]
            n = [a * b for a, b in lv]
            na = sum(1 for v in n[1:] if v > MG_TAIL)
            above = max(above, na)
            post = max(post, na - (1 if onces and onces[k] and na and n[-1] > MG_TAIL else 0))
            tail = max(tail, 1 if any(v <= MG_TAIL for v in n[1:]) else 0)
        out.update({"RS": its * above, "PC": its * post, "TAIL": its * tail, "R": its * tail})
    return out


def solve_bytes(p, precision):
    """Algorithmic bytes of a layer outside the PCG iterations, per grid continuum: the
    right-hand side (previous layer, F, the other continua's previous layers read; b and
    the warm start written: 5 FP64 words) and the initial residual (b, x, diag, tx, ty read,
    r and the first preconditioned residual written: 7 FP64 words)."""
    return p.n_omega * p.ncell * (5 + 7) * 8


def options(args):
    o = dict(scheme="D", precision=args.precision, precond=args.precond,
             warm_start=args.warm_start, small_max=args.small_max)
    if args.precision == "mixed":
        o.update(outer_tol=args.tol, inner_tol=args.inner_tol)
    else:
        o.update(tol=args.tol)
    return o


def accuracy_after(g, workload, step, scheme):
    """Accuracy on the stored oracle sample at layer `step`, or, if that layer is not stored,
    at the next stored layer after stepping there (untimed, after the timed region)."""
    acc = golden_states(g.get_state, workload, step, scheme)
    if acc is not None:
        return acc
    path = os.path.join(ROOT, "tests", "golden", f"{workload.lower()}_oracle.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    later = sorted(int(k) for k in z[f"steps_{scheme}"] if int(k) > step)
    if not later:
        return None
    g.step(later[0] - step)
    acc = golden_states(g.get_state, workload, later[0], scheme)
    if acc is not None:
        acc["note"] = f"stepped untimed from layer {step} to the stored layer {later[0]}"
    return acc


def form_run(g, p, p0, args, change, scheme, profile=False):
    """Another form of the same decoupled scheme on the same problem and GPU (options
    changed by `change`): ms per layer over the timed layers, PCG iterations, accuracy (the
    next stored layer) and, with profile, its dominant grid kernel."""
    import torch
    opt = dict(options(args))
    opt.update(change)
    precond = opt["precond"]
    g.set_options(**opt)
    g.set_states(p0)
    g.step(2)                           # graphs of the new tables captured
    g.set_states(p0)
    if profile:
        g.profile(True, every=args.sample_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, lat = [], []
    for _ in range(args.steps):
        ts = time.perf_counter()
        rep = g.step(1)
        lat.append(time.perf_counter() - ts)
        iters.append(rep["iters"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = {"options": change, "value": p.dof() * args.steps / el, "unit": "cell-updates/s",
           "steps": args.steps, "ms_per_step": el / args.steps * 1e3,
           "latency_ms": {"p50": float(np.percentile(np.array(lat) * 1e3, 50)),
                          "p99": float(np.percentile(np.array(lat) * 1e3, 99))},
           "pcg_iters_per_step": np.array(iters).mean(axis=0).tolist()}
    if profile:
        tot = {k: 0.0 for k in kernels_of(precond)}
        nlev = list(g.info().mg_levels)
        once = [v == 1 for v in g.info().mg_stop_sweeps]
        for it in iters:
            sb = step_bytes(p, {"iters": it}, opt["precision"], precond, nlev, once)
            for kk in tot:
                tot[kk] += sb[kk]
        prof = read_profile(g, kernels_of(precond))
        g.profile(False)
        work = working_launches([r[:p.n_omega] for r in iters], precond, nlev[:p.n_omega],
                                [(p.nx, p.ny)] * p.n_omega, once[:p.n_omega])
        roof, roof2 = roofline(prof, tot, opt["precision"], precond, args.workload, work)
        res["roofline"] = roof
        res["roofline_other_kernels"] = roof2
    res["accuracy_vs_oracle"] = accuracy_after(g, args.workload, args.steps, scheme)
    log(f"form {change}: {res['value']:.4g} cell-updates/s, {res['ms_per_step']:.3f} ms/step")
    return res


def run_single(args, out):
    import torch
    import media
    from paper_2209_01158_amd import mcdec
    stream = torch.cuda.Stream()
    t = time.time()
    p = media.config_problem(args.workload)
    log(f"workload {args.workload}: {p.nx}x{p.ny}, {p.n_cont} continua, nf={p.nf}, "
        f"dof={p.dof()} (generated in {time.time() - t:.1f}s)")
    dof = p.dof()
    p0 = p.initial_state()
    with torch.cuda.stream(stream):
        t = time.time()
        g = mcdec.Problem(p, stream=stream.cuda_stream, **options(args))
        if args.autotune:
            ta = time.time()
            mcdec.autotune([g], iters=20)
            log(f"autotune {time.time() - ta:.2f}s: {mcdec.tilings(g)}")
        log(f"setup {time.time() - t:.2f}s, device memory {g.info().device_bytes / 2**20:.0f} MiB")
        for k in range(args.warmup):
            rep = g.step(1)
            log(f"warmup step {k + 1}: iters {rep['iters']}, {rep['seconds'] * 1e3:.2f} ms")
        g.set_states(p0)
        g.profile(True, every=args.sample_every)
        lat, iters = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ts = time.perf_counter()
            rep = g.step(1)
            lat.append(time.perf_counter() - ts)
            iters.append(rep["iters"])
            if (k + 1) % 20 == 0:
                log(f"step {k + 1}/{args.steps}: iters {rep['iters']} outer {rep['outer']}")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # algorithmic bytes of the timed layers, from their iteration counts (kept out of the
        # timed loop)
        tot = {k: 0.0 for k in kernels_of(args.precond)}
        nlev = list(g.info().mg_levels)
        once = [v == 1 for v in g.info().mg_stop_sweeps]
        for it in iters:
            sb = step_bytes(p, {"iters": it}, args.precision, args.precond, nlev, once)
            for kk in tot:
                tot[kk] += sb[kk]
        prof = read_profile(g, kernels_of(args.precond))
        g.profile(False)
        elapsed = t1 - t0
        value = dof * args.steps / elapsed
        all_bytes = sum(tot.values()) + args.steps * solve_bytes(p, args.precision)
        pcg_frac = all_bytes / elapsed / 1e9 / HBM_PEAK_GBS
        log(f"decoupled: {value:.4g} cell-updates/s, {elapsed / args.steps * 1e3:.3f} ms/step, "
            f"grid-kernel bytes / elapsed = {pcg_frac:.3f} of {HBM_PEAK_GBS / 1e3:.0f} TB/s")
        acc = accuracy_after(g, args.workload, args.steps, "D")
        extra = {}
        if args.workload == "C2" and not args.no_coupled:
            extra["fp64_tol_1e-12"] = form_run(g, p, p0, args, dict(tol=1e-12), "D")
            extra["bic0"] = form_run(g, p, p0, args, dict(precond="bic0"), "D", profile=True)
            g.set_options(**options(args))

        coupled = None
        if not args.no_coupled and args.coupled_steps > 0:
            g.set_options(scheme="coupled", precision="fp64", tol=min(args.tol, 1e-10))
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
            cacc = accuracy_after(g, args.workload, args.coupled_steps, "coupled")
            coupled = {"value": cval, "unit": "cell-updates/s", "steps": args.coupled_steps,
                       "ms_per_step": (c1 - c0) / args.coupled_steps * 1e3,
                       "pcg_iters_per_step": float(np.mean(citers)),
                       "decoupled_over_coupled": value / cval, "accuracy": cacc}
        plain = None
        if args.precision == "mixed" and not args.no_coupled:
            # the plain FP64 form of the same decoupled scheme on the same GPU
            g.set_options(scheme="D", precision="fp64", tol=args.tol)
            g.set_states(p0)
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            ns = max(1, min(args.steps, 5))
            for k in range(ns):
                g.step(1)
            torch.cuda.synchronize()
            pv = dof * ns / (time.perf_counter() - c0)
            plain = {"value": pv, "unit": "cell-updates/s", "steps": ns,
                     "scheme": "D", "precision": "fp64", "tol": args.tol,
                     "mixed_over_fp64": value / pv}
        g.close()
        calibrate(args)

    lat_ms = np.array(lat) * 1e3
    it = np.array(iters)
    work = working_launches([r[:p.n_omega] for r in iters], args.precond,
                            nlev[:p.n_omega], [(p.nx, p.ny)] * p.n_omega, once[:p.n_omega])
    roof, roof2 = roofline(prof, tot, args.precision, args.precond, args.workload, work)
    out.update({
        "value": value, "ms_per_step": elapsed / args.steps * 1e3,
        "config": {"workload": f"{args.workload}: {p.n_cont}-continuum {p.nx}x{p.ny}"
                   f"{'x%d' % p.nz if getattr(p, 'nz', 1) > 1 else ''} + "
                   f"{p.nf} fracture cells, tau={p.tau}, D-scheme {args.precision}, "
                   f"PCG {args.precond} tol {args.tol}", "dof": dof,
                   "precond": args.precond, "scheme": "D", "precision": args.precision,
                   "warm_start": args.warm_start, "autotuned": bool(args.autotune),
                   **({"inner_tol": args.inner_tol} if args.precision == "mixed" else {})},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99)), "max": float(lat_ms.max())},
        "pcg_iters_per_step": {"mean": it.mean(axis=0).tolist(), "max": it.max(axis=0).tolist()},
        "accuracy_vs_oracle": acc, "coupled_fp64": coupled, "plain_fp64": plain,
        "roofline": roof, "roofline_other_kernels": roof2,
        "pcg_roofline": {"what": "algorithmic bytes of every timed grid kernel (PCG iterations "
                         "and V-cycle levels, plus each layer's right-hand side and initial "
                         "residual) / elapsed time of the timed layers", "bytes": all_bytes,
                         "achieved": all_bytes / elapsed / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": pcg_frac},
        **extra,
    })
    if args.precision == "mixed":
        out["dtype"] = "f32+f64"


def run_batch(args, out):
    import torch
    import media
    from paper_2209_01158_amd import mcdec
    stream = torch.cuda.Stream()
    t = time.time()
    probs = media.configs.c4_problems(count=args.count)
    dof = sum(p.dof() for p in probs)
    log(f"workload C4: {len(probs)} problems, dof={dof} (generated in {time.time() - t:.1f}s)")
    with torch.cuda.stream(stream):
        t = time.time()
        opt = options(args)
        gs = [mcdec.Problem(p, stream=stream.cuda_stream, **opt) for p in probs]
        mem = sum(g.info().device_bytes for g in gs)
        log(f"setup {time.time() - t:.1f}s, device memory {mem / 2**30:.1f} GiB")
        if args.autotune:
            ta = time.time()
            mcdec.autotune(gs, iters=10)
            log(f"autotune {time.time() - ta:.1f}s")
        nlevs = [list(g.info().mg_levels) for g in gs]
        onces = [[v == 1 for v in g.info().mg_stop_sweeps] for g in gs]
        b = mcdec.Batch(stream=stream.cuda_stream, **opt)
        for k in range(args.warmup):
            reps = b.step(gs, 1)
            log(f"warmup step {k + 1}: {reps[0]['seconds'] * 1e3:.1f} ms")
        for g, p in zip(gs, probs):
            g.set_states(p.initial_state())
        b.profile(True, every=args.sample_every)
        lat = []
        all_reps = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ts = time.perf_counter()
            reps = b.step(gs, 1)
            lat.append(time.perf_counter() - ts)
            all_reps.append(reps)
            if (k + 1) % 10 == 0:
                log(f"step {k + 1}/{args.steps}: {lat[-1] * 1e3:.1f} ms, "
                    f"max iters {max(max(r['iters']) for r in reps)}")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # algorithmic bytes and iteration maxima of the timed layers (kept out of the loop)
        tot = {k: 0.0 for k in kernels_of(args.precond)}
        iters_max = []
        for reps in all_reps:
            for p, r, nl, on in zip(probs, reps, nlevs, onces):
                sb = step_bytes(p, r, args.precision, args.precond, nl, on)
                for kk in tot:
                    tot[kk] += sb[kk]
            iters_max.append(max(max(r["iters"]) for r in reps))
        prof = read_profile(b, kernels_of(args.precond))
        b.profile(False)
        elapsed = t1 - t0
        value = dof * args.steps / elapsed
        acc = golden_c4(dict(enumerate(gs)), args.steps, "D") if args.count == 256 else None
        log(f"batched: {value:.4g} cell-updates/s, {elapsed / args.steps * 1e3:.1f} ms/step")
        b.close()

        plain = None
        coupled = None
        if not args.no_coupled:
            # plain FP64 forms of the same decoupled scheme, problems created beforehand and
            # only the layers timed: (1) batched like the mixed form, (2) each problem alone
            ns = 2
            pg = [mcdec.Problem(p, stream=stream.cuda_stream, scheme="D", precision="fp64",
                                precond=args.precond, tol=args.tol) for p in probs]
            pb = mcdec.Batch(stream=stream.cuda_stream, scheme="D", precision="fp64",
                             precond=args.precond, tol=args.tol)
            pb.step(pg, 1)                                   # graphs captured
            for g, p in zip(pg, probs):
                g.set_states(p.initial_state())
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            for k in range(ns):
                pb.step(pg, 1)
            torch.cuda.synchronize()
            pbv = dof * ns / (time.perf_counter() - c0)
            pb.close()
            for g, p in zip(pg, probs):
                g.set_states(p.initial_state())
                g.step(1)                                    # graphs of the lone problem
                g.set_states(p.initial_state())
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            for g in pg:
                g.step(ns)
            torch.cuda.synchronize()
            pv = dof * ns / (time.perf_counter() - c0)
            for g in pg:
                g.close()
            plain = {"value": pbv, "unit": "cell-updates/s", "steps": ns,
                     "form": "batched like the mixed form, D-scheme FP64 PCG",
                     "batched_mixed_over_plain": value / pbv,
                     "alone": {"value": pv, "unit": "cell-updates/s", "steps": ns,
                               "form": "each problem stepped alone, D-scheme FP64 PCG",
                               "batched_mixed_over_alone_fp64": value / pv}}
            log(f"plain fp64: batched {pbv:.4g}, alone {pv:.4g} cell-updates/s")
            # coupled FP64, batched
            cg = [mcdec.Problem(p, stream=stream.cuda_stream, scheme="coupled", precision="fp64",
                                precond=args.precond, tol=args.tol) for p in probs]
            for g in gs:
                g.close()
            gs = []
            cb = mcdec.Batch(stream=stream.cuda_stream, scheme="coupled", precision="fp64",
                             precond=args.precond, tol=args.tol)
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            for k in range(args.coupled_steps):
                creps = cb.step(cg, 1)
                log(f"coupled batch step {k + 1}: max iters "
                    f"{max(r['iters'][0] for r in creps)}")
            torch.cuda.synchronize()
            cval = dof * args.coupled_steps / (time.perf_counter() - c0)
            cacc = golden_c4(dict(enumerate(cg)), args.coupled_steps, "coupled") \
                if args.count == 256 else None
            coupled = {"value": cval, "unit": "cell-updates/s", "steps": args.coupled_steps,
                       "form": "batched coupled FP64", "decoupled_over_coupled": value / cval,
                       "accuracy": cacc}
            cb.close()
            for g in cg:
                g.close()
        for g in gs:
            g.close()
        calibrate(args)
    lat_ms = np.array(lat) * 1e3
    rows = [[v for p, r in zip(probs, reps) for v in r["iters"][:p.n_omega]] for reps in all_reps]
    nl_all = [v for p, nl in zip(probs, nlevs) for v in nl[:p.n_omega]]
    on_all = [v for p, on in zip(probs, onces) for v in on[:p.n_omega]]
    shapes = [(p.nx, p.ny) for p in probs for _ in range(p.n_omega)]
    work = working_launches(rows, args.precond, nl_all, shapes, on_all)
    roof, roof2 = roofline(prof, tot, args.precision, args.precond, "C4", work)
    out.update({
        "value": value, "ms_per_step": elapsed / args.steps * 1e3, "dtype": "f32+f64",
        "config": {"workload": f"C4: {len(probs)} realizations (two/three continua, sides "
                   f"128..1024), tau=1e-3, batched D-scheme {args.precision}, "
                   f"PCG {args.precond}, refinement to {args.tol}", "dof": dof,
                   "problems": len(probs), "precond": args.precond, "scheme": "D",
                   "precision": args.precision, "warm_start": args.warm_start,
                   **({"inner_tol": args.inner_tol} if args.precision == "mixed" else {})},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99)), "max": float(lat_ms.max())},
        "pcg_iters_max_per_step": {"mean": float(np.mean(iters_max)),
                                   "max": int(np.max(iters_max))},
        "accuracy_vs_oracle": acc, "coupled_fp64": coupled, "plain_fp64": plain,
        "roofline": roof, "roofline_other_kernels": roof2,
    })


def serve_trace(args, trace, probs, steps, precision):
    """Replays the trace in real time against a server of the given precision; returns
    (request infos, server stats, server step durations, accuracy of the stored requests)."""
    import threading
    from paper_2209_01158_amd import mcdec
    budget = int(args.hbm_budget_gib * 2**30)
    opt = dict(options(args))
    opt["precision"] = precision
    if precision == "fp64":
        opt.pop("outer_tol", None)
        opt.pop("inner_tol", None)
        opt["tol"] = args.tol
    srv = mcdec.Server(budget, max_resident=args.max_resident, autotune=args.autotune, **opt)
    ids = [None] * len(trace)
    t0 = time.perf_counter()

    def feeder():
        for k, (e, p, n) in enumerate(zip(trace, probs, steps)):
            dt = e[0] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            ids[k] = srv.submit(p, n)

    th = threading.Thread(target=feeder)
    th.start()
    last = 0
    while th.is_alive():
        th.join(timeout=10)
        st = srv.stats()
        if st["finished"] != last:
            last = st["finished"]
            log(f"{precision} {time.perf_counter() - t0:.0f}s: finished {st['finished']}, "
                f"resident {st['resident']}, queued {st['queued']}")
    while True:
        try:
            srv.wait(timeout=10)
            break
        except mcdec.McError:
            st = srv.stats()
            log(f"{precision} {time.perf_counter() - t0:.0f}s: finished {st['finished']}, "
                f"resident {st['resident']}, queued {st['queued']}")
    infos = [srv.poll(i) for i in ids]
    st = srv.stats()
    step_s = srv.step_seconds()
    # accuracy: final states of the requests the oracle stored, against the oracle
    acc = None
    path = os.path.join(ROOT, "tests", "golden", "c5_oracle.npz")
    if os.path.exists(path) and len(trace) > 0:
        z = np.load(path, allow_pickle=False)
        per = {}
        for i in (int(v) for v in z["requests"]):
            if i >= len(ids) or infos[i]["state"] != "done":
                continue
            got = np.concatenate(srv.fetch(ids[i]))
            ref = np.concatenate([z[f"r{i}_c{a}"] for a in range(probs[i].n_cont)])
            per[str(i)] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        if per:
            acc = {"rel_l2_max": max(per.values()), "per_request": per,
                   "reference": os.path.relpath(path, ROOT),
                   "what": "final state of each stored request, every cell"}
    srv.close()
    return infos, st, step_s, acc


def run_serve(args, out):
    """Replays the seeded Poisson trace in real time against the server and reports the
    served throughput with per-step and per-request latency percentiles, the accuracy of
    the requests the oracle stored, and the same trace served in plain FP64."""
    import media
    trace = media.configs.c5_trace(count=args.count, rate=args.rate)
    t = time.time()
    probs = [media.configs.c5_problem(e) for e in trace]
    steps = [e[4] for e in trace]
    work = sum(p.dof() * n for p, n in zip(probs, steps))
    log(f"workload C5: {len(trace)} requests over {trace[-1][0]:.1f}s, {work:.3g} cell-updates "
        f"(built in {time.time() - t:.1f}s)")
    infos, st, step_s, acc = serve_trace(args, trace, probs, steps, args.precision)

    def served_rate(infos):
        fin = [i for i in infos if i["state"] == "done"]
        span = max(i["t_finish"] for i in fin) - min(i["t_submit"] for i in infos)
        served = sum(p.dof() * n for p, n, i in zip(probs, steps, infos) if i["state"] == "done")
        return fin, span, served / span

    fin, span, value = served_rate(infos)
    req_lat = np.array([i["t_finish"] - i["t_submit"] for i in fin])
    queue = np.array([i["t_admit"] - i["t_submit"] for i in fin])
    per_layer = np.array([(i["t_finish"] - i["t_admit"]) / i["n_steps"] for i in fin])
    log(f"served {len(fin)}/{len(infos)}: {value:.4g} cell-updates/s over {span:.1f}s")
    plain = None
    if not args.no_coupled and args.precision != "fp64":
        pinfos, pst, pstep_s, pacc = serve_trace(args, trace, probs, steps, "fp64")
        pfin, pspan, pvalue = served_rate(pinfos)
        plain = {"value": pvalue, "unit": "cell-updates/s", "form": "same trace served with "
                 "FP64 PCG (same server, same preconditioner)", "finished": len(pfin),
                 "makespan_s": pspan, "accuracy_vs_oracle": pacc,
                 "server_step_ms": {"p50": float(np.percentile(pstep_s, 50)) * 1e3,
                                    "p99": float(np.percentile(pstep_s, 99)) * 1e3},
                 "mixed_over_fp64": value / pvalue}
        log(f"plain fp64 served: {pvalue:.4g} cell-updates/s")
    pct = lambda a, q: float(np.percentile(a, q))  # noqa: E731
    out.update({
        "value": value, "ms_per_step": float(np.mean(step_s)) * 1e3, "dtype": "f32+f64",
        "steps": int(st["steps"]),
        "config": {"workload": f"C5: {len(trace)} Poisson arrivals at {args.rate}/s, sides "
                   f"64..2048, two/three continua, 10-500 layers, served with continuous "
                   f"batching in {args.precision} PCG {args.precond}, HBM budget "
                   f"{args.hbm_budget_gib} GiB", "requests": len(trace),
                   "offered_cell_updates": work, "precond": args.precond,
                   "precision": args.precision, "warm_start": args.warm_start,
                   **({"inner_tol": args.inner_tol} if args.precision == "mixed" else {})},
        "latency_ms": {"p50": pct(step_s, 50) * 1e3, "p99": pct(step_s, 99) * 1e3,
                       "max": float(step_s.max()) * 1e3,
                       "what": "server step: one layer of every resident request"},
        "request_latency_s": {"p50": pct(req_lat, 50), "p99": pct(req_lat, 99),
                              "max": float(req_lat.max())},
        "queueing_s": {"p50": pct(queue, 50), "p99": pct(queue, 99)},
        "per_layer_latency_ms": {"p50": pct(per_layer, 50) * 1e3,
                                 "p99": pct(per_layer, 99) * 1e3},
        "served": {"finished": len(fin), "failed": int(st["failed"]),
                   "makespan_s": span, "busy_s": st["busy_seconds"],
                   "cell_updates_per_busy_s": st["cell_updates"] / max(st["busy_seconds"], 1e-9)},
        "accuracy_vs_oracle": acc, "plain_fp64": plain,
    })


def run_nlmc(args, out):
    """The coarse-grid NLMC schemes (Section 4) on the paper's 2C and 3C problems (200 x 200
    fine grid with wells) on 20 x 20 and 40 x 40 coarse grids: GPU setup time (basis
    functions and coarse operator), time of 50 coarse layers per scheme, and e_H against
    the unit means of the fine coupled solution (computed on the GPU in FP64)."""
    import torch
    import media
    from paper_2209_01158_amd import mcdec
    rows = []
    layers = args.layers
    for kind in ("2C", "3C"):
        p = media.paper_problem(kind)
        nsteps = 50
        with mcdec.Problem(p, scheme="coupled", precond="mg", tol=1e-12) as g:
            g.step(nsteps)
            fine = np.concatenate(g.get_states())
        nc = p.nx * p.ny
        meas = np.concatenate([np.full(nc * p.n_omega, p.h ** 2), p.aperture * p.flen])
        for nco in (20, 40):
            b = p.nx // nco
            with mcdec.Problem(p, scheme="D", precond="mg") as g:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                nl = mcdec.Nlmc(g, b, b, layers)
                t_setup = time.perf_counter() - t0
                inf = nl.info()
                # unit means of the fine coupled solution (units: continuum by continuum,
                # coarse cells row-major; fracture units where a coarse cell hosts cells)
                y, x = np.divmod(np.arange(nc), p.nx)
                cof = (y // b) * nco + x // b
                ref = []
                for a in range(p.n_omega):
                    v = fine[a * nc:(a + 1) * nc]
                    ref.append(np.bincount(cof, v, nco * nco) / np.bincount(cof, None, nco * nco))
                fco = cof[np.asarray(p.host)]
                fm = meas[p.n_omega * nc:]
                fv = fine[p.n_omega * nc:]
                num = np.bincount(fco, fm * fv, nco * nco)
                den = np.bincount(fco, fm, nco * nco)
                ref.append((num / np.where(den > 0, den, 1))[den > 0])
                ref = np.concatenate(ref)
                res = {}
                for scheme in ("coupled", "L", "D", "U"):
                    nl.set_state()
                    nl.step(scheme, 1)                  # first launch of each kernel
                    nl.set_state()
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    nl.step(scheme, nsteps)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t1
                    xs = nl.get_state()
                    res[scheme] = {"seconds_50_layers": dt, "ms_per_layer": dt / nsteps * 1e3,
                                   "e_H_percent": 100 * float(np.linalg.norm(xs - ref) /
                                                              np.linalg.norm(ref))}
                rows.append({"problem": kind, "coarse_grid": f"{nco}x{nco}",
                             "oversampling_layers": layers, "n_units": inf.n_units,
                             "units_per_continuum": list(inf.sizes)[:inf.n_cont],
                             "largest_local_problem": inf.max_region_unknowns,
                             "largest_band": inf.max_band,
                             "setup_s": t_setup, "setup_gpu_ms": list(inf.setup_ms),
                             "schemes": res})
                log(f"NLMC {kind} {nco}x{nco}: N_H {inf.n_units}, setup {t_setup:.3f}s, "
                    + ", ".join(f"{k} {v['ms_per_layer']:.3f} ms/layer e_H "
                                f"{v['e_H_percent']:.3f}%" for k, v in res.items()))
                nl.close()
    d = [r for r in rows if r["problem"] == "2C" and r["coarse_grid"] == "20x20"][0]
    t = d["schemes"]["D"]["seconds_50_layers"]
    out.update({
        "value": d["n_units"] * 50 / t, "unit": "coarse cell-updates/s",
        "ms_per_step": t / 50 * 1e3, "steps": 50, "warmup": 1,
        "config": {"workload": "NLMC coarse-grid D-scheme (Section 4) on the paper's 2C "
                   f"problem, 200x200 fine grid, 20x20 coarse grid, {layers} oversampling "
                   "layers (value); every problem, grid and scheme under `nlmc`"},
        "nlmc": rows,
        "paper_context": {"hardware": "MacBook Pro, 2.3 GHz quad-core Core i7, Python + "
                          "PETSc CG+ILU", "2C_20x20_seconds": {"coupled": 0.174, "L": 0.035,
                          "D": 0.034, "U": 0.041}, "2C_40x40_seconds": {"coupled": 1.12,
                          "L": 0.135, "D": 0.14, "U": 0.151}, "3C_20x20_seconds": {
                          "coupled": 0.557, "L": 0.048, "D": 0.049, "U": 0.055},
                          "3C_40x40_seconds": {"coupled": 4.14, "L": 0.234, "D": 0.204,
                          "U": 0.234}, "e_H_percent_2C_20x20": {"coupled": 0.01, "L": 0.06,
                          "D": 0.08, "U": 0.01}},
    })


def calibrate(args):
    if args.calibrate_copy:
        import torch
        # known traffic for the HBM counters: a fill writes N bytes, a sum reads N bytes
        n = args.calibrate_copy * 2**20 // 8
        src = torch.full((n,), 1.0, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        tot = float(src.sum())
        torch.cuda.synchronize()
        log(f"calibration: filled and summed {args.calibrate_copy} MiB (sum {tot:.0f})")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="C2", choices=sorted(DEFAULTS))
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precond", default=None, choices=["jacobi", "bic0", "mg"])
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"])
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--warm-start", default=None,
                    choices=["extrapolate", "previous", "adaptive"],
                    help="PCG initial guess: linear extrapolation of the last two layers "
                         "(default), the previous layer, or the extrapolation order (0-3) "
                         "that best predicted the previous layer")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="mixed: inner FP32 PCG tolerance relative to the outer residual "
                         "(default 1e-4 with the V-cycle, whose passes are bounded by FP32 "
                         "rounding of the operator anyway, else 1e-6)")
    ap.add_argument("--coupled-steps", type=int, default=None)
    ap.add_argument("--count", type=int, default=None,
                    help="C4: realizations in the batch (256); C5: arrivals (400)")
    ap.add_argument("--rate", type=float, default=40.0, help="C5: arrivals per second")
    ap.add_argument("--hbm-budget-gib", type=float, default=128.0,
                    help="C5: device memory the resident requests may hold")
    ap.add_argument("--max-resident", type=int, default=0, help="C5: resident requests (0=256)")
    ap.add_argument("--small-max", type=int, default=None,
                    help="systems of at most this many unknowns run their whole PCG in one "
                         "workgroup (default 8192 for C1, else 0: off)")
    ap.add_argument("--autotune", action="store_true", default=None,
                    help="time the launch shapes per size class first (default for C4)")
    ap.add_argument("--layers", type=int, default=2,
                    help="NLMC: oversampling layers of the regions K_i^+")
    ap.add_argument("--sample-every", type=int, default=None,
                    help="time one grid PCG iteration in this many (HIP events; default 32; "
                         "4 for C3 and C4, whose launches serve systems of different "
                         "iteration counts, and 2 for the 3-D workload, whose layers take "
                         "only a few grid iterations)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-coupled", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB written by a fill and read by a sum (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    d = DEFAULTS[args.workload]
    for k in ("precond", "precision", "tol", "steps", "coupled_steps"):
        if getattr(args, k) is None:
            setattr(args, k, d[k])
    if args.sample_every is None:
        args.sample_every = d.get("sample_every", 32)
    if args.autotune is None:
        args.autotune = d.get("autotune", False)
    if args.small_max is None:
        args.small_max = d.get("small_max", 0)
    if args.inner_tol is None:
        args.inner_tol = (d["inner_tol"] if "inner_tol" in d and args.precond == d["precond"]
                          else 1e-4 if args.precond == "mg" else 1e-6)
    if args.warm_start is None:
        args.warm_start = "extrapolate"

    import torch
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    out = {"metric": METRIC, "value": None, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded generators of the workload recipe)"}
    if args.count is None:
        args.count = 400 if args.workload == "C5" else 256
    if args.workload == "NLMC":
        run_nlmc(args, out)
    elif args.workload == "C4":
        run_batch(args, out)
    elif args.workload == "C5":
        run_serve(args, out)
    else:
        run_single(args, out)
    if not args.no_cpu and args.workload not in ("C5", "NLMC"):
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
