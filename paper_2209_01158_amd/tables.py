"""The fine-grid comparison of the paper's numerical results (its Tables 1 and 2) on the GPU:
the 2C and 3C problems with wells, 50 layers with the coupled scheme and the L-, D- and
U-schemes, giving for each scheme the total solve time, the relative error e_h at the final
layer against the coupled solution (in percent, over all continua), and the average number
of PCG iterations per layer of every continuum.

    python -m paper_2209_01158_amd.tables [--precond mg|bic0|jacobi] [--tol 1e-10]
                                          [--precision fp64|mixed] [--outer-tol 1e-9]

The network geometry, sigma and the aperture are synthetic stand-ins (media.paper_problem),
so the errors are comparable with the paper's in size and order, not digit for digit.
Timings are on one GPU with every input resident; the paper's are for a CPU solver.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

import media
from . import mcdec

try:
    import torch
except Exception:  # pragma: no cover
    torch = None


def _sync():
    if torch is not None and torch.cuda.is_available():
        torch.cuda.synchronize()


def run_case(case: str, precond: str = "mg", tol: float = 1e-10, n: int = 200,
             precision: str = "fp64", outer_tol: float = 1e-9):
    p = media.paper_problem(case, n=n)
    out, states = {}, {}
    for scheme in ("coupled", "L", "D", "U"):
        # the coupled scheme is FP64 only; the decoupled ones take the chosen precision
        prec = "fp64" if scheme == "coupled" else precision
        with mcdec.Problem(p, scheme=scheme, precond=precond, tol=tol, precision=prec,
                           outer_tol=outer_tol) as g:
            g.step(1)                       # first layer outside the clock (setup, graphs)
            g.set_states(p.initial_state())
            _sync()
            t0 = time.perf_counter()
            iters = np.zeros(p.n_cont)
            for _ in range(p.nsteps):
                rep = g.step(1)
                iters += np.asarray(rep["iters"][:p.n_cont], float)
            _sync()
            secs = time.perf_counter() - t0
            states[scheme] = g.get_states()
        out[scheme] = dict(seconds=secs, iters_per_layer=list(iters / p.nsteps))
    ref = np.concatenate([np.ravel(v) for v in states["coupled"]])
    for scheme in ("L", "D", "U"):
        x = np.concatenate([np.ravel(v) for v in states[scheme]])
        out[scheme]["e_h_percent"] = 100.0 * float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
    return dict(case=case, dof=p.dof(), sizes=p.sizes(), wells=int(np.count_nonzero(p.well_q)),
                precond=precond, tol=tol, precision=precision,
                outer_tol=outer_tol if precision == "mixed" else None, schemes=out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--precond", default="mg", choices=list(mcdec.PRECONDS))
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--n", type=int, default=200)
    ap.add_argument("--precision", default="fp64", choices=list(mcdec.PRECISIONS))
    ap.add_argument("--outer-tol", type=float, default=1e-9,
                    help="mixed precision: FP64 refinement tolerance (the FP64 residual floor "
                         "of these fracture systems is near 1e-10)")
    a = ap.parse_args(argv)
    for case in ("2C", "3C"):
        r = run_case(case, a.precond, a.tol, a.n, a.precision, a.outer_tol)
        print(json.dumps(r), flush=True)
        print(f"{case}: DOF {r['dof']} {r['sizes']}, {r['wells']} well cells", flush=True)
        for s, v in r["schemes"].items():
            e = v.get("e_h_percent")
            it = " ".join(f"{x:.2f}" for x in v["iters_per_layer"])
            print(f"  {s:8s} {1e3 * v['seconds']:9.2f} ms   e_h {'-' if e is None else f'{e:.3f} %':>9s}"
                  f"   iterations per layer: {it}", flush=True)


if __name__ == "__main__":
    main()
