"""Writes stored expected values for full-size workloads by running the CPU oracle.

Calls only ``oracle`` (and the seeded input generator ``media``).  Output: one .npz per
workload with the oracle state sampled at fixed seeded cell indices after selected steps,
plus the full norms, so a GPU run at the same size can be checked entry by entry on the
sample and by relative error on the norm.

    python tests/golden/make_golden.py C2        # about 5-10 minutes, ~20 GB RAM
    python tests/golden/make_golden.py C4        # six realizations of the batch, ~1 minute
    python tests/golden/make_golden.py C3        # D layers by fast-diagonalization CG, ~1 hour
    python tests/golden/make_golden.py C5        # final states of five served requests, ~1 min
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import media  # noqa: E402
from oracle import fastdiag, schemes  # noqa: E402

NSAMPLE = 20000


def sample_indices(p, seed=99, nsample=NSAMPLE):
    rng = np.random.default_rng(seed)
    out = []
    for n in p.sizes():
        out.append(np.sort(rng.choice(n, size=min(n, nsample), replace=False)).astype(np.int64))
    return out


def run(name, d_steps, c_steps):
    p = media.config_problem(name)
    idx = sample_indices(p)
    data = {f"idx{a}": idx[a] for a in range(p.n_cont)}
    for scheme, keep in (("D", d_steps), ("coupled", c_steps)):
        t = time.time()
        st = schemes.Stepper(p, None, scheme)
        print(f"{name} {scheme}: factor {st.factor_seconds:.1f}s", flush=True)
        x = p.initial_state()
        last = max(keep)
        for n in range(1, last + 1):
            x = st.step(x)
            if n in keep:
                for a in range(p.n_cont):
                    data[f"{scheme}_s{n}_c{a}"] = x[a][idx[a]]
                    data[f"{scheme}_s{n}_norm{a}"] = np.array(np.linalg.norm(x[a]))
                print(f"  step {n} stored ({time.time() - t:.0f}s)", flush=True)
    data["steps_D"] = np.array(d_steps)
    data["steps_coupled"] = np.array(c_steps)
    out = os.path.join(HERE, f"{name.lower()}_oracle.npz")
    np.savez_compressed(out, **data)
    print("wrote", out, os.path.getsize(out), "bytes")


def run_c3(d_steps=(1, 2, 10, 50)):
    """The 4096 x 4096 three-continuum workload: D-scheme layers from the fast-diagonalization
    CG oracle (grid continua, residual 1e-14) and the sparse LU (fracture continuum)."""
    p = media.config_problem("C3")
    idx = sample_indices(p)
    data = {f"idx{a}": idx[a] for a in range(p.n_cont)}
    t = time.time()
    st = fastdiag.FDStepper(p)
    print(f"C3 setup {time.time() - t:.0f}s", flush=True)
    x = p.initial_state()
    for n in range(1, max(d_steps) + 1):
        x = st.step(x)
        print(f"  layer {n}: CG iterations {st.iterations[-1]} ({time.time() - t:.0f}s)",
              flush=True)
        if n in d_steps:
            for a in range(p.n_cont):
                data[f"D_s{n}_c{a}"] = x[a][idx[a]]
                data[f"D_s{n}_norm{a}"] = np.array(np.linalg.norm(x[a]))
    data["steps_D"] = np.array(d_steps)
    data["steps_coupled"] = np.array([], np.int64)
    out = os.path.join(HERE, "c3_oracle.npz")
    np.savez_compressed(out, **data)
    print("wrote", out, os.path.getsize(out), "bytes")


# the three smallest two-continuum and three-continuum realizations of the batched workload
C4_SUBSET = [168, 55, 253, 212, 105, 150]


def run_c4(d_steps=(1, 50), c_steps=(1, 2)):
    """Oracle states of a subset of the 256 batched realizations (each is independent, so a
    subset of the batch is checked problem by problem)."""
    data = {"problems": np.array(C4_SUBSET)}
    for i, p in zip(sorted(C4_SUBSET), media.configs.c4_problems(only=C4_SUBSET)):
        idx = sample_indices(p, seed=100 + i, nsample=3000)
        for a in range(p.n_cont):
            data[f"p{i}_idx{a}"] = idx[a]
        for scheme, keep in (("D", d_steps), ("coupled", c_steps)):
            t = time.time()
            st = schemes.Stepper(p, None, scheme)
            x = p.initial_state()
            for n in range(1, max(keep) + 1):
                x = st.step(x)
                if n in keep:
                    for a in range(p.n_cont):
                        data[f"p{i}_{scheme}_s{n}_c{a}"] = x[a][idx[a]]
            print(f"C4[{i}] n={p.nx} cont={p.n_cont} {scheme}: {time.time() - t:.1f}s", flush=True)
    data["steps_D"] = np.array(d_steps)
    data["steps_coupled"] = np.array(c_steps)
    out = os.path.join(HERE, "c4_oracle.npz")
    np.savez_compressed(out, **data)
    print("wrote", out, os.path.getsize(out), "bytes")


# five small requests of the serving trace (two- and three-continuum, contrasts 1e2..1e6)
C5_SUBSET = [288, 265, 152, 77, 389]


def run_c5():
    """Final D-scheme states of a subset of the served requests (each request is an
    independent problem advanced by its own number of layers)."""
    trace = media.configs.c5_trace()
    data = {"requests": np.array(C5_SUBSET)}
    for i in C5_SUBSET:
        p = media.configs.c5_problem(trace[i])
        t = time.time()
        x = schemes.run(p, "D", trace[i][4], keep="last")
        for a in range(p.n_cont):
            data[f"r{i}_c{a}"] = x[a]
        data[f"r{i}_steps"] = np.array(trace[i][4])
        print(f"C5[{i}] n={p.nx} cont={p.n_cont} layers={trace[i][4]}: "
              f"{time.time() - t:.1f}s", flush=True)
    out = os.path.join(HERE, "c5_oracle.npz")
    np.savez_compressed(out, **data)
    print("wrote", out, os.path.getsize(out), "bytes")


if __name__ == "__main__":
    name = sys.argv[1] if len(sys.argv) > 1 else "C2"
    if name == "C2":
        run("C2", d_steps=[1, 10, 100], c_steps=[1, 5, 100])
    elif name == "C4":
        run_c4()
    elif name == "C3":
        run_c3()
    elif name == "C5":
        run_c5()
    elif name == "C1":
        run("C1", d_steps=[1, 2, 5, 10, 20], c_steps=[1, 2, 5, 10, 20])
    else:
        raise SystemExit("unknown workload " + name)
