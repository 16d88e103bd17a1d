"""Serving form: requests of different sizes arrive while others run, are admitted by
device-memory footprint, and are advanced together by shared launches.  Each result must be
the same alone and in the mix: bitwise, since every problem keeps its own tilings and
reduction order (the stated tolerance, 1e-8 against the oracle, is checked too)."""
import time

import numpy as np
import pytest

import media
from oracle import schemes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
from paper_2209_01158_amd import mcdec  # noqa: E402

OPT = dict(scheme="D", precision="mixed", precond="bic0", outer_tol=1e-11, inner_tol=1e-5)


def requests():
    return [
        (media.small_problem(n=130, seed=8, nseg=10, seg_len=(10, 60)), 4),
        (media.small_problem(n=70, seed=5, three=True, nseg=6, seg_len=(5, 40)), 6),
        (media.small_problem(n=200, seed=11, nseg=12, seg_len=(10, 80)), 3),
        (media.small_problem(n=40, seed=2, nseg=4), 7),
        (media.small_problem(n=97, seed=9, three=True, nseg=0, lognormal=False), 5),
        (media.small_problem(n=160, seed=12, three=True, nseg=8, seg_len=(10, 60)), 2),
        (_wells(), 5),
        (media.box_problem(n=24, nz=12, seed=7, three=True), 4),   # 3-D
    ]


def _wells():
    """The numerical-results problem (wells) on a 60 x 60 grid, fracture permeability 1e3
    instead of 1e6 so that the 1e-11 outer tolerance lies above its FP64 residual floor."""
    p = media.paper_problem("3C", n=60)
    p.k_f = 1e3
    return p


def test_footprint_bounds_device_memory():
    for p, _ in requests()[:4]:
        for opt in (dict(precond="jacobi"), dict(precond="bic0"),
                    dict(precision="mixed", precond="bic0"),
                    dict(precision="mixed", precond="jacobi")):
            with mcdec.Problem(p, **opt) as g:
                used = g.info().device_bytes
            est = mcdec.footprint(p, **opt)
            assert used <= est <= 1.5 * used + (8 << 20), (p.nx, opt, used, est)


def test_server_results_equal_alone_and_memory_budget():
    reqs = requests()
    alone = []
    for p, n in reqs:
        with mcdec.Problem(p, **OPT) as g:
            g.step(n)
            alone.append(g.get_states())
    fp = [mcdec.footprint(p, **OPT) for p, _ in reqs]
    # the largest request fits only alone: it must wait until the others have left
    budget = max(fp)
    with mcdec.Server(budget, max_bypass=2, **OPT) as srv:
        ids = [srv.submit(p, n) for p, n in reqs[:4]]
        time.sleep(0.002)                              # later arrivals join a running batch
        ids += [srv.submit(p, n) for p, n in reqs[4:]]
        srv.wait(timeout=120)
        infos = [srv.poll(i) for i in ids]
        st = srv.stats()
        print(st, flush=True)
        assert st["finished"] == len(reqs) and st["failed"] == 0
        for k, (i, inf) in enumerate(zip(ids, infos)):
            assert inf["state"] == "done" and inf["steps_done"] == reqs[k][1]
            got = srv.fetch(i)
            for a, (x, y) in enumerate(zip(got, alone[k])):
                assert np.array_equal(x, y), (k, a, float(np.max(np.abs(x - y))))
            srv.release(i)
        # the budget held at every admission, and some request had to wait for memory
        for inf in infos:
            t = inf["t_admit"]
            live = sum(j["bytes"] for j in infos if j["t_admit"] <= t < j["t_finish"])
            assert live <= budget
        first_finish = min(j["t_finish"] for j in infos)
        assert any(j["t_admit"] >= first_finish for j in infos)
        assert len(srv.step_seconds()) == st["steps"]
    # the stated tolerance against the oracle, on one request
    p, n = reqs[1]
    ref = schemes.run(p, "D", n, keep="last")
    x = np.concatenate([np.ravel(v) for v in alone[1]])
    r = np.concatenate([np.ravel(v) for v in ref])
    assert np.linalg.norm(x - r) / np.linalg.norm(r) < 1e-8


def test_server_refuses_request_larger_than_budget():
    p, _ = requests()[2]
    with mcdec.Server(1 << 20, **OPT) as srv:
        with pytest.raises(mcdec.McError) as ei:
            srv.submit(p, 2)
        assert ei.value.status == mcdec.MC_ENOMEM
        with pytest.raises(mcdec.McError) as ei:
            srv.poll(12345)
        assert ei.value.status == mcdec.MC_ENOTFOUND


def test_server_with_torch_allocator():
    """A server whose problems take their device memory from torch's caching allocator
    (the hooks then run on the server's setup thread): the results equal those of each
    request stepped alone with the library's own allocation, and the memory goes back to
    torch when the server is destroyed."""
    reqs = requests()[:3]
    alone = []
    for p, n in reqs:
        with mcdec.Problem(p, **OPT) as g:
            g.step(n)
            alone.append(g.get_states())
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    with mcdec.Server(sum(mcdec.footprint(p, **OPT) for p, _ in reqs), alloc="torch",
                      **OPT) as srv:
        ids = [srv.submit(p, n) for p, n in reqs]
        srv.wait(timeout=120)
        assert torch.cuda.memory_allocated() > base
        for k, i in enumerate(ids):
            assert srv.poll(i)["state"] == "done"
            for x, y in zip(srv.fetch(i), alone[k]):
                assert np.array_equal(x, y), k
            srv.release(i)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
