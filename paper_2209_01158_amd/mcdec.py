"""ctypes binding of libmcdec.so (argument marshalling only; every computation runs in the
HIP library).  Names follow include/mcdec.h.

Importing this module loads the in-tree ``libmcdec.so`` and fails loudly if it is missing:
there is no fallback path.  torch is imported first when available so that the library and
torch share one HIP runtime (device pointers from torch tensors are then valid here).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

try:  # share torch's HIP runtime (same soname) when torch is present
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcdec.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2209_01158_amd.build` (hipcc, gfx950)")
_lib = C.CDLL(LIB_PATH)

MC_OK, MC_EINVAL, MC_ENOMEM, MC_ENOCONV, MC_EBREAKDOWN, MC_EDEVICE, MC_ENOTFOUND, \
    MC_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "MC_OK", -1: "MC_EINVAL", -2: "MC_ENOMEM", -3: "MC_ENOCONV",
                -4: "MC_EBREAKDOWN", -5: "MC_EDEVICE", -6: "MC_ENOTFOUND", -7: "MC_ETIMEOUT"}
REQ_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed"}
SCHEMES = {"D": 0, "coupled": 1, "L": 2, "U": 3, "EX": 4}
PRECISIONS = {"fp64": 0, "mixed": 1}
PRECONDS = {"jacobi": 0, "bic0": 1, "mg": 2}
WARM_STARTS = {"extrapolate": 0, "previous": 1, "adaptive": 2}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class OmegaDesc(C.Structure):
    _fields_ = [("c", C.c_double), ("k_const", C.c_double), ("k", _dp), ("src", _dp),
                ("p0", _dp)]


class ProblemDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("h", C.c_double),
                ("n_omega", C.c_int32), ("omega", OmegaDesc * 2), ("sigma_omega", C.c_double),
                ("nf", C.c_int32), ("host", _ip), ("flen", _dp), ("ne", C.c_int32),
                ("edges", _ip), ("edge_d", _dp), ("k_f", C.c_double), ("c_f", C.c_double),
                ("aperture", C.c_double), ("sigma_f", _dp), ("src_f", _dp), ("p0_f", _dp),
                ("bc_type", C.c_int32 * 4), ("bc_value", C.c_double * 4), ("tau", C.c_double),
                ("well_q", _dp), ("well_p", _dp), ("nz", C.c_int32),
                ("bc_type_z", C.c_int32 * 2), ("bc_value_z", C.c_double * 2)]


class Options(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("precision", C.c_int32), ("precond", C.c_int32),
                ("tol", C.c_double), ("max_iter", C.c_int32), ("outer_tol", C.c_double),
                ("max_outer", C.c_int32), ("inner_tol", C.c_double),
                ("check_every", C.c_int32), ("tile_rows", C.c_int32), ("warm_start", C.c_int32),
                ("small_max", C.c_int32), ("stream", C.c_void_p),
                ("dev_alloc", C.c_void_p), ("dev_free", C.c_void_p), ("alloc_ctx", C.c_void_p)]


class Report(C.Structure):
    _fields_ = [("n_cont", C.c_int32), ("iters", C.c_int32 * 3), ("outer", C.c_int32 * 3),
                ("converged", C.c_int32 * 3), ("relres", C.c_double * 3),
                ("seconds", C.c_double), ("step", C.c_int64), ("failed", C.c_int32),
                ("warm_order", C.c_int32 * 3)]

    def as_dict(self):
        n = self.n_cont
        return dict(iters=list(self.iters)[:n], outer=list(self.outer)[:n],
                    converged=list(self.converged)[:n], relres=list(self.relres)[:n],
                    seconds=self.seconds, step=self.step, failed=self.failed,
                    warm_order=list(self.warm_order)[:n])


class Info(C.Structure):
    _fields_ = [("n_cont", C.c_int32), ("sizes", C.c_int32 * 3), ("device_bytes", C.c_int64),
                ("grid_tiles", C.c_int32), ("n_chains", C.c_int32), ("tiles", C.c_int32 * 3),
                ("blocks", (C.c_int32 * 2) * 3), ("n_crossing", C.c_int32),
                ("mg_levels", C.c_int32 * 3), ("n_frac_blocks", C.c_int32),
                ("mg_stop_sweeps", C.c_int32 * 3)]


class NlmcInfo(C.Structure):
    _fields_ = [("n_units", C.c_int32), ("n_cont", C.c_int32), ("sizes", C.c_int32 * 3),
                ("n_regions", C.c_int32), ("max_region_unknowns", C.c_int32),
                ("max_band", C.c_int32), ("max_constraints", C.c_int32), ("pad", C.c_int32),
                ("n_pairs", C.c_int64), ("device_bytes", C.c_int64),
                ("setup_ms", C.c_double * 4), ("steps", C.c_int64)]


_PROBLEM = C.c_void_p


def _sig(name, restype, argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = argtypes
    return f


mc_options_default = _sig("mc_options_default", C.c_int, [C.POINTER(Options)])
mc_create_problem = _sig("mc_create_problem", C.c_int,
                         [C.POINTER(ProblemDesc), C.POINTER(Options), C.POINTER(_PROBLEM)])
mc_destroy = _sig("mc_destroy", C.c_int, [_PROBLEM])
mc_step = _sig("mc_step", C.c_int, [_PROBLEM, C.c_int32, C.POINTER(Report)])
mc_solve_continuum = _sig("mc_solve_continuum", C.c_int,
                          [_PROBLEM, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(Report)])
mc_solve_continuum_noalloc = _sig("mc_solve_continuum_noalloc", C.c_int,
                                  [_PROBLEM, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.POINTER(Report)])
mc_apply_continuum = _sig("mc_apply_continuum", C.c_int,
                          [_PROBLEM, C.c_int32, C.c_void_p, C.c_void_p])
mc_apply_coupled = _sig("mc_apply_coupled", C.c_int, [_PROBLEM, C.c_void_p, C.c_void_p])
mc_assemble_rhs = _sig("mc_assemble_rhs", C.c_int, [_PROBLEM, C.c_int32, C.c_void_p])
mc_apply_precond = _sig("mc_apply_precond", C.c_int, [_PROBLEM, C.c_int32, C.c_void_p, C.c_void_p])
mc_get_state = _sig("mc_get_state", C.c_int, [_PROBLEM, C.c_int32, _dp])
mc_set_state = _sig("mc_set_state", C.c_int, [_PROBLEM, C.c_int32, _dp])
mc_set_options = _sig("mc_set_options", C.c_int, [_PROBLEM, C.POINTER(Options)])
mc_get_info = _sig("mc_get_info", C.c_int, [_PROBLEM, C.POINTER(Info)])
mc_nlmc_create = _sig("mc_nlmc_create", C.c_int,
                      [_PROBLEM, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)])
mc_nlmc_destroy = _sig("mc_nlmc_destroy", C.c_int, [C.c_void_p])
mc_nlmc_get_info = _sig("mc_nlmc_get_info", C.c_int, [C.c_void_p, C.POINTER(NlmcInfo)])
mc_nlmc_get_system = _sig("mc_nlmc_get_system", C.c_int, [C.c_void_p, _dp, _dp, _dp])
mc_nlmc_set_state = _sig("mc_nlmc_set_state", C.c_int, [C.c_void_p, _dp])
mc_nlmc_get_state = _sig("mc_nlmc_get_state", C.c_int, [C.c_void_p, _dp])
mc_nlmc_step = _sig("mc_nlmc_step", C.c_int, [C.c_void_p, C.c_int32, C.c_int32])
mc_nlmc_last_error = _sig("mc_nlmc_last_error", C.c_char_p, [C.c_void_p])
mc_last_error = _sig("mc_last_error", C.c_char_p, [_PROBLEM])
mc_profile = _sig("mc_profile", C.c_int, [_PROBLEM, C.c_int32])
mc_profile_read = _sig("mc_profile_read", C.c_int,
                       [_PROBLEM, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                        C.POINTER(C.c_int64)])
mc_profile_read_above = _sig("mc_profile_read_above", C.c_int,
                             [_PROBLEM, C.c_int32, C.c_double, C.POINTER(C.c_int64),
                              C.POINTER(C.c_double)])


mc_autotune = _sig("mc_autotune", C.c_int, [C.POINTER(_PROBLEM), C.c_int32, C.c_int32])
mc_autotune_clear = _sig("mc_autotune_clear", C.c_int, [])

mc_footprint = _sig("mc_footprint", C.c_int,
                    [C.POINTER(ProblemDesc), C.POINTER(Options), C.POINTER(C.c_int64)])


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_resident", C.c_int32),
                ("max_bypass", C.c_int32), ("autotune", C.c_int32)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("steps_done", C.c_int32),
                ("n_steps", C.c_int32), ("bytes", C.c_int64), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_finish", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("finished", C.c_int64), ("failed", C.c_int64),
                ("queued", C.c_int64), ("resident", C.c_int64), ("bytes_in_use", C.c_int64),
                ("budget", C.c_int64), ("steps", C.c_int64), ("cell_updates", C.c_double),
                ("busy_seconds", C.c_double), ("elapsed_seconds", C.c_double)]


_SERVER = C.c_void_p
mc_server_create = _sig("mc_server_create", C.c_int,
                        [C.POINTER(ServerConfig), C.POINTER(Options), C.POINTER(_SERVER)])
mc_server_destroy = _sig("mc_server_destroy", C.c_int, [_SERVER])
mc_server_submit = _sig("mc_server_submit", C.c_int,
                        [_SERVER, C.POINTER(ProblemDesc), C.c_int32, C.POINTER(C.c_uint64)])
mc_server_poll = _sig("mc_server_poll", C.c_int, [_SERVER, C.c_uint64, C.POINTER(RequestInfo)])
mc_server_fetch = _sig("mc_server_fetch", C.c_int, [_SERVER, C.c_uint64, C.c_int32, _dp])
mc_server_release = _sig("mc_server_release", C.c_int, [_SERVER, C.c_uint64])
mc_server_wait = _sig("mc_server_wait", C.c_int, [_SERVER, C.c_double])
mc_server_get_stats = _sig("mc_server_get_stats", C.c_int, [_SERVER, C.POINTER(ServerStats)])
mc_server_step_seconds = _sig("mc_server_step_seconds", C.c_int,
                              [_SERVER, _dp, C.c_int64, C.POINTER(C.c_int64)])
mc_server_last_error = _sig("mc_server_last_error", C.c_char_p, [_SERVER])

_BATCH = C.c_void_p
mc_batch_create = _sig("mc_batch_create", C.c_int, [C.POINTER(Options), C.POINTER(_BATCH)])
mc_batch_destroy = _sig("mc_batch_destroy", C.c_int, [_BATCH])
mc_batch_step = _sig("mc_batch_step", C.c_int,
                     [_BATCH, C.POINTER(_PROBLEM), C.c_int32, C.c_int32, C.POINTER(Report)])
mc_batch_last_error = _sig("mc_batch_last_error", C.c_char_p, [_BATCH])
mc_batch_profile = _sig("mc_batch_profile", C.c_int, [_BATCH, C.c_int32])
mc_batch_profile_read = _sig("mc_batch_profile_read", C.c_int,
                             [_BATCH, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                              C.POINTER(C.c_int64)])
mc_batch_profile_read_above = _sig("mc_batch_profile_read_above", C.c_int,
                                   [_BATCH, C.c_int32, C.c_double, C.POINTER(C.c_int64),
                                    C.POINTER(C.c_double)])


class McError(RuntimeError):
    def __init__(self, status: int, msg: str, report: Optional[dict] = None):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.report = report


def _check(st, handle=None, report=None, last_error=None):
    if st != MC_OK:
        msg = (last_error or mc_last_error)(handle)
        raise McError(st, msg.decode() if msg else "", report)


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


# Device allocator hooks handing the library torch's caching allocator (mc_options.dev_alloc /
# dev_free): allocations on the current device and torch's current stream of the calling
# thread.  A failed allocation (an exception in the callback) reaches the library as NULL.
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def _torch_dev_alloc(nbytes, ctx):
    return torch.cuda.caching_allocator_alloc(nbytes)


def _torch_dev_free(ptr, ctx):
    torch.cuda.caching_allocator_delete(ptr)


_TORCH_HOOKS = (_ALLOC_FN(_torch_dev_alloc), _FREE_FN(_torch_dev_free))   # alive for the process


def make_options(scheme="D", precision="fp64", precond="jacobi", tol=1e-10, max_iter=20000,
                 outer_tol=1e-10, max_outer=30, inner_tol=1e-6, check_every=0, tile_rows=0,
                 warm_start="extrapolate", small_max=0, stream=None, alloc=None) -> Options:
    """alloc: None (the library's hipMalloc) or "torch" (torch's caching allocator)."""
    o = Options()
    _check(mc_options_default(C.byref(o)))
    o.scheme = SCHEMES[scheme]
    o.precision = PRECISIONS[precision]
    o.precond = PRECONDS[precond]
    o.tol, o.max_iter = tol, max_iter
    o.outer_tol, o.max_outer, o.inner_tol = outer_tol, max_outer, inner_tol
    o.check_every, o.tile_rows = check_every, tile_rows
    o.warm_start = WARM_STARTS[warm_start]
    o.small_max = small_max
    o.stream = stream
    if alloc == "torch":
        if torch is None:
            raise RuntimeError("alloc='torch' needs torch")
        o.dev_alloc = C.cast(_TORCH_HOOKS[0], C.c_void_p)
        o.dev_free = C.cast(_TORCH_HOOKS[1], C.c_void_p)
    elif alloc is not None:
        raise ValueError(f"unknown allocator {alloc!r}")
    return o


def _default_stream():
    if torch is not None and torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


def _sync_torch():
    """Order the caller's pending torch work (e.g. the fill of an output tensor) before a
    library call that touches caller-owned device memory on the library stream."""
    if torch is not None and torch.cuda.is_available():
        torch.cuda.current_stream().synchronize()


def _dev_ptr(t):
    """Device address of a torch tensor (contiguous float64 on the GPU)."""
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 tensor on the GPU")
    return C.c_void_p(t.data_ptr())


def describe(prob):
    """mc_problem_desc of a media.Problem, plus the numpy arrays it points into (keep them
    alive until the library has copied them)."""
    keep = []
    d = ProblemDesc()
    d.nx, d.ny, d.h = prob.nx, prob.ny, prob.h
    d.n_omega = len(prob.omega)
    for a, o in enumerate(prob.omega):
        od = d.omega[a]
        od.c, od.k_const = o.c, o.k_const
        if o.k is not None:
            k = np.ascontiguousarray(o.k, np.float64).reshape(-1)
            keep.append(k)
            od.k = _ptr(k, C.c_double)
        src = prob.source(a) if hasattr(prob, "source") else None
        if src is not None:
            src = np.ascontiguousarray(src, np.float64)
            keep.append(src)
            od.src = _ptr(src, C.c_double)
        p0 = None if prob.p0 is None else prob.p0[a]
        if p0 is not None:
            p0 = np.ascontiguousarray(p0, np.float64).reshape(-1)
            keep.append(p0)
            od.p0 = _ptr(p0, C.c_double)
    d.sigma_omega = prob.sigma_omega
    nf = int(len(prob.host))
    d.nf = nf
    if nf:
        host = np.ascontiguousarray(prob.host, np.int32)
        flen = np.ascontiguousarray(prob.flen, np.float64)
        sig = np.ascontiguousarray(prob.sigma_f, np.float64).reshape(-1)
        edges = np.ascontiguousarray(prob.edges, np.int32).reshape(-1)
        ed = np.ascontiguousarray(prob.edge_d, np.float64)
        keep += [host, flen, sig, edges, ed]
        d.host, d.flen, d.sigma_f = _ptr(host, C.c_int32), _ptr(flen, C.c_double), \
            _ptr(sig, C.c_double)
        d.ne = int(len(ed))
        d.edges, d.edge_d = _ptr(edges, C.c_int32), _ptr(ed, C.c_double)
        srcf = prob.source(d.n_omega) if hasattr(prob, "source") else None
        if srcf is not None:
            srcf = np.ascontiguousarray(srcf, np.float64)
            keep.append(srcf)
            d.src_f = _ptr(srcf, C.c_double)
        p0f = None if prob.p0 is None else prob.p0[d.n_omega]
        if p0f is not None:
            p0f = np.ascontiguousarray(p0f, np.float64)
            keep.append(p0f)
            d.p0_f = _ptr(p0f, C.c_double)
        wq = getattr(prob, "well_q", None)
        if wq is not None:
            wq = np.ascontiguousarray(wq, np.float64).reshape(-1)
            keep.append(wq)
            d.well_q = _ptr(wq, C.c_double)
            wp = getattr(prob, "well_p", None)
            if wp is not None:
                wp = np.ascontiguousarray(wp, np.float64).reshape(-1)
                keep.append(wp)
                d.well_p = _ptr(wp, C.c_double)
    d.k_f, d.c_f, d.aperture = prob.k_f, prob.c_f, prob.aperture
    for s in range(4):
        d.bc_type[s] = int(prob.bc_type[s])
        d.bc_value[s] = float(prob.bc_value[s])
    d.tau = prob.tau
    nz = int(getattr(prob, "nz", 1))
    d.nz = nz
    if nz > 1:
        for s in range(2):
            d.bc_type_z[s] = int(prob.bc_type_z[s])
            d.bc_value_z[s] = float(prob.bc_value_z[s])
    return d, keep


class Problem:
    """One multicontinuum problem resident on the GPU (wraps mc_problem)."""

    def __init__(self, prob, scheme="D", precision="fp64", precond="jacobi", tol=1e-10,
                 max_iter=20000, stream="default", **kw):
        if stream == "default":
            stream = _default_stream()
        d, self._keep = describe(prob)
        self.opt = make_options(scheme, precision, precond, tol, max_iter, stream=stream, **kw)
        h = _PROBLEM()
        _check(mc_create_problem(C.byref(d), C.byref(self.opt), C.byref(h)))
        self._keep = []
        self.h = h
        self.sizes = list(prob.sizes()) if hasattr(prob, "sizes") else None
        inf = self.info()
        self.sizes = list(inf.sizes)[:inf.n_cont]
        self.n_cont = inf.n_cont

    # --- lifecycle -----------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            mc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # --- calls ---------------------------------------------------------------------
    def step(self, n_steps: int = 1) -> dict:
        rep = Report()
        st = mc_step(self.h, n_steps, C.byref(rep))
        _check(st, self.h, rep.as_dict())
        return rep.as_dict()

    def solve_continuum(self, alpha: int, rhs, x) -> dict:
        rep = Report()
        _sync_torch()
        st = mc_solve_continuum(self.h, alpha, _dev_ptr(rhs), _dev_ptr(x), C.byref(rep))
        _check(st, self.h, rep.as_dict())
        return rep.as_dict()

    def solve_continuum_noalloc(self, alpha: int, rhs, x) -> dict:
        rep = Report()
        _sync_torch()
        st = mc_solve_continuum_noalloc(self.h, alpha, _dev_ptr(rhs), _dev_ptr(x), C.byref(rep))
        _check(st, self.h, rep.as_dict())
        return rep.as_dict()

    def apply_continuum(self, alpha: int, x, y):
        _sync_torch()
        _check(mc_apply_continuum(self.h, alpha, _dev_ptr(x), _dev_ptr(y)), self.h)

    def apply_coupled(self, x, y):
        _sync_torch()
        _check(mc_apply_coupled(self.h, _dev_ptr(x), _dev_ptr(y)), self.h)

    def apply_precond(self, alpha: int, r, z):
        _sync_torch()
        _check(mc_apply_precond(self.h, alpha, _dev_ptr(r), _dev_ptr(z)), self.h)

    def assemble_rhs(self, alpha: int, b):
        _sync_torch()
        _check(mc_assemble_rhs(self.h, alpha, _dev_ptr(b)), self.h)

    def get_state(self, alpha: int) -> np.ndarray:
        out = np.empty(self.sizes[alpha])
        _check(mc_get_state(self.h, alpha, _ptr(out, C.c_double)), self.h)
        return out

    def get_states(self):
        return [self.get_state(a) for a in range(self.n_cont)]

    def set_state(self, alpha: int, v):
        v = np.ascontiguousarray(v, np.float64).reshape(-1)
        if v.size != self.sizes[alpha]:
            raise ValueError("state size mismatch")
        _check(mc_set_state(self.h, alpha, _ptr(v, C.c_double)), self.h)

    def set_states(self, states):
        for a, v in enumerate(states):
            self.set_state(a, v)

    def set_options(self, **kw):
        cur = dict(scheme={v: k for k, v in SCHEMES.items()}[self.opt.scheme],
                   precision={v: k for k, v in PRECISIONS.items()}[self.opt.precision],
                   precond={v: k for k, v in PRECONDS.items()}[self.opt.precond],
                   tol=self.opt.tol, max_iter=self.opt.max_iter, outer_tol=self.opt.outer_tol,
                   max_outer=self.opt.max_outer, inner_tol=self.opt.inner_tol,
                   check_every=self.opt.check_every, tile_rows=self.opt.tile_rows,
                   warm_start={v: k for k, v in WARM_STARTS.items()}[self.opt.warm_start],
                   small_max=self.opt.small_max, stream=self.opt.stream)
        cur.update(kw)
        o = make_options(**cur)
        _check(mc_set_options(self.h, C.byref(o)), self.h)
        self.opt = o

    def info(self) -> Info:
        inf = Info()
        _check(mc_get_info(self.h, C.byref(inf)), self.h)
        return inf

    def profile(self, enable: bool, every: int = 8):
        """Start (sampling one grid PCG launch in `every`) or stop kernel timing."""
        _check(mc_profile(self.h, max(1, int(every)) if enable else 0), self.h)

    def profile_read(self, which: int):
        """(sampled launches, their summed ms, launches issued) of grid kernel `which`."""
        n = C.c_int64()
        ms = C.c_double()
        iss = C.c_int64()
        _check(mc_profile_read(self.h, which, C.byref(n), C.byref(ms), C.byref(iss)), self.h)
        return n.value, ms.value, iss.value

    def profile_read_above(self, which: int, min_ms: float):
        """(sampled launches of at least min_ms, their summed ms) of grid kernel `which`."""
        n = C.c_int64()
        ms = C.c_double()
        _check(mc_profile_read_above(self.h, which, float(min_ms), C.byref(n), C.byref(ms)),
               self.h)
        return n.value, ms.value


class Nlmc:
    """Coarse-grid NLMC system of a fine Problem (wraps mc_nlmc): bx x by fine cells per
    coarse cell, basis functions on regions grown by `layers` coarse cells."""

    def __init__(self, fine: "Problem", bx: int, by: int, layers: int):
        h = C.c_void_p()
        _check(mc_nlmc_create(fine.h, bx, by, layers, C.byref(h)), None,
               last_error=mc_nlmc_last_error)
        self.h = h
        self.fine = fine
        self.n = self.info().n_units

    def info(self) -> NlmcInfo:
        inf = NlmcInfo()
        _check(mc_nlmc_get_info(self.h, C.byref(inf)), self.h, last_error=mc_nlmc_last_error)
        return inf

    def system(self):
        """(A_bar, diagonal of M_bar, F_bar) as numpy arrays."""
        A = np.empty((self.n, self.n))
        M = np.empty(self.n)
        F = np.empty(self.n)
        _check(mc_nlmc_get_system(self.h, _ptr(A, C.c_double), _ptr(M, C.c_double),
                                  _ptr(F, C.c_double)), self.h, last_error=mc_nlmc_last_error)
        return A, M, F

    def set_state(self, x=None):
        xa = None if x is None else np.ascontiguousarray(x, np.float64)
        if xa is not None and xa.size != self.n:
            raise ValueError("state size mismatch")
        _check(mc_nlmc_set_state(self.h, _ptr(xa, C.c_double)), self.h,
               last_error=mc_nlmc_last_error)

    def get_state(self) -> np.ndarray:
        out = np.empty(self.n)
        _check(mc_nlmc_get_state(self.h, _ptr(out, C.c_double)), self.h,
               last_error=mc_nlmc_last_error)
        return out

    def step(self, scheme: str, n: int = 1):
        _check(mc_nlmc_step(self.h, SCHEMES[scheme], n), self.h, last_error=mc_nlmc_last_error)

    def close(self):
        if getattr(self, "h", None):
            mc_nlmc_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(problems, iters: int = 20):
    """Pick the PCG launch shapes per size class by timing (mc_autotune); applies to these
    problems and to problems created later in the process."""
    n = len(problems)
    arr = (_PROBLEM * n)(*[p.h for p in problems])
    _check(mc_autotune(arr, n, iters), problems[0].h)


def autotune_clear():
    _check(mc_autotune_clear())


def tilings(problem):
    """Work tiles and workgroups per launch [(tiles, operator, update)] per continuum."""
    inf = problem.info()
    return [(inf.tiles[c], inf.blocks[c][0], inf.blocks[c][1]) for c in range(inf.n_cont)]


def footprint(prob, **opt) -> int:
    """Device bytes a problem would hold (mc_footprint upper bound)."""
    d, keep = describe(prob)
    o = make_options(**opt)
    b = C.c_int64()
    _check(mc_footprint(C.byref(d), C.byref(o), C.byref(b)))
    return b.value


class Server:
    """Serving loop with continuous batching (wraps mc_server): requests are admitted by
    device-memory footprint, stay resident, and advance one layer per batched step."""

    def __init__(self, hbm_budget: int, max_resident: int = 0, max_bypass: int = 8,
                 autotune: bool = False, scheme="D", precision="mixed", precond="bic0",
                 tol=1e-10, max_iter=20000, stream=None, **kw):
        self.opt = make_options(scheme, precision, precond, tol, max_iter, stream=stream, **kw)
        cfg = ServerConfig(int(hbm_budget), int(max_resident), int(max_bypass), int(autotune))
        h = _SERVER()
        _check(mc_server_create(C.byref(cfg), C.byref(self.opt), C.byref(h)), None,
               last_error=mc_server_last_error)
        self.h = h
        self.sizes = {}

    def close(self):
        if getattr(self, "h", None):
            mc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, st):
        _check(st, self.h, last_error=mc_server_last_error)

    def submit(self, prob, n_steps: int) -> int:
        d, keep = describe(prob)
        rid = C.c_uint64()
        self._chk(mc_server_submit(self.h, C.byref(d), int(n_steps), C.byref(rid)))
        self.sizes[rid.value] = list(prob.sizes())
        return rid.value

    def poll(self, rid: int) -> dict:
        i = RequestInfo()
        self._chk(mc_server_poll(self.h, rid, C.byref(i)))
        return dict(state=REQ_STATES.get(i.state, i.state), status=i.status,
                    steps_done=i.steps_done, n_steps=i.n_steps, bytes=i.bytes,
                    t_submit=i.t_submit, t_admit=i.t_admit, t_finish=i.t_finish)

    def fetch(self, rid: int):
        out = []
        for a, n in enumerate(self.sizes[rid]):
            v = np.empty(n)
            self._chk(mc_server_fetch(self.h, rid, a, _ptr(v, C.c_double)))
            out.append(v)
        return out

    def release(self, rid: int):
        self._chk(mc_server_release(self.h, rid))
        self.sizes.pop(rid, None)

    def wait(self, timeout: float = -1.0):
        self._chk(mc_server_wait(self.h, float(timeout)))

    def stats(self) -> dict:
        st = ServerStats()
        self._chk(mc_server_get_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def step_seconds(self) -> np.ndarray:
        n = C.c_int64()
        self._chk(mc_server_step_seconds(self.h, None, 0, C.byref(n)))
        out = np.empty(n.value)
        self._chk(mc_server_step_seconds(self.h, _ptr(out, C.c_double), n.value, C.byref(n)))
        return out


class Batch:
    """Executor that advances many resident problems together (wraps mc_batch): every PCG
    launch covers all continua of all problems passed to `step`."""

    def __init__(self, scheme="D", precision="fp64", precond="jacobi", tol=1e-10,
                 max_iter=20000, stream="default", **kw):
        if stream == "default":
            stream = _default_stream()
        self.opt = make_options(scheme, precision, precond, tol, max_iter, stream=stream, **kw)
        h = _BATCH()
        _check(mc_batch_create(C.byref(self.opt), C.byref(h)), None,
               last_error=mc_batch_last_error)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            mc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, problems, n_steps: int = 1):
        """Advance every Problem in `problems` by n_steps layers; one report dict each."""
        n = len(problems)
        arr = (_PROBLEM * n)(*[p.h for p in problems])
        reps = (Report * n)()
        st = mc_batch_step(self.h, arr, n, n_steps, reps)
        out = [r.as_dict() for r in reps]
        _check(st, self.h, out, last_error=mc_batch_last_error)
        return out

    def profile(self, enable: bool, every: int = 8):
        _check(mc_batch_profile(self.h, max(1, int(every)) if enable else 0), self.h,
               last_error=mc_batch_last_error)

    def profile_read(self, which: int):
        n = C.c_int64()
        ms = C.c_double()
        iss = C.c_int64()
        _check(mc_batch_profile_read(self.h, which, C.byref(n), C.byref(ms), C.byref(iss)),
               self.h, last_error=mc_batch_last_error)
        return n.value, ms.value, iss.value

    def profile_read_above(self, which: int, min_ms: float):
        n = C.c_int64()
        ms = C.c_double()
        _check(mc_batch_profile_read_above(self.h, which, float(min_ms), C.byref(n),
                                           C.byref(ms)), self.h, last_error=mc_batch_last_error)
        return n.value, ms.value


EXPORTS = ["mc_options_default", "mc_create_problem", "mc_destroy", "mc_step",
           "mc_solve_continuum", "mc_solve_continuum_noalloc", "mc_apply_continuum", "mc_apply_coupled", "mc_assemble_rhs",
           "mc_apply_precond",
           "mc_get_state", "mc_set_state", "mc_set_options", "mc_get_info", "mc_last_error",
           "mc_profile", "mc_profile_read", "mc_profile_read_above", "mc_batch_create",
           "mc_batch_destroy", "mc_batch_step", "mc_batch_last_error", "mc_batch_profile",
           "mc_batch_profile_read", "mc_batch_profile_read_above",
           "mc_autotune", "mc_autotune_clear", "mc_footprint", "mc_server_create",
           "mc_server_destroy", "mc_server_submit", "mc_server_poll", "mc_server_fetch",
           "mc_server_release", "mc_server_wait", "mc_server_get_stats",
           "mc_server_step_seconds", "mc_server_last_error", "mc_nlmc_create",
           "mc_nlmc_destroy", "mc_nlmc_get_info", "mc_nlmc_get_system", "mc_nlmc_set_state",
           "mc_nlmc_get_state", "mc_nlmc_step", "mc_nlmc_last_error"]
