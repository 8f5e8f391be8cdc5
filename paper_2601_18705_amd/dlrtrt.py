"""ctypes binding of libdlrtrt.so (include/dlrtrt.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts numpy
arrays and problem dicts to the C structs and back.  Importing the functions
here fails loudly if the library has not been built -- there is no CPU path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdlrtrt.so")

DLR_ABI_VERSION = 3
DLR_OK = 0
STATUS_NAMES = {0: "DLR_OK", -1: "DLR_ERR_ARG", -2: "DLR_ERR_OOM", -3: "DLR_ERR_HIP", -4: "DLR_ERR_NOT_CONVERGED",
                -5: "DLR_ERR_NONFINITE", -6: "DLR_ERR_STATE", -7: "DLR_ERR_UNSUPPORTED", -8: "DLR_ERR_NUMERIC",
                -9: "DLR_ERR_TIMEOUT"}
DLR_FP64, DLR_FP32_SWEEP, DLR_FP32_SWEEP_BF16_PROJ = 0, 1, 2

EXPORTED = ["dlr_set_allocator", "dlr_create", "dlr_create_augmented", "dlr_sn_create", "dlr_step", "dlr_sync", "dlr_read_fields", "dlr_read_factors", "dlr_load_factors",
            "dlr_read_stats", "dlr_force_selection", "dlr_set_dsa", "dlr_sweep_shape", "dlr_set_sweep_shape",
            "dlr_destroy", "dlr_batch_footprint", "dlr_batch_create",
            "dlr_batch_admit", "dlr_batch_advance", "dlr_batch_poll", "dlr_batch_read", "dlr_batch_read_stats",
            "dlr_batch_release", "dlr_batch_usage", "dlr_batch_destroy", "dlr_batch_set_graphs", "dlr_batch_graph_steps",
            "dlr_q1_create", "dlr_q1_sweep", "dlr_q1_sync", "dlr_q1_time", "dlr_q1_destroy", "dlr_q1_sweep_noalloc",
            "dlr_status_string", "dlr_last_error"]

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class DlrProblem(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
                ("n_polar", ctypes.c_int32), ("n_azim", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("dt", ctypes.c_double), ("c", ctypes.c_double), ("a", ctypes.c_double),
                ("sigma_a", _dp), ("rho_cv", _dp), ("q_ext", _dp), ("T_init", _dp),
                ("bc", ctypes.c_int32 * 4), ("T_b", ctypes.c_double * 4),
                ("precision", ctypes.c_int32), ("si_tol", ctypes.c_double), ("si_max_iter", ctypes.c_int32),
                ("deim_tie_tol", ctypes.c_double)]


class DlrStepStats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int64), ("si_iters", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("si_residual", ctypes.c_double), ("deim_min_margin", ctypes.c_double),
                ("sum_abs_cw_over_4pi", ctypes.c_double), ("energy", ctypes.c_double),
                ("sweep_ms", ctypes.c_double), ("step_ms", ctypes.c_double),
                ("svd_sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("inflow", ctypes.c_double), ("outflow", ctypes.c_double), ("source", ctypes.c_double),
                ("si_ms", ctypes.c_double)]


# dlr_set_allocator callbacks: alloc(bytes, stream, user) -> device pointer or NULL,
# release(ptr, stream, user)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = None   # keeps the installed callbacks alive


class DlrError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {detail}")


_lib = None


def library():
    """Load libdlrtrt.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the HIP library is the only implementation)")
        # PyTorch ships its own HIP and HSA runtimes under the same sonames as the system
        # ones.  Loaded first, they satisfy the library's dependencies, so the process holds
        # one runtime; loaded after the library, they would be a second copy that finds no GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        h = ctypes.c_void_p
        lib.dlr_create.argtypes = [ctypes.POINTER(DlrProblem), ctypes.c_void_p, ctypes.POINTER(h)]
        lib.dlr_create_augmented.argtypes = [ctypes.POINTER(DlrProblem), ctypes.c_void_p, ctypes.POINTER(h)]
        lib.dlr_sn_create.argtypes = [ctypes.POINTER(DlrProblem), ctypes.c_void_p, ctypes.POINTER(h)]
        lib.dlr_step.argtypes = [h, ctypes.c_int32]
        lib.dlr_sync.argtypes = [h]
        lib.dlr_read_fields.argtypes = [h, _dp, _dp]
        lib.dlr_read_factors.argtypes = [h, _dp, _dp, _dp, _ip]
        lib.dlr_load_factors.argtypes = [h, _dp, _dp, _dp, _dp]
        lib.dlr_read_stats.argtypes = [h, ctypes.POINTER(DlrStepStats)]
        lib.dlr_force_selection.argtypes = [h, _ip]
        lib.dlr_set_dsa.argtypes = [h, ctypes.c_int32, ctypes.c_double, ctypes.c_int32]
        lib.dlr_sweep_shape.argtypes = [h, _ip, _ip]
        lib.dlr_set_sweep_shape.argtypes = [h, ctypes.c_int32, ctypes.c_int32]
        lib.dlr_destroy.argtypes = [h]
        sz = ctypes.c_size_t
        i64 = ctypes.c_int64
        lib.dlr_batch_footprint.argtypes = [ctypes.POINTER(DlrProblem), ctypes.POINTER(sz)]
        lib.dlr_batch_create.argtypes = [sz, ctypes.c_void_p, ctypes.POINTER(h)]
        lib.dlr_batch_admit.argtypes = [h, ctypes.POINTER(DlrProblem), ctypes.c_int32, ctypes.POINTER(i64)]
        lib.dlr_batch_advance.argtypes = [h]
        lib.dlr_batch_poll.argtypes = [h, ctypes.POINTER(i64), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        lib.dlr_batch_read.argtypes = [h, i64, _dp, _dp]
        lib.dlr_batch_read_stats.argtypes = [h, i64, ctypes.POINTER(DlrStepStats)]
        lib.dlr_batch_release.argtypes = [h, i64]
        lib.dlr_batch_usage.argtypes = [h, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(sz)]
        lib.dlr_batch_destroy.argtypes = [h]
        lib.dlr_batch_set_graphs.argtypes = [h, ctypes.c_int32]
        lib.dlr_batch_graph_steps.argtypes = [h, ctypes.POINTER(i64)]
        vp = ctypes.c_void_p
        lib.dlr_q1_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                      _dp, _dp, ctypes.c_int32, vp, ctypes.POINTER(h)]
        lib.dlr_q1_sweep.argtypes = [h, vp, vp, vp, vp, vp]
        lib.dlr_q1_sync.argtypes = [h]
        lib.dlr_q1_time.argtypes = [h, vp, vp, vp, vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        lib.dlr_q1_destroy.argtypes = [h]
        lib.dlr_q1_sweep_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp]
        lib.dlr_set_allocator.argtypes = [ALLOC_FN, RELEASE_FN, ctypes.c_void_p]
        lib.dlr_status_string.argtypes = [ctypes.c_int]
        lib.dlr_status_string.restype = ctypes.c_char_p
        lib.dlr_last_error.argtypes = []
        lib.dlr_last_error.restype = ctypes.c_char_p
        for name in ("dlr_set_allocator", "dlr_create", "dlr_create_augmented", "dlr_sn_create", "dlr_step", "dlr_sync", "dlr_read_fields", "dlr_read_factors",
                     "dlr_load_factors", "dlr_read_stats", "dlr_force_selection", "dlr_set_dsa", "dlr_sweep_shape",
                     "dlr_set_sweep_shape", "dlr_destroy",
                     "dlr_batch_footprint", "dlr_batch_create", "dlr_batch_admit", "dlr_batch_advance",
                     "dlr_batch_poll", "dlr_batch_read", "dlr_batch_read_stats", "dlr_batch_release",
                     "dlr_batch_usage", "dlr_batch_destroy", "dlr_batch_set_graphs", "dlr_batch_graph_steps",
                     "dlr_q1_create", "dlr_q1_sweep", "dlr_q1_sync",
                     "dlr_q1_time", "dlr_q1_destroy", "dlr_q1_sweep_noalloc"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def set_allocator(alloc=None, release=None):
    """dlr_set_allocator with Python callables alloc(nbytes, stream) -> int device pointer (0 on
    failure) and release(ptr, stream); both None restores hipMalloc / hipFree."""
    global _allocator_refs
    lib = library()
    if alloc is None and release is None:
        _check(lib.dlr_set_allocator(ALLOC_FN(), RELEASE_FN(), None))
        _allocator_refs = None
        return

    def _a(nbytes, stream, _user):
        return int(alloc(int(nbytes), stream or 0)) or None

    def _r(ptr, stream, _user):
        release(int(ptr), stream or 0)

    refs = (ALLOC_FN(_a), RELEASE_FN(_r))
    _check(lib.dlr_set_allocator(refs[0], refs[1], None))
    _allocator_refs = refs


def torch_allocator():
    """(alloc, release) callables backed by PyTorch's caching allocator on the current device."""
    import torch

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, stream=stream)

    def release(ptr, _stream):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, release


def _check(status):
    if status != DLR_OK:
        raise DlrError(status, library().dlr_last_error().decode())


def _f64(a, n=None):
    arr = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and arr.size != n:
        raise ValueError(f"expected {n} values, got {arr.size}")
    return arr


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def marshal_problem(problem):
    """Problem dict -> (DlrProblem, arrays that must stay alive while it is used)."""
    n = int(problem["nx"]) * int(problem["ny"])
    keep = [_f64(problem["sigma_a"], n), _f64(problem["rho_cv"], n), _f64(problem["T_init"], n)]
    qext = problem.get("q_ext")
    keep.append(None if qext is None else _f64(qext, n))
    p = DlrProblem()
    p.abi_version = DLR_ABI_VERSION
    p.nx, p.ny = int(problem["nx"]), int(problem["ny"])
    p.x0, p.x1, p.y0, p.y1 = (float(problem[k]) for k in ("x0", "x1", "y0", "y1"))
    p.n_polar, p.n_azim, p.rank = int(problem["n_polar"]), int(problem["n_azim"]), int(problem["rank"])
    p.dt, p.c, p.a = float(problem["dt"]), float(problem["c"]), float(problem["a"])
    p.sigma_a, p.rho_cv, p.T_init = (_ptr(a) for a in keep[:3])
    p.q_ext = _ptr(keep[3])
    for k in range(4):
        p.bc[k] = int(problem["bc"][k])
        p.T_b[k] = float(problem["T_b"][k])
    p.precision = int(problem.get("precision", DLR_FP64))
    p.si_tol = float(problem.get("si_tol", 1e-14))
    p.si_max_iter = int(problem.get("si_max_iter", 10000))
    p.deim_tie_tol = float(problem.get("deim_tie_tol", 1e-6))
    return p, keep


def footprint(problem):
    """Device bytes the problem occupies once admitted to a batch."""
    p, _keep = marshal_problem(problem)
    out = ctypes.c_size_t()
    _check(library().dlr_batch_footprint(ctypes.byref(p), ctypes.byref(out)))
    return int(out.value)


class Batch:
    """Independent problems resident on the device, advanced together (dlr_batch_*)."""

    def __init__(self, hbm_budget=0, stream=None):
        self._h = ctypes.c_void_p()
        self._shape = {}
        _check(library().dlr_batch_create(ctypes.c_size_t(int(hbm_budget)), ctypes.c_void_p(stream or 0),
                                          ctypes.byref(self._h)))

    def admit(self, problem, n_steps):
        """Slot id, or None when the footprint does not fit (DLR_ERR_OOM: retry after a release)."""
        p, _keep = marshal_problem(problem)
        slot = ctypes.c_int64()
        st = library().dlr_batch_admit(self._h, ctypes.byref(p), int(n_steps), ctypes.byref(slot))
        if st == -2:
            return None
        _check(st)
        self._shape[slot.value] = int(problem["nx"]) * int(problem["ny"])
        return slot.value

    def advance(self):
        _check(library().dlr_batch_advance(self._h))

    def poll(self, cap=4096):
        ids = (ctypes.c_int64 * cap)()
        n = ctypes.c_int32()
        _check(library().dlr_batch_poll(self._h, ids, int(cap), ctypes.byref(n)))
        return [ids[k] for k in range(n.value)]

    def read(self, slot):
        n = self._shape[slot]
        E = np.empty(n)
        T = np.empty(n)
        _check(library().dlr_batch_read(self._h, ctypes.c_int64(slot), _ptr(E), _ptr(T)))
        return E, T

    def read_stats(self, slot):
        s = DlrStepStats()
        _check(library().dlr_batch_read_stats(self._h, ctypes.c_int64(slot), ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in DlrStepStats._fields_}

    def release(self, slot):
        _check(library().dlr_batch_release(self._h, ctypes.c_int64(slot)))
        self._shape.pop(slot, None)

    def usage(self):
        a = ctypes.c_int32()
        b = ctypes.c_size_t()
        _check(library().dlr_batch_usage(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, int(b.value)

    def set_graphs(self, enable):
        """0: eager steps only; 1: recorded-graph steps (default); 2..64: at most that many source
        iterations recorded per step."""
        _check(library().dlr_batch_set_graphs(self._h, int(enable)))

    def graph_steps(self):
        n = ctypes.c_int64()
        _check(library().dlr_batch_graph_steps(self._h, ctypes.byref(n)))
        return n.value

    def close(self):
        if self._h:
            library().dlr_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Instance:
    """One problem resident on the device (dlr_create ... dlr_destroy).

    method="dlr" steps the low-rank method; method="augmented" its variant with
    the old basis added to the Galerkin space and a rank-2r -> r truncation
    (dlr_create_augmented); method="sn" creates a plain discrete-ordinates
    instance of the same problem (dlr_sn_create), which has no factors."""

    def __init__(self, problem, stream=None, method="dlr"):
        lib = library()
        self.nx, self.ny, self.n = int(problem["nx"]), int(problem["ny"]), int(problem["nx"]) * int(problem["ny"])
        self.nq = int(problem["n_polar"]) * int(problem["n_azim"])
        self.method = method
        if method == "sn":
            self.rank = self.nq
            problem = dict(problem, rank=1)
            create = lib.dlr_sn_create
        elif method in ("dlr", "augmented"):
            self.rank = int(problem["rank"])
            create = lib.dlr_create if method == "dlr" else lib.dlr_create_augmented
        else:
            raise ValueError(f"unknown method {method!r}")
        p, self._keep = marshal_problem(problem)
        self._p = p
        self._h = ctypes.c_void_p()
        _check(create(ctypes.byref(p), ctypes.c_void_p(stream or 0), ctypes.byref(self._h)))
        if problem.get("dsa"):
            self.set_dsa(True, float(problem.get("dsa_cg_tol", 1e-8)), int(problem.get("dsa_cg_max_iter", 100)))

    def set_dsa(self, enable=True, cg_tol=1e-8, cg_max_iter=100):
        """dlr_set_dsa: diffusion synthetic acceleration of the source iteration."""
        _check(library().dlr_set_dsa(self._h, int(bool(enable)), float(cg_tol), int(cg_max_iter)))

    def sweep_shape(self):
        """dlr_sweep_shape: (prefetch depth, persistent workgroups) of the sweeps; (0, 0) before the first."""
        p = ctypes.c_int32()
        g = ctypes.c_int32()
        _check(library().dlr_sweep_shape(self._h, ctypes.byref(p), ctypes.byref(g)))
        return p.value, g.value

    def set_sweep_shape(self, prefetch=0, grid_blocks=0):
        """dlr_set_sweep_shape: a fixed launch shape, or (0, 0) for the tuner's choice."""
        _check(library().dlr_set_sweep_shape(self._h, int(prefetch), int(grid_blocks)))

    def step(self, n_steps=1):
        _check(library().dlr_step(self._h, int(n_steps)))

    def sync(self):
        _check(library().dlr_sync(self._h))

    def read_fields(self):
        E = np.empty(self.n)
        T = np.empty(self.n)
        _check(library().dlr_read_fields(self._h, _ptr(E), _ptr(T)))
        return E, T

    def read_factors(self):
        X = np.empty((self.n, self.rank))
        S = np.empty((self.rank, self.rank))
        W = np.empty((self.nq, self.rank))
        sel = np.empty(self.rank, dtype=np.int32)
        _check(library().dlr_read_factors(self._h, _ptr(X), _ptr(S), _ptr(W), sel.ctypes.data_as(_ip)))
        return X, S, W, sel

    def load_factors(self, X, S, W, T):
        Xa = _f64(X, self.n * self.rank)
        Sa = _f64(S, self.rank * self.rank)
        Wa = _f64(W, self.nq * self.rank)
        Ta = _f64(T, self.n)
        _check(library().dlr_load_factors(self._h, _ptr(Xa), _ptr(Sa), _ptr(Wa), _ptr(Ta)))

    def read_stats(self):
        s = DlrStepStats()
        _check(library().dlr_read_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in DlrStepStats._fields_}

    def force_selection(self, sel):
        if sel is None:
            _check(library().dlr_force_selection(self._h, None))
            return
        a = np.ascontiguousarray(sel, dtype=np.int32)
        _check(library().dlr_force_selection(self._h, a.ctypes.data_as(_ip)))

    def close(self):
        if self._h:
            library().dlr_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def q1_sweep_noalloc(nx, ny, hx, hy, mu, eta, precision, sigma_t, src, inflow_x, inflow_y, psi, status,
                     stream=None):
    """dlr_q1_sweep_noalloc: one Q1 sweep without an operator handle and without allocating.
    mu, eta: float64 GPU tensors [n_dir]; status: int32 GPU tensor [1] (the caller clears it);
    the arrays as in Q1Sweep.  Asynchronous on `stream` (None = the null stream)."""
    import torch
    nd = int(mu.numel())
    dt = torch.float64 if int(precision) == DLR_FP64 else torch.float32
    n = int(nx) * int(ny)
    want = ((mu, torch.float64, nd), (eta, torch.float64, nd), (sigma_t, dt, n), (src, dt, nd * n * 4),
            (inflow_x, dt, nd * int(ny) * 2), (inflow_y, dt, nd * int(nx) * 2), (psi, dt, nd * n * 4),
            (status, torch.int32, 1))
    ptrs = []
    for t, tdt, size in want:
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == tdt and t.is_contiguous()
                and t.numel() == size):
            raise ValueError(f"expected a contiguous {tdt} GPU tensor of {size} elements")
        ptrs.append(ctypes.c_void_p(t.data_ptr()))
    _check(library().dlr_q1_sweep_noalloc(int(nx), int(ny), float(hx), float(hy), nd, ptrs[0], ptrs[1],
                                          int(precision), ctypes.c_void_p(stream or 0), *ptrs[2:]))


class Q1Sweep:
    """Bilinear (Q1) upwind DG sweep operator (dlr_q1_create ... dlr_q1_destroy).

    Arrays are device tensors (torch, on the GPU, contiguous) of the operator's
    precision: sigma_t [ny*nx], src [nd, ny*nx, 4], inflow_x [nd, ny, 2],
    inflow_y [nd, nx, 2], psi [nd, ny*nx, 4]; cell e = j*nx + i, node
    a = ix + 2*iy.  Every call runs on `stream` (a hipStream_t handle, None =
    the null stream)."""

    def __init__(self, nx, ny, hx, hy, mu, eta, precision=DLR_FP64, stream=None):
        lib = library()
        self.nx, self.ny = int(nx), int(ny)
        mu_a = _f64(mu)
        self.nd = mu_a.size
        eta_a = _f64(eta, self.nd)
        self.precision = int(precision)
        self._h = ctypes.c_void_p()
        _check(lib.dlr_q1_create(self.nx, self.ny, float(hx), float(hy), self.nd, _ptr(mu_a), _ptr(eta_a),
                                 self.precision, ctypes.c_void_p(stream or 0), ctypes.byref(self._h)))

    def _ptrs(self, sigma_t, src, inflow_x, inflow_y, psi):
        import torch
        dt = torch.float64 if self.precision == DLR_FP64 else torch.float32
        n = self.nx * self.ny
        want = ((sigma_t, n), (src, self.nd * n * 4), (inflow_x, self.nd * self.ny * 2),
                (inflow_y, self.nd * self.nx * 2), (psi, self.nd * n * 4))
        out = []
        for t, size in want:
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()
                    and t.numel() == size):
                raise ValueError(f"expected a contiguous {dt} GPU tensor of {size} elements")
            out.append(ctypes.c_void_p(t.data_ptr()))
        return out

    def sweep(self, sigma_t, src, inflow_x, inflow_y, psi):
        _check(library().dlr_q1_sweep(self._h, *self._ptrs(sigma_t, src, inflow_x, inflow_y, psi)))

    def sync(self):
        _check(library().dlr_q1_sync(self._h))

    def time(self, sigma_t, src, inflow_x, inflow_y, psi, reps):
        ms = ctypes.c_double()
        _check(library().dlr_q1_time(self._h, *self._ptrs(sigma_t, src, inflow_x, inflow_y, psi), int(reps),
                                     ctypes.byref(ms)))
        return ms.value

    def close(self):
        if self._h:
            library().dlr_q1_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
