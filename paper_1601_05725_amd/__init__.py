"""Python binding of libbasker_mi355x.so (include/basker.h): argument marshalling only.

Every step of the factorization, refactorization and solve runs in the HIP library;
this module converts numpy arrays and torch tensors to pointers and status codes to
exceptions.  Importing it does not build anything; ``build.build()`` does.  If the
library is missing the first call raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbasker_mi355x.so")

OK = 0
REFACTOR_FELL_BACK = 1
ERR_INVALID = -1
ERR_STRUCT_SINGULAR = -2
ERR_NUM_SINGULAR = -3
ERR_OOM = -4
ERR_PATTERN = -5
ERR_DEVICE = -6
ERR_WORKSPACE = -7

EXPORTED = ["basker_default_options", "basker_symbolic", "basker_symbolic_ordered", "basker_factor",
            "basker_refactor", "basker_solve", "basker_solve_noalloc", "basker_info", "basker_get_ordering", "basker_extract",
            "basker_free", "basker_status_string", "basker_last_error"]


class basker_options(ctypes.Structure):
    _fields_ = [("pivot_tol", ctypes.c_double), ("diag_pref", ctypes.c_int32), ("matching", ctypes.c_int32),
                ("btf", ctypes.c_int32), ("fill_order", ctypes.c_int32), ("nd_leaves", ctypes.c_int32),
                ("nd_min_block", ctypes.c_int32), ("capacity_factor", ctypes.c_double),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("refactor_graph", ctypes.c_int32),
                ("max_grid", ctypes.c_int32), ("hbm_budget", ctypes.c_int64), ("sched_flags", ctypes.c_int32),
                ("item_cols", ctypes.c_int32), ("coop_waves", ctypes.c_int32), ("bin_edge", ctypes.c_int32),
                ("autotune", ctypes.c_int32)]


class basker_info_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("nnz_diag", ctypes.c_int64),
                ("nnz_offdiag", ctypes.c_int64), ("nblocks", ctypes.c_int32), ("ngroups", ctypes.c_int32),
                ("struct_rank", ctypes.c_int32), ("max_depth", ctypes.c_int32), ("lnz", ctypes.c_int64),
                ("unz", ctypes.c_int64), ("fail_col", ctypes.c_int32), ("offdiag_pivots", ctypes.c_int32),
                ("bottleneck", ctypes.c_double), ("factor_kernel_ms", ctypes.c_double),
                ("solve_kernel_ms", ctypes.c_double), ("scatter_kernel_ms", ctypes.c_double),
                ("factor_calls", ctypes.c_int32), ("refactor_calls", ctypes.c_int32),
                ("refactor_fallbacks", ctypes.c_int32), ("pool_regrows", ctypes.c_int32),
                ("nd_blocks", ctypes.c_int32), ("nlevels", ctypes.c_int32), ("solve_levels", ctypes.c_int32),
                ("crit_cols", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("dense_seps", ctypes.c_int32), ("sparse_seps", ctypes.c_int32),
                ("device_bytes_plan", ctypes.c_int64), ("coop_items", ctypes.c_int32),
                ("coop_waves", ctypes.c_int32), ("redo_items", ctypes.c_int32), ("learn_events", ctypes.c_int32),
                ("solve_order_fallbacks", ctypes.c_int32), ("rows_kernel_ms", ctypes.c_double),
                ("sym_lnz", ctypes.c_int64), ("sym_unz", ctypes.c_int64), ("fill_bound", ctypes.c_int32),
                ("sym_ws_rows", ctypes.c_int32), ("sched_bin_edge", ctypes.c_int32),
                ("autotune_trials", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if not name.startswith("reserved")}


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libbasker_mi355x.so is not built (run paper_1601_05725_amd/build.py); "
                           "there is no CPU fallback")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    lib.basker_default_options.restype = i32
    lib.basker_default_options.argtypes = [ctypes.POINTER(basker_options)]
    lib.basker_symbolic.restype = i32
    lib.basker_symbolic.argtypes = [i32, P, P, P, ctypes.POINTER(basker_options), ctypes.POINTER(P)]
    lib.basker_symbolic_ordered.restype = i32
    lib.basker_symbolic_ordered.argtypes = [i32, P, P, P, P, i32, P, i32, P, ctypes.POINTER(basker_options),
                                            ctypes.POINTER(P)]
    lib.basker_factor.restype = i32
    lib.basker_factor.argtypes = [P, P, i32]
    lib.basker_refactor.restype = i32
    lib.basker_refactor.argtypes = [P, P, i32]
    lib.basker_solve.restype = i32
    lib.basker_solve.argtypes = [P, i32, P, i32, i32]
    lib.basker_solve_noalloc.restype = i32
    lib.basker_solve_noalloc.argtypes = [P, i32, P, i32]
    lib.basker_info.restype = i32
    lib.basker_info.argtypes = [P, ctypes.POINTER(basker_info_t)]
    lib.basker_get_ordering.restype = i32
    lib.basker_get_ordering.argtypes = [P, P, P, P, P, P]
    lib.basker_extract.restype = i32
    lib.basker_extract.argtypes = [P, P, P, P, P, P, P, P]
    lib.basker_free.restype = None
    lib.basker_free.argtypes = [P]
    lib.basker_status_string.restype = ctypes.c_char_p
    lib.basker_status_string.argtypes = [i32]
    lib.basker_last_error.restype = ctypes.c_char_p
    lib.basker_last_error.argtypes = [P]
    _lib = lib
    return lib


class BaskerError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d)%s" % (load().basker_status_string(status).decode(), status,
                                        (": " + msg) if msg else ""))
        self.status = status


def default_options(**kw) -> basker_options:
    o = basker_options()
    load().basker_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _values_ptr(values):
    """(pointer, on_device, keepalive) for a numpy array or a torch tensor."""
    if hasattr(values, "data_ptr") and hasattr(values, "is_cuda"):
        if values.dtype.__str__() != "torch.float64":
            raise TypeError("values must be float64")
        if not values.is_contiguous():
            raise ValueError("values tensor must be contiguous")
        return ctypes.c_void_p(values.data_ptr()), int(values.is_cuda), values
    arr = np.ascontiguousarray(values, dtype=np.float64)
    return _np_ptr(arr), 0, arr


@dataclasses.dataclass
class Extracted:
    piv: np.ndarray
    Lp: np.ndarray
    Li: np.ndarray
    Lx: np.ndarray
    Up: np.ndarray
    Ui: np.ndarray
    Ux: np.ndarray


class Handle:
    """Owns one basker_handle (symbolic analysis + device factors)."""

    def __init__(self, ptr, n: int):
        self._h = ptr
        self.n = n

    def _check(self, st: int, ok=(OK,)) -> int:
        if st not in ok:
            msg = load().basker_last_error(self._h).decode() if self._h else ""
            raise BaskerError(st, msg)
        return st

    # -- constructors ------------------------------------------------------
    @staticmethod
    def symbolic(a, options: basker_options | None = None) -> "Handle":
        lib = load()
        cp = np.ascontiguousarray(a.colptr, np.int32)
        ri = np.ascontiguousarray(a.rowind, np.int32)
        vx = np.ascontiguousarray(a.values, np.float64)
        h = ctypes.c_void_p()
        o = options or default_options()
        st = lib.basker_symbolic(a.n, _np_ptr(cp), _np_ptr(ri), _np_ptr(vx), ctypes.byref(o), ctypes.byref(h))
        if st != OK:
            raise BaskerError(st, "symbolic")
        return Handle(h, a.n)

    @staticmethod
    def symbolic_ordered(a, prow, qcol, blkptr, grpptr, options: basker_options | None = None) -> "Handle":
        lib = load()
        cp = np.ascontiguousarray(a.colptr, np.int32)
        ri = np.ascontiguousarray(a.rowind, np.int32)
        pr = np.ascontiguousarray(prow, np.int32)
        qc = np.ascontiguousarray(qcol, np.int32)
        bp = np.ascontiguousarray(blkptr, np.int32)
        gp = np.ascontiguousarray(grpptr, np.int32)
        h = ctypes.c_void_p()
        o = options or default_options()
        st = lib.basker_symbolic_ordered(a.n, _np_ptr(cp), _np_ptr(ri), _np_ptr(pr), _np_ptr(qc), len(bp) - 1,
                                         _np_ptr(bp), len(gp) - 1, _np_ptr(gp), ctypes.byref(o), ctypes.byref(h))
        if st != OK:
            raise BaskerError(st, "symbolic_ordered")
        return Handle(h, a.n)

    # -- numeric -----------------------------------------------------------
    def factor(self, values) -> int:
        p, dev, keep = _values_ptr(values)
        return self._check(load().basker_factor(self._h, p, dev))

    def refactor(self, values) -> int:
        p, dev, keep = _values_ptr(values)
        return self._check(load().basker_refactor(self._h, p, dev), ok=(OK, REFACTOR_FELL_BACK))

    def solve(self, b):
        """Returns X for a numpy B (n or n x nrhs); solves a float64 device tensor in place."""
        if hasattr(b, "data_ptr") and hasattr(b, "is_cuda") and b.is_cuda:
            if b.dim() == 1:
                nrhs, ld = 1, b.shape[0]
            else:  # column-major storage: a (nrhs, n) contiguous tensor holds n x nrhs columns
                nrhs, ld = b.shape[0], b.shape[1]
            self._check(load().basker_solve(self._h, nrhs, ctypes.c_void_p(b.data_ptr()), ld, 1))
            return b
        B = np.array(b, dtype=np.float64, order="F", copy=True)
        vec = B.ndim == 1
        if vec:
            B = B.reshape(-1, 1, order="F")
        self._check(load().basker_solve(self._h, B.shape[1], _np_ptr(B), B.shape[0], 0))
        return B[:, 0] if vec else B

    def solve_noalloc(self, b):
        """Solve a float64 device tensor in place through the entry point that allocates
        nothing (a (nrhs, n) contiguous tensor holds the n x nrhs column-major B)."""
        if not (hasattr(b, "data_ptr") and getattr(b, "is_cuda", False)):
            raise TypeError("solve_noalloc takes a device tensor")
        if not b.is_contiguous() or str(b.dtype) != "torch.float64":
            raise ValueError("B must be a contiguous float64 tensor")
        nrhs, ld = (1, b.shape[0]) if b.dim() == 1 else (b.shape[0], b.shape[1])
        self._check(load().basker_solve_noalloc(self._h, nrhs, ctypes.c_void_p(b.data_ptr()), ld))
        return b

    # -- queries -----------------------------------------------------------
    def info(self) -> dict:
        inf = basker_info_t()
        self._check(load().basker_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def ordering(self):
        inf = self.info()
        prow = np.zeros(self.n, np.int32)
        qcol = np.zeros(self.n, np.int32)
        bp = np.zeros(inf["nblocks"] + 1, np.int32)
        gp = np.zeros(inf["ngroups"] + 1, np.int32)
        self._check(load().basker_get_ordering(self._h, _np_ptr(prow), _np_ptr(qcol), _np_ptr(bp), _np_ptr(gp),
                                               None))
        return prow, qcol, bp, gp

    def group_tree(self) -> np.ndarray:
        inf = self.info()
        gpar = np.zeros(inf["ngroups"], np.int32)
        self._check(load().basker_get_ordering(self._h, None, None, None, None, _np_ptr(gpar)))
        return gpar

    def extract(self) -> Extracted:
        inf = self.info()
        n = self.n
        e = Extracted(np.zeros(n, np.int32), np.zeros(n + 1, np.int64), np.zeros(inf["lnz"], np.int32),
                      np.zeros(inf["lnz"]), np.zeros(n + 1, np.int64), np.zeros(inf["unz"], np.int32),
                      np.zeros(inf["unz"]))
        self._check(load().basker_extract(self._h, _np_ptr(e.piv), _np_ptr(e.Lp), _np_ptr(e.Li), _np_ptr(e.Lx),
                                          _np_ptr(e.Up), _np_ptr(e.Ui), _np_ptr(e.Ux)))
        return e

    def free(self):
        if self._h:
            load().basker_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()
