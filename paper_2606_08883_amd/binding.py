"""ctypes binding of ``libmrcm.so`` (include/mrcm.h).

Argument marshalling only: every step of setup, apply and GMRES runs in the
library.  Device vectors are torch CUDA (HIP) float64 tensors; the stream is
torch's current stream unless one is given.  There is no fallback: when the
library is missing every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmrcm.so")

MRCM_OK, MRCM_EINVAL, MRCM_ENOMEM, MRCM_ESINGULAR, MRCM_ENOCONV, MRCM_EDEVICE = 0, -1, -2, -3, -4, -5
_NAMES = {-1: "EINVAL", -2: "ENOMEM", -3: "ESINGULAR", -4: "ENOCONV", -5: "EDEVICE"}

# Every symbol the headers declare (checked by the test suite).
EXPORTED = ["mrcm_map_sizes", "mrcm_maps", "mrcm_setup", "mrcm_apply", "mrcm_apply_noalloc",
            "mrcm_apply_many",
            "op_apply", "gmres_solve", "mrcm_rhs", "mrcm_footprint", "mrcm_timing_enable",
            "mrcm_timing_read", "mrcm_query", "mrcm_set_allocator", "mrcm_set_lanes", "mrcm_set_batch",
            "mrcm_set_host_threads",
            "gmres_batch_create", "gmres_batch_add", "gmres_batch_tick", "gmres_batch_poll",
            "gmres_batch_remove", "gmres_batch_destroy",
            "mrcm3d_setup", "mrcm3d_apply", "mrcm3d_op_apply", "mrcm3d_rhs", "mrcm3d_gmres_solve",
            "mrcm3d_timing_enable", "mrcm3d_timing_read", "mrcm3d_query", "mrcm3d_destroy",
            "mrcm_destroy",
            "mrcm_last_error"]
QUERIES = {"setup_seconds": 0, "device_bytes": 1, "coarse_pivot": 2, "coarse_levels": 3,
           "coarse_dofs": 4, "coarse_bytes": 5, "coarse_launches": 6, "tune_ms": 7,
           "tune_changes": 8, "coarse_refine": 9, "mfma_recon": 10, "setup_host_s": 11,
           "setup_device_s": 12, "setup_coarse_s": 13}
PHASES = ["local", "coarse", "reconstruct", "residual", "patch", "finalize"]
TEST_EXPORTED = ["mrcm_test_coarse_sizes", "mrcm_test_coarse_matrix", "mrcm_test_host_apply",
                 "mrcm_test_coarse_solve", "mrcm_test_zero_cell_setup", "mrcm3d_test_host_apply",
                 "mrcm3d_test_dissection"]


class MrcmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"MRCM_{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("bc", ctypes.c_int32 * 4)]


class Params(ctypes.Structure):
    _fields_ = [("sx", ctypes.c_int32), ("sy", ctypes.c_int32), ("oversample", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("beta_len", ctypes.c_int32),
                ("smooth_sweeps", ctypes.c_int32), ("smooth_overlap", ctypes.c_int32),
                ("iface_degree", ctypes.c_int32), ("precision", ctypes.c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Grid3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 6)]


class Params3(ctypes.Structure):
    _fields_ = [("sx", ctypes.c_int32), ("sy", ctypes.c_int32), ("sz", ctypes.c_int32),
                ("oversample", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("beta_len", ctypes.c_int32), ("smooth_sweeps", ctypes.c_int32),
                ("smooth_overlap", ctypes.c_int32), ("iface_degree", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("hist_cap", ctypes.c_int32),
                ("hist_len", ctypes.c_int32), ("true_len", ctypes.c_int32),
                ("final_relres", ctypes.c_double), ("est_hist", ctypes.POINTER(ctypes.c_double)),
                ("true_hist", ctypes.POINTER(ctypes.c_double))]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built (run python -m paper_2606_08883_amd.build_lib)")
        # PyTorch ships its own HIP and HSA runtimes.  Importing it first
        # makes the library bind to those same runtimes; loaded the other way
        # round, the process held two runtime stacks and the library's first
        # device call found no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        pG, pP = ctypes.POINTER(Grid), ctypes.POINTER(Params)
        pi32 = ctypes.POINTER(ctypes.c_int32)
        pi64 = ctypes.POINTER(ctypes.c_int64)
        pd = ctypes.POINTER(ctypes.c_double)
        sig = {
            "mrcm_map_sizes": ([pG, pP, pi64, pi64, pi64], i32),
            "mrcm_maps": ([pG, pP] + [pi32] * 8, i32),
            "mrcm_setup": ([pG, pP, P, P, ctypes.POINTER(P)], i32),
            "mrcm_apply": ([P, P, P, i32, P], i32),
            "mrcm_apply_noalloc": ([P, P, P, i32, P], i32),
            "mrcm_apply_many": ([ctypes.POINTER(P), i32, ctypes.POINTER(P), ctypes.POINTER(P),
                                 pi32, P], i32),
            "mrcm_set_allocator": ([ALLOC_FN, FREE_FN], None),
            "op_apply": ([P, P, P, i32, P], i32),
            "gmres_solve": ([P, P, P, i32, dbl, i32, i32, ctypes.POINTER(Stats), P], i32),
            "mrcm_rhs": ([P, P, P, dbl, P, P], i32),
            "mrcm_set_lanes": ([P, i32], i32),
            "mrcm_set_batch": ([P, i32], i32),
            "mrcm_set_host_threads": ([i32], i32),
            "mrcm_footprint": ([pG, pP, i32], ctypes.c_size_t),
            "mrcm_timing_enable": ([P, i32], i32),
            "mrcm_timing_read": ([P, pd, pi64], i32),
            "mrcm_query": ([P, i32, pd], i32),
            "mrcm_destroy": ([P], None),
            "gmres_batch_create": ([i32, ctypes.POINTER(P)], i32),
            "mrcm3d_setup": ([ctypes.POINTER(Grid3), ctypes.POINTER(Params3), P, P,
                              ctypes.POINTER(P)], i32),
            "mrcm3d_apply": ([P, P, P, P], i32),
            "mrcm3d_op_apply": ([P, P, P, P], i32),
            "mrcm3d_rhs": ([P, P, P, dbl, P, P], i32),
            "mrcm3d_gmres_solve": ([P, P, P, dbl, i32, i32, ctypes.POINTER(Stats), P], i32),
            "mrcm3d_timing_enable": ([P, i32], i32),
            "mrcm3d_timing_read": ([P, pd, pi64], i32),
            "mrcm3d_query": ([P, i32, pd], i32),
            "mrcm3d_destroy": ([P], None),
            "mrcm3d_test_host_apply": ([ctypes.POINTER(Grid3), ctypes.POINTER(Params3), pd, pd,
                                        pd, pi64], i32),
            "mrcm3d_test_dissection": ([i32, i32, i32, pi32, pi32, pi32, pi32, pi32, i32, i32,
                                        pi32], i32),
            "gmres_batch_add": ([P, P, P, P, i32, dbl, i32, P, pi32], i32),
            "gmres_batch_tick": ([P, pi32], i32),
            "gmres_batch_poll": ([P, i32, pi32, ctypes.POINTER(Stats)], i32),
            "gmres_batch_remove": ([P, i32], i32),
            "gmres_batch_destroy": ([P], None),
            "mrcm_last_error": ([], ctypes.c_char_p),
            "mrcm_test_coarse_sizes": ([pG, pP, pd, pi64, pi64], i32),
            "mrcm_test_coarse_matrix": ([pG, pP, pd, pi32, pi32, pd], i32),
            "mrcm_test_host_apply": ([pG, pP, pd, pd, pd, pd], i32),
            "mrcm_test_coarse_solve": ([pG, pP, pd, pd, pd], i32),
            "mrcm_test_zero_cell_setup": ([pG, pP, pd, i64], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(code: int):
    if code != MRCM_OK:
        raise MrcmError(code, lib().mrcm_last_error().decode())


@dataclass
class Config:
    """Grid and method parameters (see include/mrcm.h)."""
    nx: int
    ny: int
    bc: tuple = (0, 0, 0, 0)
    sx: int = 16
    sy: int = 16
    oversample: int = 0
    alpha: float = 10.0
    beta_len: int = 0
    smooth_sweeps: int = 0
    smooth_overlap: int = 2
    iface_degree: int = 1
    precision: int = 0

    def grid(self) -> Grid:
        return Grid(self.nx, self.ny, (ctypes.c_int32 * 4)(*self.bc))

    def params(self) -> Params:
        return Params(self.sx, self.sy, self.oversample, self.alpha, self.beta_len,
                      self.smooth_sweeps, self.smooth_overlap, self.iface_degree, self.precision)


def _i32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def map_sizes(cfg: Config):
    m, e, nc = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    g, p = cfg.grid(), cfg.params()
    _check(lib().mrcm_map_sizes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(m),
                                ctypes.byref(e), ctypes.byref(nc)))
    return m.value, e.value, nc.value


def maps(cfg: Config) -> dict:
    m, e, nc = map_sizes(cfg)
    out = {"owner": np.zeros(cfg.nx * cfg.ny, np.int32), "boxes": np.zeros((m, 4), np.int32),
           "oboxes": np.zeros((m, 4), np.int32), "pboxes": np.zeros((m, 4), np.int32),
           "edges": np.zeros((e, 5), np.int32), "dof_table": np.zeros((nc, 3), np.int32),
           "dof_offset": np.zeros(m + 1, np.int32), "row_table": np.zeros((nc, 3), np.int32)}
    g, p = cfg.grid(), cfg.params()
    _check(lib().mrcm_maps(ctypes.byref(g), ctypes.byref(p), _i32(out["owner"]),
                           _i32(out["boxes"]), _i32(out["oboxes"]), _i32(out["pboxes"]),
                           _i32(out["edges"]), _i32(out["dof_table"]), _i32(out["dof_offset"]),
                           _i32(out["row_table"])))
    return out


def set_host_threads(threads: int) -> None:
    """mrcm_set_host_threads: host threads of this thread's later set-ups."""
    _check(lib().mrcm_set_host_threads(threads))


def footprint(cfg: Config, nrhs: int = 1) -> int:
    g, p = cfg.grid(), cfg.params()
    return int(lib().mrcm_footprint(ctypes.byref(g), ctypes.byref(p), nrhs))


# ---- test hooks of the host setup (host memory) ------------------------------
def test_coarse_matrix(cfg: Config, K: np.ndarray):
    import scipy.sparse as sp
    K = np.ascontiguousarray(K, dtype=np.float64)
    g, p = cfg.grid(), cfg.params()
    nc, nnz = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().mrcm_test_coarse_sizes(ctypes.byref(g), ctypes.byref(p), _f64(K),
                                        ctypes.byref(nc), ctypes.byref(nnz)))
    rp = np.zeros(nc.value + 1, np.int32)
    ci = np.zeros(max(nnz.value, 1), np.int32)
    cv = np.zeros(max(nnz.value, 1), np.float64)
    _check(lib().mrcm_test_coarse_matrix(ctypes.byref(g), ctypes.byref(p), _f64(K), _i32(rp),
                                         _i32(ci), _f64(cv)))
    return sp.csr_matrix((cv[:nnz.value], ci[:nnz.value], rp), shape=(nc.value, nc.value))


def test_host_apply(cfg: Config, K: np.ndarray, r: np.ndarray):
    K = np.ascontiguousarray(K, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.zeros_like(r)
    piv = ctypes.c_double()
    g, p = cfg.grid(), cfg.params()
    _check(lib().mrcm_test_host_apply(ctypes.byref(g), ctypes.byref(p), _f64(K), _f64(r), _f64(z),
                                      ctypes.byref(piv)))
    return z, piv.value


def test_coarse_solve(cfg: Config, K: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    K = np.ascontiguousarray(K, dtype=np.float64)
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    x = np.zeros_like(rhs)
    g, p = cfg.grid(), cfg.params()
    _check(lib().mrcm_test_coarse_solve(ctypes.byref(g), ctypes.byref(p), _f64(K), _f64(rhs),
                                        _f64(x)))
    return x


# ---- device entry points --------------------------------------------------------
_allocator = None  # the callback objects in use (kept alive while installed)


def test_zero_cell_setup(cfg: Config, K: np.ndarray, cell: int) -> None:
    """Host set-up with K = 0 on one cell after validation (failure injection)."""
    g, p = cfg.grid(), cfg.params()
    K = np.ascontiguousarray(K, dtype=np.float64)
    _check(lib().mrcm_test_zero_cell_setup(ctypes.byref(g), ctypes.byref(p), _f64(K), cell))


@dataclass
class Config3:
    """A 3-D grid and the method parameters (include/mrcm3d.h)."""
    nx: int
    ny: int
    nz: int
    bc: tuple
    sx: int
    sy: int
    sz: int
    oversample: int
    alpha: float = 10.0
    beta_len: int = 0
    sweeps: int = 1
    overlap: int = 2
    degree: int = 1
    precision: int = 0

    def grid(self) -> Grid3:
        return Grid3(self.nx, self.ny, self.nz, (ctypes.c_int32 * 6)(*self.bc))

    def params(self) -> Params3:
        return Params3(self.sx, self.sy, self.sz, self.oversample, self.alpha, self.beta_len,
                       self.sweeps, self.overlap, self.degree, self.precision)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


def test3d_host_apply(cfg: Config3, K: np.ndarray, r: np.ndarray) -> tuple:
    """z = T r on a 3-D grid from the host tables of mrcm3d_setup; (z, nc)."""
    g, p = cfg.grid(), cfg.params()
    K = np.ascontiguousarray(K, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.empty(cfg.n)
    nc = ctypes.c_int64()
    _check(lib().mrcm3d_test_host_apply(ctypes.byref(g), ctypes.byref(p), _f64(K), _f64(r),
                                        _f64(z), ctypes.byref(nc)))
    return z, nc.value


def test3d_dissection(mx: int, my: int, mz: int) -> dict:
    """The 3-D interface solve's dissection tree: elim (per subdomain), parent,
    depth and border lists per node (post-order)."""
    m = mx * my * mz
    cap = 4 * m + 8
    elim = np.full(m, -1, dtype=np.int32)
    parent = np.empty(cap, dtype=np.int32)
    depth = np.empty(cap, dtype=np.int32)
    bptr = np.empty(cap + 1, dtype=np.int32)
    border = np.empty(6 * m * cap // 4 + 64, dtype=np.int32)
    nn = ctypes.c_int32()
    p32 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
    _check(lib().mrcm3d_test_dissection(mx, my, mz, p32(elim), p32(parent), p32(depth), p32(bptr),
                                        p32(border), cap, len(border), ctypes.byref(nn)))
    k = nn.value
    return {"elim": elim, "parent": parent[:k].copy(), "depth": depth[:k].copy(),
            "border": [border[bptr[t]:bptr[t + 1]].copy() for t in range(k)]}


class Context3:
    """A set-up 3-D MRCM-OS operator (mrcm3d_setup)."""

    def __init__(self, cfg: Config3, K, stream=None):
        self.cfg = cfg
        self.n = cfg.n
        self._ptr = ctypes.c_void_p()
        self._g, self._p = cfg.grid(), cfg.params()
        _check(lib().mrcm3d_setup(ctypes.byref(self._g), ctypes.byref(self._p),
                                  _dptr(K, self.n), _stream(stream), ctypes.byref(self._ptr)))

    def close(self):
        if self._ptr:
            lib().mrcm3d_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, r, z, stream=None):
        _check(lib().mrcm3d_apply(self._ptr, _dptr(r, self.n), _dptr(z, self.n), _stream(stream)))

    def op(self, x, y, stream=None):
        _check(lib().mrcm3d_op_apply(self._ptr, _dptr(x, self.n), _dptr(y, self.n),
                                     _stream(stream)))

    def rhs(self, f, g, h: float, b, stream=None):
        """b = f h^2 + 2 K g on the Dirichlet faces (mrcm3d_rhs); f, g: device or None."""
        c = self.cfg
        ng = 2 * (c.ny * c.nz + c.nx * c.nz + c.nx * c.ny)
        _check(lib().mrcm3d_rhs(self._ptr, _dptr(f, self.n) if f is not None else None,
                                _dptr(g, ng) if g is not None else None, h,
                                _dptr(b, self.n), _stream(stream)))

    def gmres(self, b, p, rtol: float = 1e-8, restart: int = 10, maxit: int = 300,
              stream=None, raise_on_noconv: bool = True) -> SolveStats:
        st = Stats(0, 0, 0, 0, 0, 0, 0.0, None, None)
        code = lib().mrcm3d_gmres_solve(self._ptr, _dptr(b, self.n), _dptr(p, self.n), rtol,
                                        restart, maxit, ctypes.byref(st), _stream(stream))
        if code != MRCM_OK and (code != MRCM_ENOCONV or raise_on_noconv):
            _check(code)
        return SolveStats(st.iterations, st.cycles, bool(st.converged), st.final_relres, [], [])

    def timing(self, on: bool):
        _check(lib().mrcm3d_timing_enable(self._ptr, 1 if on else 0))

    def timing_read(self) -> dict:
        ms = (ctypes.c_double * 6)()
        cnt = (ctypes.c_int64 * 6)()
        _check(lib().mrcm3d_timing_read(self._ptr, ms, cnt))
        return {PHASES[k]: (ms[k], cnt[k]) for k in range(6)}

    def query(self, what: str) -> float:
        """setup_seconds, device_bytes, coarse_dofs, factor_bytes, coarse_bytes,
        coarse_refine, coarse_levels."""
        idx = {"setup_seconds": 0, "device_bytes": 1, "coarse_dofs": 2, "factor_bytes": 3,
               "coarse_bytes": 4, "coarse_refine": 5, "coarse_levels": 6}[what]
        v = ctypes.c_double()
        _check(lib().mrcm3d_query(self._ptr, idx, ctypes.byref(v)))
        return v.value


def set_allocator(alloc=None, release=None):
    """mrcm_set_allocator: alloc(nbytes, stream_handle) -> device pointer (int),
    release(ptr, stream_handle); None restores hipMalloc / hipFree.  Contexts
    set up while a pair is installed allocate through it; close them before
    installing another pair or letting the callables go."""
    global _allocator
    if alloc is None or release is None:
        lib().mrcm_set_allocator(ALLOC_FN(), FREE_FN())
        _allocator = None
        return

    def _a(nbytes, stream):
        try:
            return int(alloc(int(nbytes), stream))
        except Exception:
            return 0

    def _f(ptr, stream):
        try:
            release(int(ptr), stream)
        except Exception:
            pass

    pair = (ALLOC_FN(_a), FREE_FN(_f))
    lib().mrcm_set_allocator(*pair)
    _allocator = pair


def torch_allocator(device: int = 0):
    """(alloc, release) that take device memory from torch's caching
    allocator on the stream the library names."""
    import torch

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, device, stream or 0)

    def release(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, release


def apply_many(contexts, rs, zs, stream=None):
    """z_i = T_i r_i for several contexts in one call (mrcm_apply_many)."""
    n = len(contexts)
    if not (len(rs) == len(zs) == n):
        raise ValueError("contexts, rs and zs must have the same length")
    P = ctypes.c_void_p
    ctx = (P * n)(*[c._ptr for c in contexts])
    rp = (P * n)(*[_dptr(r) for r in rs])
    zp = (P * n)(*[_dptr(z, r.numel()) for r, z in zip(rs, zs)])
    k = (ctypes.c_int32 * n)(*[c._nrhs(r) for c, r in zip(contexts, rs)])
    _check(lib().mrcm_apply_many(ctx, n, rp, zp, k, _stream(stream)))


class Batch:
    """Batched GMRES over several contexts in ticks (gmres_batch_*)."""

    def __init__(self, restart: int = 10):
        self._ptr = ctypes.c_void_p()
        _check(lib().gmres_batch_create(restart, ctypes.byref(self._ptr)))

    def add(self, ctx: "Context", b, p, rtol: float = 1e-8, maxit: int = 300,
            stream=None) -> int:
        """Add the right-hand sides b of a context (solutions into p); returns the tag."""
        tag = ctypes.c_int32()
        _check(lib().gmres_batch_add(self._ptr, ctx._ptr, _dptr(b), _dptr(p, b.numel()),
                                     ctx._nrhs(b), rtol, maxit, _stream(stream),
                                     ctypes.byref(tag)))
        return tag.value

    def tick(self) -> int:
        """One tick; returns the right-hand sides still running."""
        active = ctypes.c_int32()
        _check(lib().gmres_batch_tick(self._ptr, ctypes.byref(active)))
        return active.value

    def poll(self, tag: int):
        """None while the tag runs, else its SolveStats."""
        done = ctypes.c_int32()
        st = Stats(0, 0, 0, 0, 0, 0, 0.0, None, None)
        _check(lib().gmres_batch_poll(self._ptr, tag, ctypes.byref(done), ctypes.byref(st)))
        if not done.value:
            return None
        return SolveStats(st.iterations, st.cycles, bool(st.converged), st.final_relres, [], [])

    def remove(self, tag: int) -> None:
        _check(lib().gmres_batch_remove(self._ptr, tag))

    def close(self):
        if self._ptr:
            lib().gmres_batch_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t, n_expected: int | None = None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 \
            or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 device tensor")
    if n_expected is not None and t.numel() != n_expected:
        raise ValueError(f"expected {n_expected} values, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class SolveStats:
    iterations: int
    cycles: int
    converged: bool
    final_relres: float
    est_history: list
    true_history: list


class Context:
    """A set-up MRCM-OS operator for one permeability field (mrcm_setup)."""

    def __init__(self, cfg: Config, K, stream=None):
        self.cfg = cfg
        self.n = cfg.nx * cfg.ny
        self._ptr = ctypes.c_void_p()
        self._g, self._p = cfg.grid(), cfg.params()
        _check(lib().mrcm_setup(ctypes.byref(self._g), ctypes.byref(self._p),
                                _dptr(K, self.n), _stream(stream), ctypes.byref(self._ptr)))

    def close(self):
        if self._ptr:
            lib().mrcm_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _nrhs(self, t) -> int:
        if t.numel() % self.n:
            raise ValueError("vector length is not a multiple of the cell count")
        return t.numel() // self.n

    def query(self, what: str) -> float:
        """mrcm_query: setup_seconds, device_bytes, coarse_pivot, coarse_levels, coarse_dofs,
        coarse_bytes, coarse_launches."""
        v = ctypes.c_double()
        _check(lib().mrcm_query(self._ptr, QUERIES[what], ctypes.byref(v)))
        return v.value

    def timing(self, on: bool):
        """Start (and clear) or stop per-phase event timing (mrcm_timing_enable)."""
        _check(lib().mrcm_timing_enable(self._ptr, 1 if on else 0))

    def timing_read(self) -> dict:
        """{phase: (total device ms, launches)} since timing(True)."""
        ms = (ctypes.c_double * 6)()
        cnt = (ctypes.c_int64 * 6)()
        _check(lib().mrcm_timing_read(self._ptr, ms, cnt))
        return {PHASES[k]: (ms[k], cnt[k]) for k in range(6)}

    def apply(self, r, z, stream=None):
        """z = T r (mrcm_apply)."""
        k = self._nrhs(r)
        _check(lib().mrcm_apply(self._ptr, _dptr(r), _dptr(z, r.numel()), k, _stream(stream)))

    def apply_noalloc(self, r, z, stream=None):
        """z = T r with the library's static work space (mrcm_apply_noalloc)."""
        k = self._nrhs(r)
        _check(lib().mrcm_apply_noalloc(self._ptr, _dptr(r), _dptr(z, r.numel()), k,
                                        _stream(stream)))

    def op(self, x, y, stream=None):
        """y = A x (op_apply)."""
        k = self._nrhs(x)
        _check(lib().op_apply(self._ptr, _dptr(x), _dptr(y, x.numel()), k, _stream(stream)))

    def rhs(self, f, g_bc, h: float, b, stream=None):
        _check(lib().mrcm_rhs(self._ptr, None if f is None else _dptr(f, self.n),
                              None if g_bc is None else _dptr(g_bc), h, _dptr(b, self.n),
                              _stream(stream)))

    def set_lanes(self, lanes: int) -> None:
        """mrcm_set_lanes: right-hand sides one gmres call advances at once."""
        _check(lib().mrcm_set_lanes(self._ptr, lanes))

    def set_batch(self, width: int) -> None:
        """mrcm_set_batch: right-hand sides one lane advances together."""
        _check(lib().mrcm_set_batch(self._ptr, width))

    def gmres(self, b, p, rtol: float = 1e-8, restart: int = 10, maxit: int = 300,
              stream=None, raise_on_noconv: bool = True) -> SolveStats:
        """Solve A p = b (gmres_solve)."""
        k = self._nrhs(b)
        cap = max(1, maxit * 2 + 8)
        est = (ctypes.c_double * cap)()
        tru = (ctypes.c_double * cap)()
        st = Stats(0, 0, 0, cap, 0, 0, 0.0, est, tru)
        code = lib().gmres_solve(self._ptr, _dptr(b), _dptr(p, b.numel()), k, rtol, restart,
                                 maxit, ctypes.byref(st), _stream(stream))
        if code != MRCM_OK and (code != MRCM_ENOCONV or raise_on_noconv):
            _check(code)
        return SolveStats(st.iterations, st.cycles, bool(st.converged), st.final_relres,
                          list(est[:st.hist_len]), list(tru[:st.true_len]))
