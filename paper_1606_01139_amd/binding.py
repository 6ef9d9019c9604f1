"""ctypes binding of libtransec_gpu (include/transec_gpu.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory and the stream for the calls that
take device buffers.  There is no fallback: if the library is missing or no
gfx950 device is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .build import library_path

TSG_OK, TSG_EINVAL, TSG_ENOMEM, TSG_ENOCONV, TSG_EBREAKDOWN, TSG_EDEVICE, TSG_ESTATE, TSG_ECAPACITY = range(8)
STATUS_NAMES = ["TSG_OK", "TSG_EINVAL", "TSG_ENOMEM", "TSG_ENOCONV", "TSG_EBREAKDOWN", "TSG_EDEVICE",
                "TSG_ESTATE", "TSG_ECAPACITY"]
FP64, FP32_BULK = 0, 1
PLAN_ALG1, PLAN_EQUAL, PLAN_SAMPLED, PLAN_SEMICLASSICAL = 0, 1, 2, 3
SELECT_NEAREST, SELECT_SMALLEST_REAL, SELECT_LARGEST_REAL = 0, 1, 2
C128, C64 = 0, 1
EXTRACT_RITZ, EXTRACT_HARMONIC = 0, 1

# Every symbol include/transec_gpu.h declares.
EXPORTS = [
    "tsg_default_opts", "tsg_build_operator", "tsg_plan_windows", "tsg_solve_partition",
    "tsg_solve_all_partitions", "tsg_fill_holes", "tsg_solve_batch", "tsg_combine", "tsg_get_eigenvalues", "tsg_get_eigenvectors",
    "tsg_get_partition", "tsg_get_stats", "tsg_transmission", "tsg_transmission_vjp", "tsg_apply_operator",
    "tsg_dense_eig", "tsg_dense_eig_noalloc", "tsg_tune_stencil", "tsg_load_tuning",
    "tsg_stencil_geometry",
    "tsg_last_error", "tsg_destroy",
]


class TsgGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double),
                ("fd_radius", C.c_int32)]


class TsgAbsorber(C.Structure):
    _fields_ = [("amp_L", C.c_double), ("width_L", C.c_double), ("z_L", C.c_double),
                ("amp_R", C.c_double), ("width_R", C.c_double), ("z_R", C.c_double)]


class TsgWindow(C.Structure):
    _fields_ = [("shift", C.c_double), ("nev", C.c_int32), ("shift_im", C.c_double)]


def _window(shift, nev) -> TsgWindow:
    """tsg_window from a real or complex shift."""
    z = complex(shift)
    return TsgWindow(z.real, int(nev), z.imag)


def _shift_of(w: TsgWindow):
    return complex(w.shift, w.shift_im) if w.shift_im != 0.0 else w.shift


class TsgOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("tol", C.c_double), ("block", C.c_int32), ("basis", C.c_int32),
                ("keep", C.c_int32), ("max_restarts", C.c_int32), ("seed", C.c_uint64),
                ("keep_lowest", C.c_int32), ("select", C.c_int32), ("bulk_tol", C.c_double),
                ("graphs", C.c_int32), ("groups", C.c_int32), ("imag_bands", C.c_int32),
                ("extraction", C.c_int32)]


class TsgWindowStats(C.Structure):
    _fields_ = [("shift", C.c_double), ("nev", C.c_int32), ("n_conv", C.c_int32), ("restarts", C.c_int32),
                ("matvecs", C.c_int64), ("max_backward_error", C.c_double), ("restarts_bulk", C.c_int32),
                ("breakdowns", C.c_int32), ("cnorm_failures", C.c_int32), ("shift_im", C.c_double)]


class TsgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")
        self.status = status


_LIB: Optional[C.CDLL] = None
DEFAULT_TUNING = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "stencil_gfx950.json")


def load(path: Optional[str] = None) -> C.CDLL:
    """Loads the built library; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    p = path or library_path()
    if not os.path.exists(p):
        raise RuntimeError(f"libtransec_gpu is not built ({p} missing); run __graft_entry__.build()")
    lib = C.CDLL(p)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    lib.tsg_default_opts.argtypes = [C.POINTER(TsgOpts)]
    lib.tsg_default_opts.restype = None
    lib.tsg_build_operator.argtypes = [C.POINTER(TsgGrid), dp, C.POINTER(TsgAbsorber), vp, C.POINTER(vp)]
    lib.tsg_plan_windows.argtypes = [vp, i32, i32, i32, C.POINTER(TsgOpts), C.POINTER(TsgWindow), dp]
    lib.tsg_solve_partition.argtypes = [vp, TsgWindow, C.POINTER(TsgOpts), C.POINTER(i32)]
    lib.tsg_solve_all_partitions.argtypes = [vp, C.POINTER(TsgWindow), i32, C.POINTER(TsgOpts), C.POINTER(i32),
                                             C.POINTER(C.c_uint8)]
    lib.tsg_fill_holes.argtypes = [vp, C.c_double, i32, i32, C.POINTER(TsgOpts), C.POINTER(i32), C.POINTER(i32),
                                   C.POINTER(i32), C.POINTER(i32)]
    lib.tsg_solve_batch.argtypes = [C.POINTER(vp), i32, C.POINTER(C.POINTER(TsgWindow)), C.POINTER(i32),
                                    C.POINTER(TsgOpts), C.POINTER(i32)]
    lib.tsg_combine.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(C.c_uint8)]
    lib.tsg_get_eigenvalues.argtypes = [vp, dp, i32, C.POINTER(i32)]
    lib.tsg_get_eigenvectors.argtypes = [vp, C.POINTER(vp), C.POINTER(i64), C.POINTER(i32)]
    lib.tsg_get_partition.argtypes = [vp, i32, dp, i32, C.POINTER(i32), C.POINTER(vp), C.POINTER(i64)]
    lib.tsg_get_stats.argtypes = [vp, i32, C.POINTER(TsgWindowStats)]
    lib.tsg_transmission.argtypes = [vp, dp, i32, dp]
    lib.tsg_transmission_vjp.argtypes = [vp, dp, i32, dp, dp, dp]
    lib.tsg_apply_operator.argtypes = [vp, vp, vp, i32, i64, i32]
    lib.tsg_dense_eig.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    lib.tsg_dense_eig_noalloc.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    lib.tsg_tune_stencil.argtypes = [vp, i32, i32, i32, C.c_char_p, C.POINTER(i32), dp]
    lib.tsg_load_tuning.argtypes = [C.c_char_p, C.POINTER(i32)]
    lib.tsg_stencil_geometry.argtypes = [i32, i32, i32, i32, i32, i32, C.POINTER(i32)]
    lib.tsg_last_error.argtypes = [vp]
    lib.tsg_last_error.restype = C.c_char_p
    lib.tsg_destroy.argtypes = [vp]
    lib.tsg_destroy.restype = None
    for name in EXPORTS:
        f = getattr(lib, name)
        if f.restype is C.c_int:  # default restype
            f.restype = C.c_int
    _LIB = lib
    # stencil geometries measured by the autotuner (tune.py), if present
    tpath = os.environ.get("TSG_TUNING_FILE") or DEFAULT_TUNING
    if tpath and os.path.exists(tpath):
        n = C.c_int32()
        if lib.tsg_load_tuning(tpath.encode(), C.byref(n)) != TSG_OK:
            raise RuntimeError(f"tuning file {tpath}: {lib.tsg_last_error(None).decode(errors='replace')}")
    return lib


def _check(lib, ctx, status: int, allow=()):
    if status != TSG_OK and status not in allow:
        raise TsgError(status, lib.tsg_last_error(ctx).decode(errors="replace"))
    return status


def default_opts(**kw) -> TsgOpts:
    lib = load()
    o = TsgOpts()
    lib.tsg_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(f"tsg_opts has no field {k}")
        setattr(o, k, v)
    return o


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None  # the library reports the missing device itself
        return torch.cuda.current_stream().cuda_stream or None
    return int(stream)


class _DevView:
    """__cuda_array_interface__ wrapper for a borrowed device pointer."""

    def __init__(self, ptr: int, shape, typestr: str, strides=None):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 2,
                                         "strides": strides}


def _complex_view(ptr: int, rows: int, cols: int, ld: int):
    """rows x cols complex128 view of `cols` contiguous vectors at stride ld."""
    import torch
    if rows * cols == 0 or not ptr:
        return torch.zeros((rows, cols), dtype=torch.complex128, device="cuda")
    v = _DevView(ptr, (rows, cols), "<c16", (16, ld * 16))
    return torch.as_tensor(v, device="cuda")


@dataclass
class WindowStats:
    shift: float
    nev: int
    n_conv: int
    restarts: int
    matvecs: int
    max_backward_error: float
    restarts_bulk: int
    breakdowns: int = 0
    cnorm_failures: int = 0
    shift_im: float = 0.0


class Operator:
    """A context: the operator of Eq. (1) plus the partitions solved on it."""

    def __init__(self, nx: int, ny: int, nz: int, h: float, V: np.ndarray, absorber: Sequence[float],
                 fd_radius: int = 6, stream=None):
        self.lib = load()
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        V = np.ascontiguousarray(V, dtype=np.float64)
        g = TsgGrid(nx, ny, nz, h, fd_radius)
        ab = TsgAbsorber(*[float(x) for x in absorber])
        ctx = C.c_void_p()
        st = _stream_handle(stream)
        s = self.lib.tsg_build_operator(C.byref(g), V.ctypes.data_as(C.POINTER(C.c_double)), C.byref(ab),
                                        C.c_void_p(st) if st else None, C.byref(ctx))
        _check(self.lib, None, s)
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.tsg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- K1
    def apply(self, X, Y):
        """Y = A X for X, Y of shape (ncols, N): one grid vector per row."""
        import torch
        assert X.is_cuda and Y.is_cuda and X.dim() == 2 and X.shape[1] == self.N and Y.shape == X.shape
        assert X.stride(1) == 1 and Y.stride(1) == 1 and X.stride(0) == Y.stride(0)
        dt = {torch.complex128: C128, torch.complex64: C64}[X.dtype]
        assert Y.dtype == X.dtype
        s = self.lib.tsg_apply_operator(self.ctx, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
                                        X.shape[0], X.stride(0), dt)
        _check(self.lib, self.ctx, s)

    # -- Algorithm 1 planning
    def plan_windows(self, n_r: int, p: int, mode: int = PLAN_ALG1, opts: Optional[TsgOpts] = None):
        out = (TsgWindow * p)()
        er = (C.c_double * 2)()
        s = self.lib.tsg_plan_windows(self.ctx, n_r, p, mode, C.byref(opts) if opts else None, out, er)
        _check(self.lib, self.ctx, s)
        return [(_shift_of(w), w.nev) for w in out], (er[0], er[1])

    def solve_partition(self, shift: float, nev: int, opts: Optional[TsgOpts] = None, allow_noconv=False) -> int:
        n = C.c_int32()
        s = self.lib.tsg_solve_partition(self.ctx, _window(shift, nev), C.byref(opts) if opts else None,
                                         C.byref(n))
        _check(self.lib, self.ctx, s, allow=(TSG_ENOCONV,) if allow_noconv else ())
        return n.value

    def solve_all_partitions(self, windows: Sequence[Tuple[float, int]], opts: Optional[TsgOpts] = None,
                             allow_noconv=False):
        p = len(windows)
        arr = (TsgWindow * p)(*[_window(s, n) for s, n in windows])
        n = C.c_int32()
        holes = (C.c_uint8 * max(p - 1, 1))()
        s = self.lib.tsg_solve_all_partitions(self.ctx, arr, p, C.byref(opts) if opts else None, C.byref(n),
                                              holes)
        status = _check(self.lib, self.ctx, s, allow=(TSG_ENOCONV, TSG_EBREAKDOWN) if allow_noconv else ())
        return n.value, [bool(holes[i]) for i in range(p - 1)], status

    def fill_holes(self, e_min: float, n_cap: int, max_rounds: int, opts: Optional[TsgOpts] = None,
                   allow_noconv=False):
        """Algorithm 1's repeat loop on the stored partitions (tsg_fill_holes).
        Returns (partitions added, rounds run, combined count, flags left, status)."""
        out = [C.c_int32() for _ in range(4)]
        s = self.lib.tsg_fill_holes(self.ctx, float(e_min), int(n_cap), int(max_rounds),
                                    C.byref(opts) if opts else None, *[C.byref(x) for x in out])
        status = _check(self.lib, self.ctx, s, allow=(TSG_ENOCONV,) if allow_noconv else ())
        return (*[x.value for x in out], status)

    def combine(self, keep_lowest: int = 0):
        n = C.c_int32()
        holes = (C.c_uint8 * 4096)()
        s = self.lib.tsg_combine(self.ctx, keep_lowest, C.byref(n), holes)
        _check(self.lib, self.ctx, s)
        return n.value, holes

    def eigenvalues(self) -> np.ndarray:
        n = C.c_int32()
        s = self.lib.tsg_get_eigenvalues(self.ctx, None, 0, C.byref(n))
        if s not in (TSG_OK, TSG_ECAPACITY):
            _check(self.lib, self.ctx, s)
        buf = np.zeros(2 * max(n.value, 1))
        s = self.lib.tsg_get_eigenvalues(self.ctx, buf.ctypes.data_as(C.POINTER(C.c_double)), n.value,
                                         C.byref(n))
        _check(self.lib, self.ctx, s)
        return buf[0:2 * n.value:2] + 1j * buf[1:2 * n.value:2]

    def eigenvectors(self):
        """Borrowed zero-copy torch view (N x n complex128) of the combined set."""
        p = C.c_void_p()
        ld = C.c_int64()
        n = C.c_int32()
        s = self.lib.tsg_get_eigenvectors(self.ctx, C.byref(p), C.byref(ld), C.byref(n))
        _check(self.lib, self.ctx, s)
        return _complex_view(p.value or 0, self.N, n.value, ld.value)

    def partition(self, j: int):
        n = C.c_int32()
        s = self.lib.tsg_get_partition(self.ctx, j, None, 0, C.byref(n), None, None)
        _check(self.lib, self.ctx, s)
        buf = np.zeros(2 * max(n.value, 1))
        p = C.c_void_p()
        ld = C.c_int64()
        s = self.lib.tsg_get_partition(self.ctx, j, buf.ctypes.data_as(C.POINTER(C.c_double)), n.value,
                                       C.byref(n), C.byref(p), C.byref(ld))
        _check(self.lib, self.ctx, s)
        eps = buf[0:2 * n.value:2] + 1j * buf[1:2 * n.value:2]
        return eps, _complex_view(p.value or 0, self.N, n.value, ld.value)

    def stats(self, j: int) -> WindowStats:
        st = TsgWindowStats()
        s = self.lib.tsg_get_stats(self.ctx, j, C.byref(st))
        _check(self.lib, self.ctx, s)
        return WindowStats(st.shift, st.nev, st.n_conv, st.restarts, st.matvecs, st.max_backward_error,
                           st.restarts_bulk, st.breakdowns, st.cnorm_failures, st.shift_im)

    def tune_stencil(self, ncols: int, dtype: int = C128, reps: int = 10, path: Optional[str] = None):
        """tsg_tune_stencil: times every candidate stencil geometry for a
        launch of ncols vectors on this grid and keeps the fastest.  Returns
        ({tx, yb, zchunk, xcd, nt, cb, tried}, best microseconds per launch)."""
        g = (C.c_int32 * 7)()
        us = C.c_double()
        s = self.lib.tsg_tune_stencil(self.ctx, int(ncols), int(dtype), int(reps),
                                      path.encode() if path else None, g, C.byref(us))
        _check(self.lib, self.ctx, s)
        return {"tx": g[0], "yb": g[1], "zchunk": g[2], "xcd": g[3], "nt": g[4], "cb": g[5], "tried": g[6]}, us.value

    def transmission(self, energies: Sequence[float]) -> np.ndarray:
        E = np.ascontiguousarray(energies, dtype=np.float64)
        T = np.zeros(len(E))
        s = self.lib.tsg_transmission(self.ctx, E.ctypes.data_as(C.POINTER(C.c_double)), len(E),
                                      T.ctypes.data_as(C.POINTER(C.c_double)))
        _check(self.lib, self.ctx, s)
        return T


    def transmission_vjp(self, energies: Sequence[float], dL_dT: Sequence[float], allow_noconv=False):
        """Gradient of sum_e dL_dT[e] T(E[e]) w.r.t. V (N,) and
        (amp_L, width_L, amp_R, width_R) (4,).  With allow_noconv, a
        projected solve that missed its tolerance (TSG_ENOCONV, outputs
        still written) does not raise; the status is in self.vjp_status."""
        E = np.ascontiguousarray(energies, dtype=np.float64)
        w = np.ascontiguousarray(dL_dT, dtype=np.float64)
        assert w.shape == E.shape
        dV = np.zeros(self.N)
        dab = np.zeros(4)
        dp = C.POINTER(C.c_double)
        s = self.lib.tsg_transmission_vjp(self.ctx, E.ctypes.data_as(dp), len(E), w.ctypes.data_as(dp),
                                          dV.ctypes.data_as(dp), dab.ctypes.data_as(dp))
        self.vjp_status = _check(self.lib, self.ctx, s, allow=(TSG_ENOCONV,) if allow_noconv else ())
        return dV, dab


def solve_batch(operators: Sequence["Operator"], windows: Sequence[Sequence[Tuple[float, int]]],
                opts: Optional[TsgOpts] = None, allow_noconv=False):
    """All windows of several systems in one batched iteration
    (tsg_solve_batch).  Returns the unique count per system and the status."""
    lib = load()
    ns = len(operators)
    ctxs = (C.c_void_p * ns)(*[op.ctx for op in operators])
    arrs = [(TsgWindow * len(w))(*[_window(s, n) for s, n in w]) for w in windows]
    ptrs = (C.POINTER(TsgWindow) * ns)(*[C.cast(a, C.POINTER(TsgWindow)) for a in arrs])
    p = (C.c_int32 * ns)(*[len(w) for w in windows])
    nu = (C.c_int32 * ns)()
    s = lib.tsg_solve_batch(ctxs, ns, ptrs, p, C.byref(opts) if opts else None, nu)
    status = _check(lib, operators[0].ctx, s, allow=(TSG_ENOCONV,) if allow_noconv else ())
    return [nu[i] for i in range(ns)], status


def dense_eig(H, stream=None):
    """Batched dense eigen-decomposition on the device (K4).

    H: torch complex128 CUDA tensor (batch, m, m), row-major; overwritten.
    Returns (theta (batch, m), Y (batch, m, m) unit-norm eigenvector columns, info (batch,))."""
    import torch
    lib = load()
    assert H.is_cuda and H.dtype == torch.complex128 and H.dim() == 3 and H.is_contiguous()
    b, m, _ = H.shape
    theta = torch.empty((b, m), dtype=torch.complex128, device=H.device)
    Y = torch.empty((b, m, m), dtype=torch.complex128, device=H.device)
    info = torch.empty((b,), dtype=torch.int32, device=H.device)
    st = _stream_handle(stream)
    s = lib.tsg_dense_eig(C.c_void_p(H.data_ptr()), m, b, C.c_void_p(theta.data_ptr()),
                          C.c_void_p(Y.data_ptr()), C.c_void_p(info.data_ptr()), C.c_void_p(st) if st else None)
    _check(lib, None, s)
    return theta, Y, info


def dense_eig_noalloc(H, theta, Y, info, stream=None):
    """tsg_dense_eig_noalloc: the batched dense eigen-decomposition into
    caller-provided outputs with the library's fixed device scratch (no
    allocation, no synchronisation).  H (batch, m, m) complex128 is
    overwritten; theta (batch, m), Y (batch, m, m) complex128 and info
    (batch,) int32 are outputs."""
    import torch
    lib = load()
    assert H.is_cuda and H.dtype == torch.complex128 and H.dim() == 3 and H.is_contiguous()
    b, m, _ = H.shape
    assert theta.shape == (b, m) and theta.dtype == torch.complex128 and theta.is_contiguous()
    assert Y.shape == (b, m, m) and Y.dtype == torch.complex128 and Y.is_contiguous()
    assert info.shape == (b,) and info.dtype == torch.int32
    st = _stream_handle(stream)
    s = lib.tsg_dense_eig_noalloc(C.c_void_p(H.data_ptr()), m, b, C.c_void_p(theta.data_ptr()),
                                  C.c_void_p(Y.data_ptr()), C.c_void_p(info.data_ptr()),
                                  C.c_void_p(st) if st else None)
    _check(lib, None, s)


def load_tuning(path: str) -> int:
    """tsg_load_tuning: reads a stencil tuning file into the library's table."""
    lib = load()
    n = C.c_int32()
    _check(lib, None, lib.tsg_load_tuning(path.encode(), C.byref(n)))
    return n.value


def stencil_geometry(nx: int, ny: int, nz: int, ncols: int, dtype: int = C128, radius: int = 6) -> dict:
    """tsg_stencil_geometry: the launch geometry the library uses for ncols
    vectors of this grid (the tuned entry if the table holds one)."""
    lib = load()
    g = (C.c_int32 * 7)()
    _check(lib, None, lib.tsg_stencil_geometry(int(nx), int(ny), int(nz), int(radius), int(ncols), int(dtype), g))
    return {"tx": g[0], "yb": g[1], "zchunk": g[2], "xcd": g[3], "nt": g[4], "cb": g[5], "tuned": bool(g[6])}
