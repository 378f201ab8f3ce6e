"""Python binding of libssart (ctypes): argument marshalling only.

Every computation runs in the library's own code (host C++ for the system
build, HIP kernels for everything on the device).  PyTorch provides device
memory and the current stream; nothing here computes on tensors.  Importing
this module never falls back to anything else: if the library is missing the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libssart.so")

SS_OK, SS_NOT_CONVERGED = 0, 1
WDTYPES = {"f32": 0, "bf16": 1, "f16": 2}


class SSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[ssart {code}] {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nz", C.c_int32), ("pitch", C.c_double)]


class GeometryC(C.Structure):
    _fields_ = [("K", C.c_int32), ("src_x", C.POINTER(C.c_double)),
                ("src_z", C.POINTER(C.c_double)), ("B", C.c_int32),
                ("bin_x", C.POINTER(C.c_double)), ("det_z", C.c_double)]


class PolarGridC(C.Structure):
    _fields_ = [("rings", C.c_int32), ("sectors", C.c_int32), ("radius", C.c_double)]


class ParallelScanC(C.Structure):
    _fields_ = [("K", C.c_int32), ("phi", C.POINTER(C.c_double)), ("B", C.c_int32),
                ("offset", C.POINTER(C.c_double))]


class MatrixC(C.Structure):
    _fields_ = [("M", C.c_int64), ("N", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.POINTER(C.c_int64)), ("col_idx", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_float)), ("col_ptr", C.POINTER(C.c_int64)),
                ("row_idx", C.POINTER(C.c_int32)), ("val_t", C.POINTER(C.c_float))]


class MatrixDevC(C.Structure):
    _fields_ = [("M", C.c_int64), ("N", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("col_ptr", C.c_void_p), ("row_idx", C.c_void_p), ("val_t", C.c_void_p)]


class SystemC(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("nvals", C.c_int32), ("wdtype", C.c_int32),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("col_ptr", C.c_void_p), ("row_idx", C.c_void_p), ("val_t", C.c_void_p),
                ("p", C.c_void_p), ("inv_row", C.c_void_p), ("inv_col", C.c_void_p),
                ("row_lanes", C.c_int32), ("col_lanes", C.c_int32)]


class SartOptsC(C.Structure):
    _fields_ = [("lambda_", C.c_float), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("check_every", C.c_int32), ("use_graph", C.c_int32),
                ("rows_per_wave", C.c_int32), ("cols_per_wave", C.c_int32),
                ("xcd_remap", C.c_int32), ("zero_start", C.c_int32),
                ("unroll", C.c_int32), ("persistent", C.c_int32), ("chunked", C.c_int32),
                ("nonneg", C.c_int32), ("staged", C.c_int32), ("band_width", C.c_int32),
                ("tile_cols", C.c_int32), ("tile_entries", C.c_int32), ("residual_every", C.c_int32)]


class SubsetsC(C.Structure):
    _fields_ = [("S", C.c_int32), ("col_sub", C.c_void_p), ("inv_col_sub", C.c_void_p),
                ("col_ptr_os", C.c_void_p), ("row_idx_os", C.c_void_p), ("val_t_os", C.c_void_p)]


_SIGNATURES = {
    "ss_last_error": (C.c_char_p, []),
    "ss_version": (C.c_char_p, []),
    "ss_build_polar_system": (C.c_int32, [C.POINTER(PolarGridC), C.POINTER(ParallelScanC), C.c_int32,
                               C.POINTER(MatrixC)]),
    "ss_build_system": (C.c_int32, [C.POINTER(Grid), C.POINTER(GeometryC), C.c_int32,
                                    C.POINTER(MatrixC)]),
    "ss_matrix_free": (None, [C.POINTER(MatrixC)]),
    "ss_snake_order": (C.c_int32, [C.POINTER(Grid), C.POINTER(C.c_int64)]),
    "ss_stream_len": (C.c_int64, [C.c_int64]),
    "ss_normal_workspace_bytes": (C.c_int32, [C.POINTER(SystemC), C.POINTER(C.c_size_t)]),
    "ss_normal_solve": (C.c_int32, [C.POINTER(SystemC), C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "ss_subsets_build": (C.c_int32, [C.POINTER(SystemC), C.POINTER(SubsetsC), C.c_void_p]),
    "ss_ossart_workspace_bytes": (C.c_int32, [C.POINTER(SystemC), C.POINTER(SubsetsC), C.c_int32,
                                              C.POINTER(SartOptsC), C.POINTER(C.c_size_t)]),
    "ss_ossart_solve": (C.c_int32, [C.POINTER(SystemC), C.POINTER(SubsetsC), C.c_int32, C.POINTER(C.c_void_p),
                                    C.POINTER(C.c_void_p), C.POINTER(SartOptsC), C.POINTER(C.c_int32),
                                    C.c_void_p, C.c_size_t, C.c_void_p]),
    "ss_fold_workspace_bytes": (C.c_int32, [C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "ss_recombine_batch": (C.c_int32, [C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_void_p),
                                       C.c_int32, C.c_void_p]),
    "ss_fold_batch_workspace_bytes": (C.c_int32, [C.POINTER(MatrixDevC), C.c_int32, C.POINTER(C.c_size_t)]),
    "ss_fold_batch": (C.c_int32, [C.POINTER(MatrixDevC), C.POINTER(C.c_void_p), C.POINTER(SystemC), C.c_int32,
                                  C.c_void_p, C.c_size_t, C.c_void_p]),
    "ss_fold_size": (C.c_int32, [C.POINTER(MatrixDevC), C.c_void_p, C.c_void_p, C.c_size_t,
                                 C.POINTER(C.c_int64), C.c_void_p]),
    "ss_fold_size_batch": (C.c_int32, [C.POINTER(MatrixDevC), C.POINTER(C.c_void_p), C.c_int32, C.c_void_p,
                                       C.c_size_t, C.POINTER(C.c_int64), C.c_void_p]),
    "ss_fold": (C.c_int32, [C.POINTER(MatrixDevC), C.c_void_p, C.POINTER(SystemC), C.c_void_p,
                            C.c_size_t, C.c_void_p]),
    "ss_fold_noalloc": (C.c_int32, [C.POINTER(MatrixDevC), C.c_void_p, C.POINTER(SystemC), C.c_void_p]),
    "ss_unsplit": (C.c_int32, [C.POINTER(MatrixDevC), C.c_void_p, C.POINTER(SystemC), C.c_void_p]),
    "ss_sart_workspace_bytes": (C.c_int32, [C.POINTER(SystemC), C.c_int32, C.POINTER(SartOptsC),
                                            C.POINTER(C.c_size_t)]),
    "ss_sart_solve": (C.c_int32, [C.POINTER(SystemC), C.c_int32, C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_void_p), C.POINTER(SartOptsC),
                                  C.POINTER(C.c_int32), C.c_void_p, C.c_size_t, C.c_void_p]),
    "ss_sart_time_kernels": (C.c_int32, [C.POINTER(SystemC), C.c_int32, C.POINTER(C.c_void_p),
                                         C.POINTER(SartOptsC), C.c_int32,
                                         C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.c_void_p, C.c_size_t, C.c_void_p]),
    "ss_sart_time_phases": (C.c_int32, [C.POINTER(SystemC), C.c_int32, C.POINTER(C.c_void_p),
                                        C.POINTER(SartOptsC), C.c_int32, C.POINTER(C.c_double),
                                        C.c_void_p, C.c_size_t, C.c_void_p]),
    "ss_sart_staged_info": (C.c_int32, [C.POINTER(SystemC), C.c_int32, C.POINTER(C.c_void_p),
                                        C.POINTER(SartOptsC), C.POINTER(C.c_int64), C.c_void_p, C.c_size_t,
                                        C.c_void_p]),
    "ss_sart_autotune": (C.c_int32, [C.POINTER(SystemC), C.c_int32, C.POINTER(C.c_void_p),
                                     C.POINTER(SartOptsC), C.c_void_p, C.c_size_t, C.c_void_p]),
    "ss_recombine": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "ss_image_fold": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "ss_project": (C.c_int32, [C.POINTER(MatrixDevC), C.c_void_p, C.c_void_p, C.c_void_p]),
    "ss_fold_rhs": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "ss_nn_prep_weights": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
    "ss_nn_conv3x3": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                  C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p]),
    "ss_nn_wgrad_workspace_bytes": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                                C.POINTER(C.c_size_t)]),
    "ss_nn_conv3x3_wgrad": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                        C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_size_t, C.c_void_p]),
    "ss_nn_mse_workspace_bytes": (C.c_int32, [C.c_int64, C.POINTER(C.c_size_t)]),
    "ss_nn_relu_mask": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "ss_nn_pool2": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                C.c_void_p]),
    "ss_nn_pool2_grad": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                     C.c_int32, C.c_void_p]),
    "ss_nn_to_slice": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                   C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "ss_nn_from_slice": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p]),
    "ss_nn_residual_mse": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "ss_nn_to_bf16": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "ss_nn_adam": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float,
                               C.c_float, C.c_float, C.c_float, C.c_int32, C.c_void_p]),
    "ss_nn_snake_image": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                      C.c_void_p, C.c_void_p]),
}

_lib = None


def lib() -> C.CDLL:
    """The loaded library (torch is imported first so that both share one HIP
    runtime).  Raises if the library has not been built."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the HIP runtime the library links to)
        if not os.path.exists(LIB_PATH):
            raise SSError(-7, f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, allow_warning: bool = False) -> int:
    if status < 0 or (status > 0 and not allow_warning):
        raise SSError(status, lib().ss_last_error().decode())
    return status


def _stream(device=None) -> C.c_void_p:
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


# ------------------------------------------------------------------ host
@dataclasses.dataclass
class HostMatrix:
    M: int
    N: int
    nnz: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    col_ptr: np.ndarray
    row_idx: np.ndarray
    val_t: np.ndarray

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.M, self.N))


def build_system(geom, nthreads: int = 0) -> HostMatrix:
    """ss_build_system for a scan described by ``inputs.Geometry``."""
    g = Grid(geom.nx, geom.nz, float(geom.pitch))
    sx = np.ascontiguousarray(geom.src_x, dtype=np.float64)
    sz = np.ascontiguousarray(geom.src_z, dtype=np.float64)
    bx = np.ascontiguousarray(geom.bin_x, dtype=np.float64)
    dp = C.POINTER(C.c_double)
    gc = GeometryC(len(sx), sx.ctypes.data_as(dp), sz.ctypes.data_as(dp), len(bx),
                   bx.ctypes.data_as(dp), float(geom.det_z))
    m = MatrixC()
    _check(lib().ss_build_system(C.byref(g), C.byref(gc), int(nthreads), C.byref(m)))
    return _take_host(m)


def build_polar_system(geom, nthreads: int = 0) -> HostMatrix:
    """ss_build_polar_system for a polar grid and parallel scan described by
    ``inputs.PolarGeometry``."""
    g = PolarGridC(int(geom.rings), int(geom.sectors), float(geom.radius))
    phi = np.ascontiguousarray(geom.phi, dtype=np.float64)
    off = np.ascontiguousarray(geom.offset, dtype=np.float64)
    dp = C.POINTER(C.c_double)
    sc = ParallelScanC(len(phi), phi.ctypes.data_as(dp), len(off), off.ctypes.data_as(dp))
    m = MatrixC()
    _check(lib().ss_build_polar_system(C.byref(g), C.byref(sc), int(nthreads), C.byref(m)))
    return _take_host(m)


def _take_host(m: MatrixC) -> HostMatrix:
    """Copies a library-owned host matrix into numpy arrays and frees it."""
    try:
        M, N, nnz = m.M, m.N, m.nnz
        out = HostMatrix(M, N, nnz,
                         np.ctypeslib.as_array(m.row_ptr, shape=(M + 1,)).copy(),
                         np.ctypeslib.as_array(m.col_idx, shape=(max(nnz, 1),))[:nnz].copy(),
                         np.ctypeslib.as_array(m.val, shape=(max(nnz, 1),))[:nnz].copy(),
                         np.ctypeslib.as_array(m.col_ptr, shape=(N + 1,)).copy(),
                         np.ctypeslib.as_array(m.row_idx, shape=(max(nnz, 1),))[:nnz].copy(),
                         np.ctypeslib.as_array(m.val_t, shape=(max(nnz, 1),))[:nnz].copy())
    finally:
        lib().ss_matrix_free(C.byref(m))
    return out


def snake_order(nx: int, nz: int) -> np.ndarray:
    """snake[r, c] = vertical-snake index of voxel (c, r) (ss_snake_order)."""
    out = np.empty(nx * nz, dtype=np.int64)
    g = Grid(nx, nz, 1.0)
    _check(lib().ss_snake_order(C.byref(g), out.ctypes.data_as(C.POINTER(C.c_int64))))
    return out.reshape(nz, nx)


# ---------------------------------------------------------------- device
@dataclasses.dataclass
class DeviceMatrix:
    M: int
    N: int
    nnz: int
    row_ptr: "torch.Tensor"
    col_idx: "torch.Tensor"
    val: "torch.Tensor"
    col_ptr: "torch.Tensor"
    row_idx: "torch.Tensor"
    val_t: "torch.Tensor"

    def c(self) -> MatrixDevC:
        return MatrixDevC(self.M, self.N, self.nnz, _ptr(self.row_ptr), _ptr(self.col_idx),
                          _ptr(self.val), _ptr(self.col_ptr), _ptr(self.row_idx), _ptr(self.val_t))


def to_device(hm, device="cuda") -> DeviceMatrix:
    """Copies a host CSR+CSC (HostMatrix, or any object with the same fields)
    into device tensors."""
    import torch

    def t(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)

    def stream(a, dt):   # room for the solver's chunked reads (ss_stream_len)
        a = np.ascontiguousarray(a, dtype=dt)
        buf = stream_tensor(a.size, 1, {np.int32: torch.int32, np.float32: torch.float32}[dt], device)
        buf.copy_(torch.from_numpy(a))
        return buf
    return DeviceMatrix(int(hm.M), int(hm.N), int(hm.nnz), t(hm.row_ptr, np.int64),
                        stream(hm.col_idx, np.int32), stream(hm.val, np.float32), t(hm.col_ptr, np.int64),
                        stream(hm.row_idx, np.int32), stream(hm.val_t, np.float32))


def stream_len(nnz: int) -> int:
    """ss_stream_len: entries the index/value arrays of a system must hold."""
    return int(lib().ss_stream_len(nnz))


def stream_tensor(nnz: int, per_entry: int, dtype, device):
    """A view of `nnz * per_entry` elements on a buffer with room for
    ss_stream_len(nnz) entries (torch allocations are 512-byte aligned)."""
    import torch
    cap = stream_len(nnz) if nnz > 0 else 0
    buf = torch.empty(max(cap, 1) * per_entry, dtype=dtype, device=device)
    return buf[: nnz * per_entry]


@dataclasses.dataclass
class System:
    """A solver system (ss_system) and the tensors behind it."""
    m: int
    n: int
    nnz: int
    nvals: int
    wdtype: str
    row_ptr: "torch.Tensor"
    col_idx: "torch.Tensor"
    val: "torch.Tensor"
    col_ptr: "torch.Tensor"
    row_idx: "torch.Tensor"
    val_t: "torch.Tensor"
    p: "torch.Tensor"
    inv_row: "torch.Tensor"
    inv_col: "torch.Tensor"
    # order of the entries within each row / column: 0 ascending, L the
    # solver's interleaved order for groups of L lanes (what ss_fold writes)
    row_lanes: int = 0
    col_lanes: int = 0

    def c(self) -> SystemC:
        return SystemC(self.m, self.n, self.nnz, self.nvals, WDTYPES[self.wdtype],
                       _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.val),
                       _ptr(self.col_ptr), _ptr(self.row_idx), _ptr(self.val_t),
                       _ptr(self.p), _ptr(self.inv_row), _ptr(self.inv_col),
                       self.row_lanes, self.col_lanes)

    def new_image(self):
        import torch
        shape = (self.n, 2) if self.nvals == 2 else (self.n,)
        return torch.zeros(shape, dtype=torch.float32, device=self.p.device)


def fold_size(A: DeviceMatrix, p=None) -> int:
    """ss_fold_size: validates A (and p) and returns the shared-pattern size."""
    ws = fold_workspace(A)
    out = C.c_int64()
    mc = A.c()
    _check(lib().ss_fold_size(C.byref(mc), _ptr(p), _ptr(ws), ws.numel(), C.byref(out),
                              _stream(A.val.device)))
    return int(out.value)


def _value_tensor(nnz: int, nvals: int, wdtype: str, device):
    import torch
    dt = torch.float32 if wdtype == "f32" else torch.int16   # int16: raw 16-bit storage
    return stream_tensor(nnz, nvals, dt, device)


def fold(A: DeviceMatrix, p, wdtype: str = "f32", nnz_half: int | None = None, row_lanes: int = 0,
         col_lanes: int = 0) -> System:
    """ss_fold: the split pair (A(1), A(2)), (p1, p2) and the SART sums;
    rows (columns) written in the interleaved order for row_lanes
    (col_lanes) lanes when nonzero."""
    import torch
    dev = A.val.device
    if nnz_half is None:
        nnz_half = fold_size(A, p)
    m, n = A.M // 2, A.N // 2
    S = System(m, n, nnz_half, 2, wdtype,
               torch.empty(m + 1, dtype=torch.int64, device=dev),
               stream_tensor(nnz_half, 1, torch.int32, dev),
               _value_tensor(nnz_half, 2, wdtype, dev),
               torch.empty(n + 1, dtype=torch.int64, device=dev),
               stream_tensor(nnz_half, 1, torch.int32, dev),
               _value_tensor(nnz_half, 2, wdtype, dev),
               torch.empty(2 * m, dtype=torch.float32, device=dev),
               torch.empty(m, dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.float32, device=dev), row_lanes, col_lanes)
    fold_into(A, p, S)
    return S


_fold_ws = {}


def fold_workspace(A: DeviceMatrix):
    """Device scratch for ss_fold_size / ss_fold, cached per (device, M, N)."""
    import torch
    key = (str(A.val.device), A.M, A.N)
    if key not in _fold_ws:
        nb = C.c_size_t()
        _check(lib().ss_fold_workspace_bytes(A.M, A.N, C.byref(nb)))
        _fold_ws[key] = torch.empty(nb.value, dtype=torch.uint8, device=A.val.device)
    return _fold_ws[key]


def fold_into(A: DeviceMatrix, p, S: System) -> None:
    """ss_fold into an existing system's arrays (same sizes)."""
    mc, sc = A.c(), S.c()
    ws = fold_workspace(A)
    _check(lib().ss_fold(C.byref(mc), _ptr(p), C.byref(sc), _ptr(ws), ws.numel(),
                         _stream(A.val.device)))


def fold_noalloc_into(A: DeviceMatrix, p, S: System) -> None:
    """ss_fold_noalloc into an existing system's arrays (no workspace)."""
    mc, sc = A.c(), S.c()
    _check(lib().ss_fold_noalloc(C.byref(mc), _ptr(p), C.byref(sc), _stream(A.val.device)))


class FoldBatch:
    """ss_fold_batch over fixed lists of matrices, right-hand sides and
    systems (the descriptor arrays are built once)."""

    def __init__(self, As, ps, systems):
        import torch
        assert len(As) == len(ps) == len(systems) > 0
        self.count = len(As)
        self._keep = (list(As), list(ps), list(systems))
        self._A = (MatrixDevC * self.count)(*[A.c() for A in As])
        self._p = (C.c_void_p * self.count)(*[_ptr(p) for p in ps])
        self._S = (SystemC * self.count)(*[S.c() for S in systems])
        nb = C.c_size_t()
        _check(lib().ss_fold_batch_workspace_bytes(self._A, self.count, C.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device=ps[0].device)

    def __call__(self):
        _check(lib().ss_fold_batch(self._A, self._p, self._S, self.count, _ptr(self.ws), self.ws_bytes,
                                   _stream(self.ws.device)))

    def sizes(self):
        """ss_fold_size_batch on the same matrices: validates every matrix
        (and p) and returns the shared-pattern sizes (synchronises once)."""
        out = (C.c_int64 * self.count)()
        _check(lib().ss_fold_size_batch(self._A, self._p, self.count, _ptr(self.ws), self.ws_bytes, out,
                                        _stream(self.ws.device)))
        return list(out)


class FoldCheckBatch:
    """ss_fold_size_batch over fixed lists of matrices and right-hand sides
    (entries of ps may be None): call it to validate all of them and get
    the shared-pattern sizes."""

    def __init__(self, As, ps=None):
        import torch
        self.count = len(As)
        assert self.count > 0
        ps = list(ps) if ps is not None else [None] * self.count
        self._keep = (list(As), ps)
        self._A = (MatrixDevC * self.count)(*[A.c() for A in As])
        self._p = (C.c_void_p * self.count)(*[_ptr(p) for p in ps])
        nb = C.c_size_t()
        _check(lib().ss_fold_batch_workspace_bytes(self._A, self.count, C.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device=As[0].val.device)

    def __call__(self):
        out = (C.c_int64 * self.count)()
        _check(lib().ss_fold_size_batch(self._A, self._p, self.count, _ptr(self.ws), self.ws_bytes, out,
                                        _stream(self.ws.device)))
        return list(out)


def unsplit(A: DeviceMatrix, p, wdtype: str = "f32") -> System:
    """ss_unsplit: A itself as a single system (the unsplit baseline)."""
    import torch
    dev = A.val.device
    if wdtype == "f32":
        val, val_t = A.val, A.val_t
    else:
        val, val_t = _value_tensor(A.nnz, 1, wdtype, dev), _value_tensor(A.nnz, 1, wdtype, dev)
    S = System(A.M, A.N, A.nnz, 1, wdtype, A.row_ptr, A.col_idx, val, A.col_ptr, A.row_idx,
               val_t, torch.empty(A.M, dtype=torch.float32, device=dev),
               torch.empty(A.M, dtype=torch.float32, device=dev),
               torch.empty(A.N, dtype=torch.float32, device=dev))
    mc, sc = A.c(), S.c()
    _check(lib().ss_unsplit(C.byref(mc), _ptr(p), C.byref(sc), _stream(dev)))
    return S


@dataclasses.dataclass
class SartOptions:
    lam: float = 0.5
    max_iter: int = 20
    tol: float = 0.0
    check_every: int = 50
    use_graph: bool = True
    rows_per_wave: int = 0
    cols_per_wave: int = 0
    xcd_remap: int = 0
    zero_start: bool = False
    unroll: int = 0
    persistent: int = 0
    chunked: int = 0
    nonneg: bool = False
    staged: int = 0
    band_width: int = 0
    tile_cols: int = 0
    tile_entries: int = 0
    residual_every: int = 0

    def c(self) -> SartOptsC:
        return SartOptsC(self.lam, self.max_iter, self.tol, self.check_every,
                         int(self.use_graph), self.rows_per_wave, self.cols_per_wave,
                         self.xcd_remap, int(self.zero_start), self.unroll, self.persistent, self.chunked,
                         int(self.nonneg), self.staged, self.band_width, self.tile_cols, self.tile_entries,
                         self.residual_every)


class Solver:
    """Marshals ss_sart_solve / ss_sart_time_kernels / ss_sart_autotune for a
    fixed list of systems, owning the workspace."""

    def __init__(self, systems, opts: SartOptions | None = None):
        import torch
        self.systems = list(systems)
        self.opts = opts or SartOptions()
        self._arr = (SystemC * len(self.systems))(*[s.c() for s in self.systems])
        self.ws_bytes = 0
        self.ws = None
        self._reserve(self.opts)

    def _bytes(self, opts) -> int:
        nb = C.c_size_t()
        oc = opts.c()
        _check(lib().ss_sart_workspace_bytes(self._arr, len(self.systems), C.byref(oc), C.byref(nb)))
        return nb.value

    def _reserve(self, opts):
        """Grows the workspace to what ``opts`` needs (the interleaved stream
        form keeps copies of the streams there)."""
        import torch
        need = self._bytes(opts)
        if need > self.ws_bytes:
            self.ws = None
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.systems[0].p.device)
            self.ws_bytes = need

    def _imgs(self, f):
        assert len(f) == len(self.systems)
        for s, t in zip(self.systems, f):
            assert t.is_contiguous() and t.numel() == s.n * s.nvals and t.dtype.itemsize == 4
        return (C.c_void_p * len(f))(*[t.data_ptr() for t in f])

    def solve(self, f, res_hist=None, want_iters: bool = True):
        """Runs SART in place on the images ``f``; returns (status, iters)."""
        o = self.opts
        oc = o.c()
        if res_hist is not None:
            for s, h in zip(self.systems, res_hist):
                assert h.numel() >= o.max_iter + 1 and h.dtype.itemsize == 8
            rh = (C.c_void_p * len(res_hist))(*[h.data_ptr() for h in res_hist])
        else:
            rh = None
        it = (C.c_int32 * len(self.systems))() if want_iters else None
        self._reserve(o)
        st = lib().ss_sart_solve(self._arr, len(self.systems), self._imgs(f), rh, C.byref(oc),
                                 it, _ptr(self.ws), self.ws_bytes, _stream(self.ws.device))
        _check(st, allow_warning=True)
        return st, (list(it) if it is not None else None)

    def time_kernels(self, f, reps: int = 20):
        fp, bp = C.c_double(), C.c_double()
        self._reserve(self.opts)
        oc = self.opts.c()
        _check(lib().ss_sart_time_kernels(self._arr, len(self.systems), self._imgs(f), C.byref(oc),
                                          reps, C.byref(fp), C.byref(bp), _ptr(self.ws),
                                          self.ws_bytes, _stream(self.ws.device)))
        return fp.value, bp.value

    def time_phases(self, f, reps: int = 20):
        """ss_sart_time_phases: mean ms of (forward kernel, staged residual
        kernel or 0, back projection)."""
        ms = (C.c_double * 3)()
        self._reserve(self.opts)
        oc = self.opts.c()
        _check(lib().ss_sart_time_phases(self._arr, len(self.systems), self._imgs(f), C.byref(oc), reps, ms,
                                         _ptr(self.ws), self.ws_bytes, _stream(self.ws.device)))
        return tuple(ms)

    def staged_info(self, f):
        """ss_sart_staged_info: [forward segments, forward work tiles,
        back-projection tiles, of those staged, rows they stage]."""
        info = (C.c_int64 * 5)()
        self._reserve(self.opts)
        oc = self.opts.c()
        _check(lib().ss_sart_staged_info(self._arr, len(self.systems), self._imgs(f), C.byref(oc), info,
                                         _ptr(self.ws), self.ws_bytes, _stream(self.ws.device)))
        return list(info)

    def autotune(self, f):
        # room for the interleaved candidates, where the systems allow them
        try:
            self._reserve(dataclasses.replace(self.opts, chunked=12))
        except SSError:
            self._reserve(self.opts)
        oc = self.opts.c()
        _check(lib().ss_sart_autotune(self._arr, len(self.systems), self._imgs(f), C.byref(oc),
                                      _ptr(self.ws), self.ws_bytes, _stream(self.ws.device)))
        self.opts.rows_per_wave = oc.rows_per_wave
        self.opts.cols_per_wave = oc.cols_per_wave
        self.opts.xcd_remap = oc.xcd_remap
        self.opts.unroll = oc.unroll
        self.opts.persistent = oc.persistent
        self.opts.chunked = oc.chunked
        return self.opts


class Subsets:
    """ss_subsets of one folded FP32 pair: S blocks of m/S folded rows (for
    the symmetric scan, S = K/2 mirror-paired views)."""

    def __init__(self, S: System, n_subsets: int):
        import torch
        self.S = int(n_subsets)
        dev = S.p.device
        self.col_sub = torch.empty(S.n * (self.S + 1), dtype=torch.int32, device=dev)
        self.inv_col_sub = torch.empty(self.S * S.n, dtype=torch.float32, device=dev)
        self.col_ptr_os = torch.empty(self.S * S.n + 1, dtype=torch.int64, device=dev)
        self.row_idx_os = stream_tensor(S.nnz, 1, torch.int32, dev)
        self.val_t_os = stream_tensor(S.nnz, 2, torch.float32, dev)
        sc, bc = S.c(), self.c()
        _check(lib().ss_subsets_build(C.byref(sc), C.byref(bc), _stream(dev)))

    def c(self) -> SubsetsC:
        return SubsetsC(self.S, _ptr(self.col_sub), _ptr(self.inv_col_sub), _ptr(self.col_ptr_os),
                        _ptr(self.row_idx_os), _ptr(self.val_t_os))


class OsSolver:
    """Marshals ss_ossart_solve for fixed lists of systems and subsets,
    owning the workspace.  Options as SartOptions, max_iter counting passes."""

    def __init__(self, systems, subsets, opts: SartOptions | None = None):
        import torch
        self.systems = list(systems)
        self.subsets = list(subsets)
        assert len(self.systems) == len(self.subsets)
        self.opts = opts or SartOptions()
        self._arr = (SystemC * len(self.systems))(*[s.c() for s in self.systems])
        self._sub = (SubsetsC * len(self.subsets))(*[b.c() for b in self.subsets])
        nb = C.c_size_t()
        oc = self.opts.c()
        _check(lib().ss_ossart_workspace_bytes(self._arr, self._sub, len(self.systems), C.byref(oc), C.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.systems[0].p.device)

    def solve(self, f, res_hist=None, want_passes: bool = True):
        """Runs ordered-subset SART in place on ``f``; returns (status, passes)."""
        o = self.opts
        oc = o.c()
        assert len(f) == len(self.systems)
        for s, t in zip(self.systems, f):
            assert t.is_contiguous() and t.numel() == 2 * s.n and t.dtype.itemsize == 4
        imgs = (C.c_void_p * len(f))(*[t.data_ptr() for t in f])
        if res_hist is not None:
            for h in res_hist:
                assert h.numel() >= o.max_iter + 1 and h.dtype.itemsize == 8
            rh = (C.c_void_p * len(res_hist))(*[h.data_ptr() for h in res_hist])
        else:
            rh = None
        it = (C.c_int32 * len(self.systems))() if want_passes else None
        st = lib().ss_ossart_solve(self._arr, self._sub, len(self.systems), imgs, rh, C.byref(oc), it,
                                   _ptr(self.ws), self.ws_bytes, _stream(self.ws.device))
        _check(st, allow_warning=True)
        return st, (list(it) if it is not None else None)


def normal_solve(S: System, out=None):
    """ss_normal_solve: the normal-equation solution (FP64), recombined by
    eq. (5) for a folded pair."""
    import torch
    sc = S.c()
    nb = C.c_size_t()
    _check(lib().ss_normal_workspace_bytes(C.byref(sc), C.byref(nb)))
    dev = S.p.device
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty(S.n * S.nvals, dtype=torch.float64, device=dev)
    _check(lib().ss_normal_solve(C.byref(sc), _ptr(out), _ptr(ws), nb.value, _stream(dev)))
    return out


def recombine(f12, out=None):
    """ss_recombine: Theorem 1, eq. (5)."""
    import torch
    n = f12.shape[0]
    if out is None:
        out = torch.empty(2 * n, dtype=torch.float32, device=f12.device)
    _check(lib().ss_recombine(_ptr(f12), n, _ptr(out), _stream(f12.device)))
    return out


class RecombineBatch:
    """ss_recombine_batch over fixed lists of half-image pairs and outputs."""

    def __init__(self, f12s, outs):
        assert len(f12s) == len(outs) > 0
        self.count = len(f12s)
        self._keep = (list(f12s), list(outs))
        self._f12 = (C.c_void_p * self.count)(*[_ptr(f) for f in f12s])
        self._n = (C.c_int64 * self.count)(*[f.shape[0] for f in f12s])
        self._out = (C.c_void_p * self.count)(*[_ptr(o) for o in outs])
        self._dev = f12s[0].device

    def __call__(self):
        _check(lib().ss_recombine_batch(self._f12, self._n, self._out, self.count, _stream(self._dev)))


def image_fold(f, out=None):
    """ss_image_fold: the inverse of eq. (5)."""
    import torch
    N = f.shape[0]
    if out is None:
        out = torch.empty((N // 2, 2), dtype=torch.float32, device=f.device)
    _check(lib().ss_image_fold(_ptr(f), N, _ptr(out), _stream(f.device)))
    return out


def project(A: DeviceMatrix, f, out=None):
    """ss_project: q = A f."""
    import torch
    if out is None:
        out = torch.empty(A.M, dtype=torch.float32, device=f.device)
    mc = A.c()
    _check(lib().ss_project(C.byref(mc), _ptr(f), _ptr(out), _stream(f.device)))
    return out


def fold_rhs(p, out=None):
    """ss_fold_rhs: (p1, p2) interleaved, for systems sharing a folded matrix."""
    import torch
    M = p.shape[0]
    if out is None:
        out = torch.empty(M, dtype=torch.float32, device=p.device)
    _check(lib().ss_fold_rhs(_ptr(p), M, _ptr(out), _stream(p.device)))
    return out


# -------------------------------------------------- learned initialiser ops
def nn_prep_weights(w32, O, C, w_fwd, w_bwd):
    _check(lib().ss_nn_prep_weights(_ptr(w32), O, C, _ptr(w_fwd), _ptr(w_bwd), _stream(w32.device)))


def nn_conv3x3(x, N, H, W, C, w, bias, O, relu, y, y_f32=False):
    _check(lib().ss_nn_conv3x3(_ptr(x), N, H, W, C, _ptr(w), _ptr(bias), O, int(relu), _ptr(y),
                               int(y_f32), _stream(x.device)))


def nn_wgrad_workspace_bytes(N, H, W, Cin, O) -> int:
    nb = C.c_size_t()
    _check(lib().ss_nn_wgrad_workspace_bytes(N, H, W, Cin, O, C.byref(nb)))
    return nb.value


def nn_mse_workspace_bytes(n) -> int:
    nb = C.c_size_t()
    _check(lib().ss_nn_mse_workspace_bytes(n, C.byref(nb)))
    return nb.value


def _scratch(nbytes, device, ws=None):
    """A caller-given workspace, or a fresh one of nbytes."""
    import torch
    if ws is not None:
        assert ws.numel() * ws.element_size() >= nbytes
        return ws
    return torch.empty(max(1, nbytes), dtype=torch.uint8, device=device)


def nn_conv3x3_wgrad(x, gy, N, H, W, C, O, gw, gb, ws=None):
    need = nn_wgrad_workspace_bytes(N, H, W, C, O)
    w = _scratch(need, x.device, ws)
    _check(lib().ss_nn_conv3x3_wgrad(_ptr(x), _ptr(gy), N, H, W, C, O, _ptr(gw), _ptr(gb), _ptr(w),
                                     w.numel() * w.element_size(), _stream(x.device)))


def nn_relu_mask(g, y, out):
    _check(lib().ss_nn_relu_mask(_ptr(g), _ptr(y), g.numel(), _ptr(out), _stream(g.device)))


def nn_pool2(x, N, H, W, C, y):
    _check(lib().ss_nn_pool2(_ptr(x), N, H, W, C, _ptr(y), _stream(x.device)))


def nn_pool2_grad(gy, N, H, W, C, gx, accumulate=False):
    _check(lib().ss_nn_pool2_grad(_ptr(gy), N, H, W, C, _ptr(gx), int(accumulate), _stream(gy.device)))


def nn_to_slice(x, N, Hy, Wy, C, up, y, Ctot, coff):
    _check(lib().ss_nn_to_slice(_ptr(x), N, Hy, Wy, C, int(up), _ptr(y), Ctot, coff, _stream(x.device)))


def nn_from_slice(gy, N, Hx, Wx, C, up, Ctot, coff, gx, accumulate=False):
    _check(lib().ss_nn_from_slice(_ptr(gy), N, Hx, Wx, C, int(up), Ctot, coff, _ptr(gx),
                                  int(accumulate), _stream(gy.device)))


def nn_residual_mse(r, x, target, out, g=None, loss=None, ws=None):
    w = _scratch(nn_mse_workspace_bytes(r.numel()), r.device, ws) if loss is not None else None
    _check(lib().ss_nn_residual_mse(_ptr(r), _ptr(x), _ptr(target), r.numel(), _ptr(out), _ptr(g),
                                    _ptr(loss), _ptr(w), w.numel() * w.element_size() if w is not None else 0,
                                    _stream(r.device)))


def nn_to_bf16(x, y):
    _check(lib().ss_nn_to_bf16(_ptr(x), x.numel(), _ptr(y), _stream(x.device)))


def nn_adam(w, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    _check(lib().ss_nn_adam(_ptr(w), _ptr(g), _ptr(m), _ptr(v), w.numel(), lr, b1, b2, eps, step,
                            _stream(w.device)))


def nn_snake_image(src, nimg, nx, nz, to_image, dst32=None, dst16=None):
    _check(lib().ss_nn_snake_image(_ptr(src), nimg, nx, nz, int(to_image), _ptr(dst32), _ptr(dst16),
                                   _stream(src.device)))
