"""Python binding of libsp2.so: SP2 density-matrix purification on one MI355X.

Argument marshalling only.  Every step of the solve (bounds, initial iterate,
squarings, steering, final copy) runs in the HIP kernels of libsp2.so; torch
is used to own device memory and to name the stream.  There is no CPU
fallback: importing this package fails if the library is not built.

Entry points mirror include/sp2.h:
    sp2_version(), sp2_status_str(code), sp2_workspace_size(n, dtype, compute),
    sp2_density(H, n_occ, ...), sp2_history(workspace, count)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsp2.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
        "(hipcc --offload-arch=gfx950) first")

_lib = ctypes.CDLL(LIB_PATH)

# status codes (include/sp2.h)
OK, NOT_CONVERGED, STAGNATED, FALLBACK = 0, 1, 2, 3
E_INVALID, E_DEGENERATE, E_WORKSPACE, E_HIP, E_UNSUPPORTED = -1, -2, -3, -4, -5
MAX_ITER = 128
WORKSPACE_ALIGN = 256

DTYPES = {"f64": 0, "f32": 1}
COMPUTES = {"f64": 0, "f32": 1, "f16x2": 2, "bf16x3": 3, "bf16x2": 4, "fp8": 5}


class sp2_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("fp64_prefix_iters", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("trace", ctypes.c_double), ("trace_error", ctypes.c_double),
                ("idempotency", ctypes.c_double), ("emin", ctypes.c_double),
                ("emax", ctypes.c_double), ("branch_mask", ctypes.c_uint64 * 2)]


_vp = ctypes.c_void_p
_lib.sp2_version.restype = ctypes.c_int
_lib.sp2_status_str.restype = ctypes.c_char_p
_lib.sp2_status_str.argtypes = [ctypes.c_int]
_lib.sp2_workspace_size.restype = ctypes.c_size_t
_lib.sp2_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
_lib.sp2_density.restype = ctypes.c_int
_lib.sp2_density.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                             ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp,
                             ctypes.c_size_t, _vp, ctypes.POINTER(sp2_info)]
_lib.sp2_history.restype = ctypes.c_int
_lib.sp2_history.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), _vp]
_lib.sp2_profile_enable.restype = ctypes.c_int
_lib.sp2_profile_enable.argtypes = [ctypes.c_int]
_lib.sp2_profile_read.restype = ctypes.c_int
_lib.sp2_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
_lib.sp2_profile_read_split.restype = ctypes.c_int
_lib.sp2_profile_read_split.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]


@dataclass
class Info:
    status: int
    iterations: int
    fp64_prefix_iters: int
    refine_steps: int
    trace: float
    trace_error: float
    idempotency: float
    emin: float
    emax: float
    branch_mask: tuple

    def branches(self):
        m = self.branch_mask[0] | (self.branch_mask[1] << 64)
        return [(m >> k) & 1 for k in range(self.iterations)]

    @property
    def status_str(self):
        return sp2_status_str(self.status)


def _info(c: sp2_info) -> Info:
    return Info(int(c.status), int(c.iterations), int(c.fp64_prefix_iters), int(c.refine_steps),
                float(c.trace), float(c.trace_error), float(c.idempotency), float(c.emin),
                float(c.emax), (int(c.branch_mask[0]), int(c.branch_mask[1])))


def sp2_version() -> int:
    return int(_lib.sp2_version())


def sp2_status_str(code: int) -> str:
    return _lib.sp2_status_str(int(code)).decode()


def _dtype_code(t) -> int:
    import torch
    if t == torch.float64:
        return DTYPES["f64"]
    if t == torch.float32:
        return DTYPES["f32"]
    raise TypeError(f"H must be float64 or float32, got {t}")


def sp2_workspace_size(n: int, dtype: str = "f64", compute: str = "f64") -> int:
    return int(_lib.sp2_workspace_size(int(n), DTYPES[dtype], COMPUTES[compute]))


def alloc_workspace(n: int, dtype: str = "f64", compute: str = "f64", device="cuda"):
    """A torch uint8 device buffer sized and aligned for sp2_density."""
    import torch
    nbytes = sp2_workspace_size(n, dtype, compute)
    if nbytes == 0:
        raise ValueError("invalid workspace request")
    ws = torch.empty(nbytes + WORKSPACE_ALIGN, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % WORKSPACE_ALIGN
    return ws[off:off + nbytes]


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def sp2_density(H, n_occ: int, tol: float = 1e-10, max_iter: int = 100, compute: str = "f64",
                fp64_prefix_iters: int = -1, D=None, workspace=None, stream=None, n: int = None,
                check: bool = False):
    """SP2 density matrix of the symmetric device matrix H (torch, float64/float32).

    H may be a row-major view with leading dimension H.stride(0).  Returns
    (D, Info).  D has H's dtype and shape (n, n); pass D to reuse a buffer.
    With check=True a negative status raises RuntimeError.
    """
    import torch
    if H.dim() != 2 or H.stride(1) != 1:
        raise ValueError("H must be a 2-D row-major device tensor")
    if n is None:
        n = H.shape[0]
    ld = H.stride(0)
    dt = _dtype_code(H.dtype)
    if D is None:
        D = torch.empty((n, ld), dtype=H.dtype, device=H.device)[:, :n]
    if D.dtype != H.dtype or D.dim() != 2 or D.stride(1) != 1 or D.stride(0) != ld:
        raise ValueError("D must have H's dtype and leading dimension, row-major")
    if workspace is None:
        workspace = alloc_workspace(n, "f64" if dt == 0 else "f32", compute, device=H.device)
    elif workspace.numel() < sp2_workspace_size(n, "f64" if dt == 0 else "f32", compute):
        raise ValueError("workspace too small for this n / compute mode")
    info = sp2_info()
    st = _lib.sp2_density(_vp(H.data_ptr()), _vp(D.data_ptr()), int(n), int(ld), int(n_occ),
                          float(tol), int(max_iter), dt, COMPUTES[compute], int(fp64_prefix_iters),
                          _vp(workspace.data_ptr()), int(workspace.numel()), _stream_handle(stream),
                          ctypes.byref(info))
    out = _info(info)
    if check and st < 0:
        raise RuntimeError(f"sp2_density failed: {sp2_status_str(st)} ({st})")
    return D, out


def sp2_history(workspace, count: int = MAX_ITER, stream=None):
    """(tr_hist, e_hist) of the last sp2_density call on this workspace."""
    import numpy as np
    tr = (ctypes.c_double * count)()
    e = (ctypes.c_double * count)()
    m = _lib.sp2_history(_vp(workspace.data_ptr()), int(count), tr, e, _stream_handle(stream))
    if m < 0:
        raise RuntimeError(f"sp2_history failed: {sp2_status_str(m)}")
    return np.array(tr[:m]), np.array(e[:m])


def sp2_profile_enable(on: bool = True) -> None:
    st = _lib.sp2_profile_enable(1 if on else 0)
    if st != OK:
        raise RuntimeError(f"sp2_profile_enable failed: {sp2_status_str(st)}")


def sp2_profile_read():
    """(summed squaring-kernel ms, number of squarings) of the last timed call."""
    ms = ctypes.c_double()
    steps = ctypes.c_int()
    st = _lib.sp2_profile_read(ctypes.byref(ms), ctypes.byref(steps))
    if st != OK:
        raise RuntimeError(f"sp2_profile_read failed: {sp2_status_str(st)}")
    return ms.value, steps.value


def sp2_profile_read_split():
    """((FP64 step ms, FP64 steps), (split step ms, split steps)) of the last timed call."""
    a, b = ctypes.c_double(), ctypes.c_double()
    na, nb = ctypes.c_int(), ctypes.c_int()
    st = _lib.sp2_profile_read_split(ctypes.byref(a), ctypes.byref(na), ctypes.byref(b), ctypes.byref(nb))
    if st != OK:
        raise RuntimeError(f"sp2_profile_read_split failed: {sp2_status_str(st)}")
    return (a.value, na.value), (b.value, nb.value)


def exported_symbols():
    """Names of the C entry points this binding wraps."""
    return ["sp2_version", "sp2_status_str", "sp2_workspace_size", "sp2_density", "sp2_history",
            "sp2_profile_enable", "sp2_profile_read", "sp2_profile_read_split"]
