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
_lib.sp2_density_noalloc.restype = ctypes.c_int
_lib.sp2_density_noalloc.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, _vp, ctypes.POINTER(sp2_info)]
NOALLOC_MAX_BYTES = 64 << 20
_lib.sp2_plan_create.restype = ctypes.c_int
_lib.sp2_plan_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int, ctypes.c_char_p]
_lib.sp2_plan_run.restype = ctypes.c_int
_lib.sp2_plan_run.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, ctypes.POINTER(sp2_info)]
_lib.sp2_plan_config.restype = ctypes.c_char_p
_lib.sp2_plan_config.argtypes = [_vp]
_lib.sp2_plan_destroy.restype = ctypes.c_int
_lib.sp2_plan_destroy.argtypes = [_vp]
PLAN_MAX_N = 2048
_lib.sp2_cheb_workspace_size.restype = ctypes.c_size_t
_lib.sp2_cheb_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int]
_lib.sp2_cheb_density.restype = ctypes.c_int
_lib.sp2_sparse_workspace_size.restype = ctypes.c_size_t
_lib.sp2_sparse_workspace_size.argtypes = [ctypes.c_int]
_lib.sp2_sparse_stats.restype = ctypes.c_int
_lib.sp2_sparse_stats.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.sp2_density_sparse.restype = ctypes.c_int
_lib.sp2_density_sparse.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_double, _vp, ctypes.c_size_t, _vp,
                                    ctypes.POINTER(sp2_info)]
_lib.sp2_graph_create.restype = ctypes.c_int
_lib.sp2_graph_create.argtypes = [ctypes.POINTER(_vp), _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int, _vp]
_lib.sp2_graph_parts.restype = ctypes.c_int
_lib.sp2_graph_parts.argtypes = [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.sp2_graph_nodes.restype = ctypes.c_int
_lib.sp2_graph_nodes.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
_lib.sp2_graph_density.restype = ctypes.c_int
_lib.sp2_graph_density.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _vp,
                                   ctypes.POINTER(sp2_info)]
_lib.sp2_graph_destroy.restype = ctypes.c_int
_lib.sp2_graph_destroy.argtypes = [_vp]
_lib.sp2_cheb_density.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t, _vp,
                                  ctypes.POINTER(sp2_info)]
_lib.sp2_learned_create.restype = ctypes.c_int
_lib.sp2_learned_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
_lib.sp2_learned_fit.restype = ctypes.c_int
_lib.sp2_learned_fit.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_uint64]
_lib.sp2_learned_coefficients.restype = ctypes.c_int
_lib.sp2_learned_coefficients.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_double)]
_lib.sp2_learned_save.restype = ctypes.c_int
_lib.sp2_learned_save.argtypes = [_vp, ctypes.c_char_p]
_lib.sp2_learned_load.restype = ctypes.c_int
_lib.sp2_learned_load.argtypes = [ctypes.POINTER(_vp), ctypes.c_char_p]
_lib.sp2_learned_density.restype = ctypes.c_int
_lib.sp2_learned_density.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                     ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, _vp, ctypes.POINTER(sp2_info)]
_lib.sp2_learned_destroy.restype = ctypes.c_int
_lib.sp2_learned_destroy.argtypes = [_vp]
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


def sp2_density_noalloc(H, n_occ: int, D, tol: float = 1e-10, max_iter: int = 100,
                        compute: str = "f64", fp64_prefix_iters: int = -1, stream=None,
                        n: int = None):
    """sp2_density with the library's fixed per-GPU workspace (no allocation in
    the call; sp2_workspace_size(n, ...) must be <= NOALLOC_MAX_BYTES).  D is a
    preallocated device tensor with H's dtype and leading dimension.
    Returns (D, Info)."""
    if H.dim() != 2 or H.stride(1) != 1:
        raise ValueError("H must be a 2-D row-major device tensor")
    if n is None:
        n = H.shape[0]
    ld = H.stride(0)
    if D.dtype != H.dtype or D.dim() != 2 or D.stride(1) != 1 or D.stride(0) != ld:
        raise ValueError("D must have H's dtype and leading dimension, row-major")
    info = sp2_info()
    _lib.sp2_density_noalloc(_vp(H.data_ptr()), _vp(D.data_ptr()), int(n), int(ld), int(n_occ),
                             float(tol), int(max_iter), _dtype_code(H.dtype), COMPUTES[compute],
                             int(fp64_prefix_iters), _stream_handle(stream), ctypes.byref(info))
    return D, _info(info)


def sp2_history(workspace, count: int = MAX_ITER, stream=None):
    """(tr_hist, e_hist) of the last sp2_density call on this workspace."""
    import numpy as np
    tr = (ctypes.c_double * count)()
    e = (ctypes.c_double * count)()
    m = _lib.sp2_history(_vp(workspace.data_ptr()), int(count), tr, e, _stream_handle(stream))
    if m < 0:
        raise RuntimeError(f"sp2_history failed: {sp2_status_str(m)}")
    return np.array(tr[:m]), np.array(e[:m])


def sp2_cheb_workspace_size(n: int, k: int) -> int:
    return int(_lib.sp2_cheb_workspace_size(int(n), int(k)))


def sp2_cheb_density(H, mu: float, beta: float, k: int, m: int, D=None, workspace=None, stream=None):
    """Chebyshev expansion of the Fermi operator (sp2_cheb_density): k m terms in
    Paterson-Stockmeyer form.  H: (n, n) device tensor, row-major (leading
    dimension H.stride(0)).  Returns (D, Info)."""
    import torch
    if H.dim() != 2 or H.stride(1) != 1:
        raise ValueError("H must be a 2-D row-major device tensor")
    n = H.shape[0]
    ld = H.stride(0)
    if D is None:
        D = torch.empty((n, ld), dtype=H.dtype, device=H.device)[:, :n]
    if D.dtype != H.dtype or D.stride(0) != ld or D.stride(1) != 1:
        raise ValueError("D must have H's dtype and leading dimension, row-major")
    nbytes = sp2_cheb_workspace_size(n, k)
    if nbytes == 0:
        raise ValueError("invalid size or k")
    if workspace is None:
        ws = torch.empty(nbytes + WORKSPACE_ALIGN, dtype=torch.uint8, device=H.device)
        off = (-ws.data_ptr()) % WORKSPACE_ALIGN
        workspace = ws[off:off + nbytes]
    info = sp2_info()
    _lib.sp2_cheb_density(_vp(H.data_ptr()), _vp(D.data_ptr()), int(n), int(ld), _dtype_code(H.dtype),
                          float(mu), float(beta), int(k), int(m), _vp(workspace.data_ptr()),
                          int(workspace.numel()), _stream_handle(stream), ctypes.byref(info))
    return D, _info(info)


def sp2_sparse_workspace_size(n: int) -> int:
    return int(_lib.sp2_sparse_workspace_size(int(n)))


def sp2_density_sparse(H, n_occ: int, tau: float, tol: float = 1e-10, max_iter: int = 100, D=None,
                       workspace=None, stream=None):
    """Thresholded SP2 with tile skipping (sp2_density_sparse).  Returns (D, Info)."""
    import torch
    if H.dim() != 2 or H.shape[0] != H.shape[1] or H.stride(1) != 1:
        raise ValueError("H must be a square row-major device tensor")
    n = H.shape[0]
    ld = H.stride(0)
    if D is None:
        D = torch.empty((n, ld), dtype=H.dtype, device=H.device)[:, :n]
    if D.dtype != H.dtype or D.stride(0) != ld or D.stride(1) != 1:
        raise ValueError("D must have H's dtype and leading dimension, row-major")
    nbytes = sp2_sparse_workspace_size(n)
    if nbytes == 0:
        raise ValueError("invalid size")
    if workspace is None:
        ws = torch.empty(nbytes + WORKSPACE_ALIGN, dtype=torch.uint8, device=H.device)
        off = (-ws.data_ptr()) % WORKSPACE_ALIGN
        workspace = ws[off:off + nbytes]
    info = sp2_info()
    _lib.sp2_density_sparse(_vp(H.data_ptr()), _vp(D.data_ptr()), int(n), int(ld), int(n_occ), float(tol),
                            int(max_iter), _dtype_code(H.dtype), float(tau), _vp(workspace.data_ptr()),
                            int(workspace.numel()), _stream_handle(stream), ctypes.byref(info))
    return D, _info(info)


def sp2_sparse_stats(workspace, stream=None):
    """(executed flops, computed (step, tile) pairs) of the last sparse solve on workspace."""
    f = ctypes.c_double()
    t = ctypes.c_double()
    st = _lib.sp2_sparse_stats(_vp(workspace.data_ptr()), _stream_handle(stream), ctypes.byref(f), ctypes.byref(t))
    if st != OK:
        raise RuntimeError(f"sp2_sparse_stats failed: {sp2_status_str(st)}")
    return f.value, t.value


class Graph:
    """A graph-partitioned solver (sp2_graph_create): core-halo parts of the
    thresholded graph of G, solved together at a chemical potential by
    density()."""

    def __init__(self, G, tau: float, parts: int, tol: float = 1e-10, max_iter: int = 100, stream=None):
        if G.dim() != 2 or G.shape[0] != G.shape[1] or G.stride(1) != 1:
            raise ValueError("G must be a square row-major device tensor")
        self.n = int(G.shape[0])
        self._h = _vp()
        st = _lib.sp2_graph_create(ctypes.byref(self._h), _vp(G.data_ptr()), self.n, int(G.stride(0)),
                                   _dtype_code(G.dtype), float(tau), int(parts), float(tol), int(max_iter),
                                   _stream_handle(stream))
        if st != OK:
            self._h = _vp()
            raise RuntimeError(f"sp2_graph_create failed: {sp2_status_str(st)} ({st})")
        self.parts = int(parts)

    def sizes(self):
        """(nodes per part, core nodes per part) as lists."""
        a = (ctypes.c_int * self.parts)()
        c = (ctypes.c_int * self.parts)()
        _lib.sp2_graph_parts(self._h, a, c)
        return list(a), list(c)

    def nodes(self, part: int):
        """Ascending node list of one part."""
        s = _lib.sp2_graph_nodes(self._h, int(part), None, 0)
        if s < 0:
            raise ValueError("no such part")
        buf = (ctypes.c_int * s)()
        st = _lib.sp2_graph_nodes(self._h, int(part), buf, s)
        if st != s:
            raise RuntimeError(f"sp2_graph_nodes failed: {st}")
        return list(buf)

    def density(self, H, mu: float, D=None, stream=None):
        """D of H at chemical potential mu; returns (D, [Info per part])."""
        import torch
        if not self._h:
            raise RuntimeError("graph is closed")
        if H.dim() != 2 or tuple(H.shape) != (self.n, self.n) or H.stride(1) != 1:
            raise ValueError("H must be an (n, n) row-major device tensor")
        ld = H.stride(0)
        if D is None:
            D = torch.empty((self.n, ld), dtype=H.dtype, device=H.device)[:, :self.n]
        if D.dtype != H.dtype or D.stride(0) != ld or D.stride(1) != 1:
            raise ValueError("D must have H's dtype and leading dimension, row-major")
        infos = (sp2_info * self.parts)()
        st = _lib.sp2_graph_density(self._h, _vp(H.data_ptr()), _vp(D.data_ptr()), int(ld),
                                    _dtype_code(H.dtype), float(mu), _stream_handle(stream), infos)
        self.last_status = int(st)
        if st in (E_HIP, E_INVALID):
            raise RuntimeError(f"sp2_graph_density failed: {sp2_status_str(st)} ({st})")
        return D, [_info(i) for i in infos]

    def close(self):
        if self._h:
            _lib.sp2_graph_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A batched plan (sp2_plan_create): `sizes[b]` x `sizes[b]` problems with
    occupations n_occ[b], solved together by run() in one graph replay."""

    def __init__(self, sizes, n_occ, dtype: str = "f64", compute: str = "f64", tol: float = 1e-10,
                 max_iter: int = 100, autotune_cache: str = None):
        self.sizes = [int(v) for v in sizes]
        self.n_occ = [int(v) for v in n_occ]
        if len(self.sizes) != len(self.n_occ) or not self.sizes:
            raise ValueError("sizes and n_occ must be non-empty and of equal length")
        self.dtype = dtype
        self.batch = len(self.sizes)
        self._h = _vp()
        ns = (ctypes.c_int * self.batch)(*self.sizes)
        no = (ctypes.c_int * self.batch)(*self.n_occ)
        st = _lib.sp2_plan_create(ctypes.byref(self._h), self.batch, ns, no, DTYPES[dtype],
                                  COMPUTES[compute], float(tol), int(max_iter),
                                  autotune_cache.encode() if autotune_cache else None)
        if st != OK:
            self._h = _vp()
            raise RuntimeError(f"sp2_plan_create failed: {sp2_status_str(st)} ({st})")
        self.last_status = None

    @property
    def config(self) -> str:
        return _lib.sp2_plan_config(self._h).decode()

    def run(self, Hs, Ds=None, stream=None):
        """Solve every problem: Hs[b] contiguous (n_b, n_b) device tensors of the
        plan's dtype.  Returns (Ds, [Info]); pass Ds to reuse buffers."""
        import torch
        if not self._h:
            raise RuntimeError("plan is closed")
        want = torch.float64 if self.dtype == "f64" else torch.float32
        if len(Hs) != self.batch:
            raise ValueError("one H per problem of the plan")
        for H, n in zip(Hs, self.sizes):
            if H.dtype != want or tuple(H.shape) != (n, n) or not H.is_contiguous():
                raise ValueError("H[b] must be a contiguous (n_b, n_b) tensor of the plan's dtype")
        if Ds is None:
            Ds = [torch.empty_like(H) for H in Hs]
        for D, H in zip(Ds, Hs):
            if D.dtype != want or D.shape != H.shape or not D.is_contiguous():
                raise ValueError("D[b] must match H[b]")
        hp = (_vp * self.batch)(*[H.data_ptr() for H in Hs])
        dp = (_vp * self.batch)(*[D.data_ptr() for D in Ds])
        infos = (sp2_info * self.batch)()
        st = _lib.sp2_plan_run(self._h, hp, dp, _stream_handle(stream), infos)
        self.last_status = int(st)
        if st == E_HIP or st == E_INVALID and not any(int(i.status) == E_INVALID for i in infos):
            raise RuntimeError(f"sp2_plan_run failed: {sp2_status_str(st)} ({st})")
        return Ds, [_info(i) for i in infos]

    def close(self):
        if self._h:
            _lib.sp2_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Learned:
    """A learned recursive expansion (sp2_learned_*): trained quadratic layers
    with trace steering, SP2 check step and plain-SP2 fallback."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def from_coefficients(cls, coef):
        import numpy as np
        c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64).reshape(-1, 3))
        h = _vp()
        st = _lib.sp2_learned_create(ctypes.byref(h), c.shape[0],
                                     c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if st != OK:
            raise RuntimeError(f"sp2_learned_create failed: {sp2_status_str(st)}")
        return cls(h)

    @classmethod
    def fit(cls, n_layers, spectra, n_occ, gersh, epochs, seed=0):
        """spectra: list of ascending eigenvalue arrays; gersh: (samples, 2)."""
        import numpy as np
        lam = np.ascontiguousarray(np.concatenate([np.asarray(w, dtype=np.float64) for w in spectra]))
        ns = np.ascontiguousarray([len(w) for w in spectra], dtype=np.int32)
        no = np.ascontiguousarray(n_occ, dtype=np.int32)
        g = np.ascontiguousarray(np.asarray(gersh, dtype=np.float64).reshape(-1, 2))
        h = _vp()
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        st = _lib.sp2_learned_fit(ctypes.byref(h), int(n_layers), lam.ctypes.data_as(dp), ns.ctypes.data_as(ip),
                                  no.ctypes.data_as(ip), len(spectra), g.ctypes.data_as(dp), int(epochs),
                                  int(seed))
        if st != OK:
            raise RuntimeError(f"sp2_learned_fit failed: {sp2_status_str(st)}")
        return cls(h)

    @classmethod
    def load(cls, path):
        h = _vp()
        st = _lib.sp2_learned_load(ctypes.byref(h), str(path).encode())
        if st != OK:
            raise RuntimeError(f"sp2_learned_load failed: {sp2_status_str(st)}")
        return cls(h)

    def save(self, path):
        st = _lib.sp2_learned_save(self._h, str(path).encode())
        if st != OK:
            raise RuntimeError(f"sp2_learned_save failed: {sp2_status_str(st)}")

    def coefficients(self):
        """((layers, 3) array, loss of the last training epoch)."""
        import numpy as np
        L = _lib.sp2_learned_coefficients(self._h, None, 0, None)
        c = np.zeros(3 * max(L, 1))
        loss = ctypes.c_double()
        _lib.sp2_learned_coefficients(self._h, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 3 * L,
                                      ctypes.byref(loss))
        return c[:3 * L].reshape(L, 3), loss.value

    def density(self, Hs, n_occ, Ds=None, idem_fallback=1e-6, compute="f64", stream=None):
        """Batch of same-size (n, n) contiguous device matrices.  Returns (Ds, [Info])."""
        import torch
        n = Hs[0].shape[0]
        dt = _dtype_code(Hs[0].dtype)
        for H in Hs:
            if tuple(H.shape) != (n, n) or H.dtype != Hs[0].dtype or not H.is_contiguous():
                raise ValueError("all H must be contiguous (n, n) tensors of one dtype")
        if Ds is None:
            Ds = [torch.empty_like(H) for H in Hs]
        b = len(Hs)
        hp = (_vp * b)(*[H.data_ptr() for H in Hs])
        dp = (_vp * b)(*[D.data_ptr() for D in Ds])
        no = (ctypes.c_int * b)(*[int(v) for v in n_occ])
        infos = (sp2_info * b)()
        st = _lib.sp2_learned_density(self._h, b, n, hp, dp, no, dt, COMPUTES[compute], float(idem_fallback),
                                      _stream_handle(stream), infos)
        if st == E_HIP or st == E_UNSUPPORTED:
            raise RuntimeError(f"sp2_learned_density failed: {sp2_status_str(st)}")
        return Ds, [_info(i) for i in infos]

    def close(self):
        if self._h:
            _lib.sp2_learned_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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
    return ["sp2_version", "sp2_status_str", "sp2_workspace_size", "sp2_density",
            "sp2_density_noalloc", "sp2_history", "sp2_plan_create", "sp2_plan_run",
            "sp2_plan_config", "sp2_plan_destroy", "sp2_learned_create", "sp2_learned_fit",
            "sp2_learned_coefficients", "sp2_learned_save", "sp2_learned_load", "sp2_learned_density",
            "sp2_learned_destroy", "sp2_cheb_workspace_size", "sp2_cheb_density",
            "sp2_graph_create", "sp2_graph_parts", "sp2_graph_nodes", "sp2_graph_density",
            "sp2_graph_destroy", "sp2_sparse_workspace_size", "sp2_density_sparse", "sp2_sparse_stats",
            "sp2_profile_enable", "sp2_profile_read", "sp2_profile_read_split"]
