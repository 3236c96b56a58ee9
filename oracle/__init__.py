"""FP64 CPU oracle for SP2 density-matrix purification -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never does, and this package never
imports the product library: the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, FP64, no BLAS/LAPACK); this
module only builds it with gcc and marshals NumPy arrays through ctypes.
Each function's docstring names the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, STAGNATED, INVALID, DEGENERATE = 0, 1, 2, -1, -2


class DegenerateError(ValueError):
    """The zero-temperature density matrix is not unique (vanishing gap)."""


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("emin", ctypes.c_double), ("emax", ctypes.c_double),
                ("trace", ctypes.c_double), ("idempotency", ctypes.c_double),
                ("branch_mask", ctypes.c_uint64 * 2)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        i = ctypes.POINTER(ctypes.c_int)
        lib.oracle_gershgorin.argtypes = [d, ctypes.c_int, d, d]
        lib.oracle_sp2_init.argtypes = [d, ctypes.c_int, ctypes.c_double, ctypes.c_double, d]
        lib.oracle_sp2_init.restype = None
        lib.oracle_jacobi_eigh.argtypes = [d, ctypes.c_int, d, d, ctypes.c_int, i]
        lib.oracle_jacobi_dm.argtypes = [d, ctypes.c_int, ctypes.c_int, d, d, d, i]
        lib.oracle_sp2.argtypes = [d, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, d, ctypes.POINTER(_Result), d, d]
        lib.oracle_sp2_spectral.argtypes = [d, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int, d,
                                            ctypes.POINTER(_Result), d, d]
        lib.oracle_sp2_step_entries.argtypes = [d, ctypes.c_int, ctypes.c_int, i, i,
                                                ctypes.c_int, d]
        lib.oracle_sp2_step_entries.restype = None
        lib.oracle_cheb_coeffs.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, d]
        lib.oracle_cheb_density.argtypes = [d, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int, ctypes.c_int, d, d, d]
        lib.oracle_cheb_ps_split.argtypes = [d, ctypes.c_int, ctypes.c_int, d]
        u64 = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_learned_spectral.argtypes = [d, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                ctypes.c_double, d, ctypes.c_int, d, u64, d]
        lib.oracle_learned_matrix.argtypes = [d, ctypes.c_int, ctypes.c_int, d, ctypes.c_int,
                                              ctypes.c_int, d, u64]
        lib.oracle_sp2_thresh.argtypes = [d, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_int, d, ctypes.POINTER(_Result), d]
        ub = ctypes.POINTER(ctypes.c_ubyte)
        lib.oracle_mu_dm.argtypes = [d, ctypes.c_int, ctypes.c_double, d, d]
        lib.oracle_graph_parts.argtypes = [d, ctypes.c_int, ctypes.c_double, ctypes.c_int, ub]
        lib.oracle_graph_density.argtypes = [d, d, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                             ctypes.c_double, d, i]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(H):
    H = np.ascontiguousarray(np.asarray(H, dtype=np.float64))
    if H.ndim != 2 or H.shape[0] != H.shape[1]:
        raise ValueError("H must be square")
    return H


def max_threads() -> int:
    return int(_load().oracle_max_threads())


class SP2Result:
    def __init__(self, D, r, tr_hist, e_hist):
        self.D = D
        self.status = int(r.status)
        self.iterations = int(r.iterations)
        self.emin = float(r.emin)
        self.emax = float(r.emax)
        self.trace = float(r.trace)
        self.idempotency = float(r.idempotency)
        self.branch_mask = (int(r.branch_mask[0]), int(r.branch_mask[1]))
        self.tr_hist = tr_hist[: self.iterations]
        self.e_hist = e_hist[: self.iterations]

    def branches(self):
        """List of 0/1 per step: 1 when the step used 2X - X^2."""
        m = self.branch_mask[0] | (self.branch_mask[1] << 64)
        return [(m >> k) & 1 for k in range(self.iterations)]


def gershgorin(H):
    """Gershgorin-circle bounds of (H + H^T)/2 (paper: Section "Distributed matrices")."""
    H = _f64(H)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    st = _load().oracle_gershgorin(_dp(H), H.shape[0], ctypes.byref(lo), ctypes.byref(hi))
    if st != OK:
        raise ValueError(f"oracle_gershgorin status {st}")
    return lo.value, hi.value


def sp2_init(H, emin, emax):
    """D_0 = (emax I - H)/(emax - emin) (paper: Section "SP2 solver", first equation)."""
    H = _f64(H)
    X0 = np.empty_like(H)
    _load().oracle_sp2_init(_dp(H), H.shape[0], emin, emax, _dp(X0))
    return X0


def jacobi_eigh(H, max_sweeps=100):
    """Cyclic-by-row Jacobi eigen-decomposition: (w ascending, V columns, sweeps)."""
    H = _f64(H)
    n = H.shape[0]
    w = np.empty(n)
    V = np.empty((n, n))
    sw = ctypes.c_int()
    st = _load().oracle_jacobi_eigh(_dp(H), n, _dp(w), _dp(V), max_sweeps, ctypes.byref(sw))
    if st != OK:
        raise ValueError(f"oracle_jacobi_eigh status {st}")
    return w, V, sw.value


def jacobi_dm(H, n_occ):
    """D = sum_{i<n_occ} v_i v_i^T (paper: Section "Single-particle density matrix",
    the Fermi-Dirac construction in the zero-temperature limit).  Returns (D, w, gap)."""
    H = _f64(H)
    n = H.shape[0]
    D = np.empty((n, n))
    w = np.empty(n)
    gap = ctypes.c_double()
    sw = ctypes.c_int()
    st = _load().oracle_jacobi_dm(_dp(H), n, n_occ, _dp(D), _dp(w), ctypes.byref(gap),
                                  ctypes.byref(sw))
    if st == DEGENERATE:
        raise DegenerateError(f"HOMO-LUMO gap {gap.value:.3e} at or below 1e-8 of the spectral width")
    if st != OK:
        raise ValueError(f"oracle_jacobi_dm status {st}")
    return D, w, gap.value


def sp2(H, n_occ, tol=1e-10, max_iter=100, nthreads=1):
    """Scalar SP2 loop (paper: Section "SP2 solver", equations and listing)."""
    H = _f64(H)
    n = H.shape[0]
    D = np.zeros((n, n))
    r = _Result()
    cap = max(max_iter, 1)
    trh = np.zeros(cap)
    eh = np.zeros(cap)
    _load().oracle_sp2(_dp(H), n, n_occ, tol, max_iter, nthreads, _dp(D), ctypes.byref(r),
                       _dp(trh), _dp(eh))
    return SP2Result(D, r, trh, eh)


def sp2_spectral(eigvals, n_occ, emin, emax, tol=1e-10, max_iter=100):
    """SP2 recursion applied eigenvalue by eigenvalue.  Returns (SP2Result, x_final)."""
    lam = np.ascontiguousarray(np.asarray(eigvals, dtype=np.float64))
    n = lam.size
    x = np.zeros(n)
    r = _Result()
    cap = max(max_iter, 1)
    trh = np.zeros(cap)
    eh = np.zeros(cap)
    _load().oracle_sp2_spectral(_dp(lam), n, n_occ, emin, emax, tol, max_iter, _dp(x),
                                ctypes.byref(r), _dp(trh), _dp(eh))
    return SP2Result(None, r, trh, eh), x


def sp2_step_entries(X, grow, I, J):
    """Entries (I[t], J[t]) of X^2 (grow=0) or 2X - X^2 (grow=1)."""
    X = _f64(X)
    I = np.ascontiguousarray(np.asarray(I, dtype=np.int32))
    J = np.ascontiguousarray(np.asarray(J, dtype=np.int32))
    out = np.empty(I.size)
    _load().oracle_sp2_step_entries(_dp(X), X.shape[0], int(grow), _ip(I), _ip(J), I.size,
                                    _dp(out))
    return out


def _coef(coef):
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64).reshape(-1, 3))
    return c, c.shape[0]


def learned_spectral(eigvals, n_occ, emin, emax, coef):
    """The learned recursive expansion on eigenvalues (layer maps a x^2 + b x + c,
    particle-hole form when tr <= n_occ).  coef: (layers, 3).
    Returns (x_final, branches, traces)."""
    lam = np.ascontiguousarray(np.asarray(eigvals, dtype=np.float64))
    c, L = _coef(coef)
    x = np.empty(lam.size)
    mask = (ctypes.c_uint64 * 2)()
    trh = np.zeros(max(L, 1))
    st = _load().oracle_learned_spectral(_dp(lam), lam.size, int(n_occ), float(emin), float(emax),
                                         _dp(c), L, _dp(x), mask, _dp(trh))
    if st != OK:
        raise ValueError(f"oracle_learned_spectral status {st}")
    m = int(mask[0]) | (int(mask[1]) << 64)
    return x, [(m >> k) & 1 for k in range(L)], trh[:L]


def learned_matrix(H, n_occ, coef, nthreads=1):
    """The learned recursive expansion on the matrix H.  Returns (D, branches)."""
    H = _f64(H)
    c, L = _coef(coef)
    D = np.empty_like(H)
    mask = (ctypes.c_uint64 * 2)()
    st = _load().oracle_learned_matrix(_dp(H), H.shape[0], int(n_occ), _dp(c), L, int(nthreads),
                                       _dp(D), mask)
    if st != OK:
        raise ValueError(f"oracle_learned_matrix status {st}")
    m = int(mask[0]) | (int(mask[1]) << 64)
    return D, [(m >> k) & 1 for k in range(L)]


def cheb_coeffs(L, beta_scaled, mu_scaled, q=None):
    """c_0..c_L of 1/(1 + exp(beta_scaled (x - mu_scaled))) on [-1, 1] (Chebyshev-Gauss
    rule, q nodes; paper: Section "Chebyshev polynomial expansion", first equation)."""
    q = 4 * (L + 1) if q is None else q
    c = np.zeros(L + 1)
    st = _load().oracle_cheb_coeffs(int(L), float(beta_scaled), float(mu_scaled), int(q), _dp(c))
    if st != OK:
        raise ValueError(f"oracle_cheb_coeffs status {st}")
    return c


def cheb_density(H, L, beta, mu, q=None, nthreads=1):
    """sum_{n<=L} c_n T_n((H - a)/b) by the serial recursion T_{n+1} = 2 H T_n - T_{n-1}
    (paper: Section "Chebyshev polynomial expansion").  Returns (D, c, (a, b))."""
    H = _f64(H)
    q = 4 * (L + 1) if q is None else q
    D = np.empty_like(H)
    c = np.zeros(L + 1)
    ab = np.zeros(2)
    st = _load().oracle_cheb_density(_dp(H), H.shape[0], int(L), float(beta), float(mu), int(q),
                                     int(nthreads), _dp(D), _dp(c), _dp(ab))
    if st != OK:
        raise ValueError(f"oracle_cheb_density status {st}")
    return D, c, (ab[0], ab[1])


def cheb_ps_split(c, k, m):
    """d[j, i] of sum_n c_n T_n = sum_j T_k^j sum_{i<k} d[j, i] T_i (Paterson-Stockmeyer
    form of the paper's ansatz equation); len(c) must be k m."""
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
    if c.size != k * m:
        raise ValueError("len(c) must be k m")
    d = np.zeros(k * m)
    st = _load().oracle_cheb_ps_split(_dp(c), int(k), int(m), _dp(d))
    if st != OK:
        raise ValueError(f"oracle_cheb_ps_split status {st}")
    return d.reshape(m, k)


def mu_dm(H, mu):
    """Zero-temperature D at chemical potential mu: the projector on the
    eigenvalues below mu (Section "Single-particle density matrix", the
    Fermi-Dirac function as beta -> infinity).  Returns (D, w)."""
    H = _f64(H)
    n = H.shape[0]
    D = np.empty((n, n))
    w = np.empty(n)
    st = _load().oracle_mu_dm(_dp(H), n, float(mu), _dp(D), _dp(w))
    if st == DEGENERATE:
        raise DegenerateError(f"an eigenvalue lies within 1e-8 of the spectral width of mu = {mu}")
    if st != OK:
        raise ValueError(f"oracle_mu_dm status {st}")
    return D, w


def graph_parts(G, tau, parts):
    """(parts, n) bool membership of the core-halo parts (Section "Graph-based
    Divide electronic structure": adjacency |G_lj| >= tau, l != j; core parts
    = regular segments of the index list; halo = neighbours of core nodes)."""
    G = _f64(G)
    n = G.shape[0]
    out = np.zeros((parts, n), dtype=np.uint8)
    st = _load().oracle_graph_parts(_dp(G), n, float(tau), int(parts),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
    if st != OK:
        raise ValueError(f"oracle_graph_parts status {st}")
    return out.astype(bool)


def segment_starts(n, parts):
    """Core part k is [starts[k], starts[k+1]): regular segments of 0..n-1."""
    return [(k * n) // parts for k in range(parts + 1)]


def graph_density(H, tau, parts, mu, G=None):
    """Graph-partitioned density matrix (the general solver routine of the
    graph section, with each part's density matrix from Jacobi at chemical
    potential mu).  G = the auxiliary graph matrix (default H).
    Returns (D, sizes)."""
    H = _f64(H)
    G = H if G is None else _f64(G)
    n = H.shape[0]
    D = np.empty((n, n))
    sizes = np.zeros(parts, dtype=np.int32)
    st = _load().oracle_graph_density(_dp(H), _dp(G), n, float(tau), int(parts), float(mu), _dp(D),
                                      _ip(sizes))
    if st == DEGENERATE:
        raise DegenerateError("a part has an eigenvalue at mu")
    if st != OK:
        raise ValueError(f"oracle_graph_density status {st}")
    return D, sizes


def sp2_thresh(H, n_occ, tau, tol=1e-10, max_iter=100, nthreads=1):
    """SP2 with the listing's drop threshold tau (entries with |x| < tau are
    dropped after the product and after the 2X - X^2 update).  Returns the
    result of sp2() plus .margin, the closest drop decision
    (| |v| - tau | / max(|v|, tau))."""
    H = _f64(H)
    n = H.shape[0]
    D = np.zeros((n, n))
    res = _Result()
    mg = ctypes.c_double()
    _load().oracle_sp2_thresh(_dp(H), n, int(n_occ), float(tol), int(max_iter), float(tau),
                              int(nthreads), _dp(D), ctypes.byref(res), ctypes.byref(mg))
    out = SP2Result(D, res, np.zeros(0), np.zeros(0))
    out.margin = mg.value
    return out
