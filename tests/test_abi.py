"""The C ABI: the library loads, exports every declared entry point, and its
host-side argument checks answer without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sp2.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(sp2_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_expected_calls():
    names = declared_functions()
    for want in ("sp2_density", "sp2_workspace_size", "sp2_status_str", "sp2_version", "sp2_history"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_2401_13772_amd as sp2
    lib = ctypes.CDLL(sp2.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(sp2.exported_symbols()) <= set(declared_functions())


def test_host_only_queries():
    import paper_2401_13772_amd as sp2
    assert sp2.sp2_version() >= 100
    assert sp2.sp2_status_str(0) == "converged"
    assert "invalid" in sp2.sp2_status_str(-1)
    n = 1000
    ws = sp2.sp2_workspace_size(n, "f64", "f64")
    ldp = 1024
    assert ws >= 2 * ldp * ldp * 8
    assert sp2.sp2_workspace_size(0, "f64", "f64") == 0
    assert sp2.sp2_workspace_size(70000, "f64", "f64") == 0
    # the split modes add two sets of 16-bit planes
    assert sp2.sp2_workspace_size(n, "f64", "f16x2") >= ws + 2 * 2 * ldp * ldp * 2
    assert sp2.sp2_workspace_size(n, "f64", "bf16x3") > sp2.sp2_workspace_size(n, "f64", "f16x2")
    assert sp2.sp2_workspace_size(n, "f64", "fp8") >= ws + 2 * 2 * ldp * ldp      # two byte planes


def _call(lib, H=1 << 20, D=1 << 24, n=4, ld=4, n_occ=2, tol=1e-10, max_iter=50, dtype=0, compute=0,
          ws=1 << 28, wsb=1 << 30):
    info = (ctypes.c_char * 128)()
    vp = ctypes.c_void_p
    return lib.sp2_density(vp(H), vp(D), n, ld, n_occ, ctypes.c_double(tol), max_iter, dtype,
                           compute, -1, vp(ws), ctypes.c_size_t(wsb), vp(0), info)


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), -1), (dict(ld=3), -1), (dict(n_occ=5), -1), (dict(n_occ=-1), -1),
    (dict(tol=0.0), -1), (dict(tol=float("nan")), -1), (dict(max_iter=129), -1),
    (dict(max_iter=-1), -1), (dict(dtype=7), -1), (dict(compute=9), -1), (dict(H=0), -1),
    (dict(compute=1), -5), (dict(ws=0), -3), (dict(ws=257), -3), (dict(wsb=16), -3),
    (dict(D=(1 << 20) + 64), -1), (dict(D=(1 << 28) + 512), -1),
])
def test_argument_checks_without_gpu(kw, code):
    """Every rejection below happens before the first HIP call."""
    import paper_2401_13772_amd as sp2
    lib = ctypes.CDLL(sp2.LIB_PATH)
    lib.sp2_density.restype = ctypes.c_int
    assert _call(lib, **kw) == code


def test_learned_model_host_calls_without_gpu(tmp_path):
    """Model create / coefficients / save / load / destroy touch no GPU: the
    coefficients are rounded to FP32 and survive the text round trip exactly."""
    import numpy as np

    import paper_2401_13772_amd as sp2
    coef = np.array([[1.0, 0.0, 0.0], [1.1, -0.1, 1e-3], [0.7, 0.3, -2.5e-4]])
    m = sp2.Learned.from_coefficients(coef)
    c, loss = m.coefficients()
    assert np.array_equal(c, coef.astype(np.float32).astype(np.float64)) and loss == 0.0
    path = tmp_path / "m.txt"
    m.save(path)
    m2 = sp2.Learned.load(path)
    assert np.array_equal(m2.coefficients()[0], c)
    m.close()
    m2.close()
    (tmp_path / "bad.txt").write_text("not a model\n")
    with pytest.raises(RuntimeError):
        sp2.Learned.load(tmp_path / "bad.txt")
    with pytest.raises(RuntimeError):
        sp2.Learned.from_coefficients(np.array([[1.0, float("nan"), 0.0]]))


def test_plan_and_learned_argument_checks_without_gpu():
    """Rejections that happen before any HIP call."""
    import paper_2401_13772_amd as sp2
    lib = ctypes.CDLL(sp2.LIB_PATH)
    lib.sp2_plan_create.restype = ctypes.c_int
    h = ctypes.c_void_p()
    ns = (ctypes.c_int * 2)(64, 64)
    no = (ctypes.c_int * 2)(32, 32)
    bad_n = (ctypes.c_int * 2)(64, 4096)
    bad_no = (ctypes.c_int * 2)(32, 65)
    assert lib.sp2_plan_create(ctypes.byref(h), 0, ns, no, 0, 0, ctypes.c_double(1e-10), 50, None) == -1
    assert lib.sp2_plan_create(ctypes.byref(h), 2, bad_n, no, 0, 0, ctypes.c_double(1e-10), 50, None) == -1
    assert lib.sp2_plan_create(ctypes.byref(h), 2, ns, bad_no, 0, 0, ctypes.c_double(1e-10), 50, None) == -1
    assert lib.sp2_plan_create(ctypes.byref(h), 2, ns, no, 0, 0, ctypes.c_double(0.0), 50, None) == -1
    assert lib.sp2_plan_create(ctypes.byref(h), 2, ns, no, 0, 2, ctypes.c_double(1e-10), 50, None) == -5
    assert not h.value
    lib.sp2_learned_density.restype = ctypes.c_int
    assert lib.sp2_learned_density(None, 1, 64, None, None, None, 0, 0, ctypes.c_double(1e-6), None,
                                   None) == -1


@pytest.mark.parametrize("k,m,beta,mu,code", [
    (0, 1, 1.0, 0.0, -1), (65, 1, 1.0, 0.0, -1), (1, 0, 1.0, 0.0, -1), (1, 6, 1.0, 0.0, -1),
    (4, 9, 1.0, 0.0, -1), (4, 4, 0.0, 0.0, -1), (4, 4, float("inf"), 0.0, -1),
    (4, 4, 1.0, float("nan"), -1), (4, 4, 1.0, 0.0, -3),
])
def test_cheb_argument_checks_without_gpu(k, m, beta, mu, code):
    """The Chebyshev entry point rejects k outside 1..64, m outside 1..k+4, a
    non-positive or non-finite beta and a non-finite mu before any HIP call;
    the last case passes every argument check and fails on the missing
    workspace."""
    import paper_2401_13772_amd as sp2
    lib = ctypes.CDLL(sp2.LIB_PATH)
    lib.sp2_cheb_density.restype = ctypes.c_int
    vp = ctypes.c_void_p
    info = (ctypes.c_char * 128)()
    assert lib.sp2_cheb_density(vp(1 << 20), vp(1 << 24), 64, 64, 0, ctypes.c_double(mu),
                                ctypes.c_double(beta), k, m, vp(0), ctypes.c_size_t(0), vp(0),
                                info) == code


@pytest.mark.parametrize("kw,code", [
    (dict(G=0), -1), (dict(n=0), -1), (dict(ld=31), -1), (dict(parts=0), -1), (dict(parts=33), -1),
    (dict(tau=-1.0), -1), (dict(tau=float("nan")), -1), (dict(tau=float("inf")), -1), (dict(dtype=5), -1),
    (dict(tol=0.0), -1), (dict(max_iter=-1), -1), (dict(max_iter=129), -1),
])
def test_graph_argument_checks_without_gpu(kw, code):
    """sp2_graph_create rejects its arguments before any HIP call; the other
    graph calls reject a NULL graph."""
    import paper_2401_13772_amd as sp2
    lib = ctypes.CDLL(sp2.LIB_PATH)
    lib.sp2_graph_create.restype = ctypes.c_int
    a = dict(G=1 << 20, n=32, ld=32, dtype=0, tau=0.1, parts=4, tol=1e-10, max_iter=50)
    a.update(kw)
    h = ctypes.c_void_p()
    vp = ctypes.c_void_p
    assert lib.sp2_graph_create(ctypes.byref(h), vp(a["G"]), a["n"], a["ld"], a["dtype"],
                                ctypes.c_double(a["tau"]), a["parts"], ctypes.c_double(a["tol"]),
                                a["max_iter"], vp(0)) == code
    assert not h.value
    assert lib.sp2_graph_parts(None, None, None) == -1
    assert lib.sp2_graph_nodes(None, 0, None, 0) == -1
    assert lib.sp2_graph_destroy(None) == -1


@pytest.mark.parametrize("kw,code", [
    (dict(H=0), -1), (dict(n=0), -1), (dict(n=70000), -1), (dict(ld=3), -1), (dict(n_occ=5), -1),
    (dict(tol=0.0), -1), (dict(max_iter=129), -1), (dict(dtype=3), -1), (dict(tau=-1.0), -1),
    (dict(tau=float("nan")), -1), (dict(ws=0), -3), (dict(ws=257), -3), (dict(wsb=16), -3),
])
def test_sparse_argument_checks_without_gpu(kw, code):
    """sp2_density_sparse rejects its arguments before any HIP call."""
    import paper_2401_13772_amd as sp2
    lib = ctypes.CDLL(sp2.LIB_PATH)
    lib.sp2_density_sparse.restype = ctypes.c_int
    a = dict(H=1 << 20, D=1 << 24, n=4, ld=4, n_occ=2, tol=1e-10, max_iter=50, dtype=0, tau=1e-6,
             ws=1 << 28, wsb=1 << 30)
    a.update(kw)
    vp = ctypes.c_void_p
    info = (ctypes.c_char * 128)()
    assert lib.sp2_density_sparse(vp(a["H"]), vp(a["D"]), a["n"], a["ld"], a["n_occ"], ctypes.c_double(a["tol"]),
                                  a["max_iter"], a["dtype"], ctypes.c_double(a["tau"]), vp(a["ws"]),
                                  ctypes.c_size_t(a["wsb"]), vp(0), info) == code
    assert sp2.sp2_sparse_workspace_size(0) == 0 and sp2.sp2_sparse_workspace_size(1000) > 2 * 1024 * 1024 * 8
