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
