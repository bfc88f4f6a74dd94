"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/csl.h, and rejects bad arguments
before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2408_00488_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csl.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB):
        B.build()
    from paper_2408_00488_amd import load_library
    return load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:csl_status|int|char)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["create_problem", "destroy_problem", "apply_A", "apply_Pinv", "minres_solve",
              "minres_adjoint", "batch_create", "batch_solve", "batch_destroy",
              "csl_last_error", "csl_version", "problem_info"]:
        assert n in names, n


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert lib.csl_version() >= 100


def _grid(dim, n, length=1.0):
    from paper_2408_00488_amd import _Grid
    g = _Grid()
    g.dim = dim
    for k in range(3):
        g.n[k] = n[k] if k < len(n) else 0
        g.length[k] = length
    return g


@pytest.mark.parametrize("dim,n,msg", [(4, (7, 7), "dim"), (2, (1024, 7), "between 3 and 1023"),
                                       (2, (7, 2047), "between 3 and 1023"),
                                       (3, (7, 7, 1), "between 3 and 1023"),
                                       (2, (2, 7), "between 3 and 1023"), (2, (7, 1500), "between 3 and 1023")])
def test_create_problem_rejects_bad_grid(lib, dim, n, msg):
    h = ctypes.c_void_p()
    g = _grid(dim, n)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    st = lib.create_problem(ctypes.byref(g), fake, 1.0, 1.0, None, None, ctypes.byref(h))
    assert st == 1
    assert msg in lib.csl_last_error().decode()
    assert not h.value


def test_create_problem_rejects_null_and_nonfinite(lib):
    h = ctypes.c_void_p()
    g = _grid(2, (7, 7))
    assert lib.create_problem(ctypes.byref(g), None, 1.0, 1.0, None, None, ctypes.byref(h)) == 1
    fake = ctypes.c_void_p(0x1000)
    assert lib.create_problem(ctypes.byref(g), fake, float("nan"), 1.0, None, None,
                              ctypes.byref(h)) == 1
    assert "finite" in lib.csl_last_error().decode()


def test_null_handles_rejected(lib):
    assert lib.apply_A(None, None, None, None) == 1
    assert lib.apply_Pinv(None, None, None, None) == 1
    assert lib.minres_solve(None, None, None, None, None, None) == 1
    assert lib.destroy_problem(None) == 1
    assert lib.batch_destroy(None) == 1
    assert lib.batch_create(None, 0, None, ctypes.byref(ctypes.c_void_p())) == 1


def test_tridiagonal_eigenvalues_against_scipy(lib):
    # the host bisection behind problem_ritz, against SciPy's tridiagonal
    # eigensolver: random, clustered and repeated spectra, the sizes 0 and 1
    import numpy as np
    import scipy.linalg as sla
    dp = ctypes.POINTER(ctypes.c_double)
    f = lib.csl_tridiagonal_eigenvalues
    f.argtypes = [dp, dp, ctypes.c_int, dp]
    f.restype = ctypes.c_int
    g = np.random.default_rng(5)
    cases = [(g.standard_normal(50), g.standard_normal(49)),
             (np.ones(40) + 1e-9 * g.standard_normal(40), 1e-6 * g.standard_normal(39)),
             (np.full(30, 2.0), np.zeros(29)),
             (g.uniform(-1, 1, 400), g.uniform(0.5, 1.0, 399)),
             (np.array([3.5]), np.zeros(0))]
    for d, e in cases:
        d = np.ascontiguousarray(d, dtype=np.float64)
        e = np.ascontiguousarray(e, dtype=np.float64)
        th = np.empty(d.size)
        assert f(d.ctypes.data_as(dp), e.ctypes.data_as(dp), d.size, th.ctypes.data_as(dp)) == 0
        ref = sla.eigvalsh_tridiagonal(d, e) if d.size > 1 else d
        scale = max(1.0, np.abs(ref).max())
        assert np.all(np.diff(th) >= 0)
        assert np.abs(th - ref).max() <= 1e-13 * scale, (d.size, np.abs(th - ref).max())
    assert f(None, None, 0, None) == 0
    assert f(None, None, -1, None) == 1


@pytest.mark.parametrize("dim,n,msg", [(2, (1023, 1023), "bytes of workspace"),
                                       (3, (127, 127, 127), "bytes of workspace"),
                                       (2, (100, 63), "power of two"),
                                       (3, (31, 31, 20), "power of two")])
def test_noalloc_refuses_on_the_host(lib, dim, n, msg):
    # the allocation-free solve refuses grids its static workspace cannot
    # hold, and axes without an FFT, before any device work
    g = _grid(dim, n)
    fake_a, fake_f, fake_z = (ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000),
                              ctypes.c_void_p(0x3000))
    st = lib.minres_solve_noalloc(ctypes.byref(g), fake_a, 1.0, 1.0, None, fake_f, fake_z, None,
                                  None, None)
    assert st == 1
    assert msg in lib.csl_last_error().decode()
    assert lib.minres_solve_noalloc(None, fake_a, 1.0, 1.0, None, fake_f, fake_z, None, None,
                                    None) == 1
    assert lib.minres_solve_noalloc(ctypes.byref(g), fake_a, 1.0, 1.0, None, fake_f, fake_f,
                                    None, None, None) == 1
