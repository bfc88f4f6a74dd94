"""GPU check of the allocation-free entry point minres_solve_noalloc (its
workspace is the library's static device array) against minres_solve on a
problem handle, through the C ABI.

Two calls in a row, the second on a smaller grid, then the first again: each
result equals the handle path's element by element (FP64 preconditioner: the
iterates after the same number of steps within 1e-10, the bar of the FP64
solver against the oracle; FP32 preconditioner: 1e-6), and the repeated call
is bitwise equal to the first one, whatever the array held before.  Grids
whose workspace exceeds the array, and axes without an FFT, are refused on
the host with CSL_ERR_ARG before any device work.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2408_00488_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def csl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_00488_amd as C
    C.load_library()
    return C


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    a = a.cpu().numpy().ravel()
    b = b.cpu().numpy().ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _handle_solve(csl, a, lam, f, fp32, iters):
    p = csl.Problem(a, lam.real, lam.imag, pinv_fp32=fp32, dst="fft")
    z, info = csl.minres_solve(p, f, timeout_ms=30000)
    if info["iters"] != iters:
        # a rounding-level difference moved the stopping test: the handle
        # path's iterate after the same number of steps
        assert abs(info["iters"] - iters) <= 1, (info, iters)
        z, info = csl.minres_solve(p, f, maxit=iters, tol=1e-30, raise_on_error=False,
                                   timeout_ms=30000)
    p.close()
    return z, info


def test_noalloc_matches_handle_solve_twice(csl):
    cases = [("c1", 255, False, 1e-10), ("c1", 63, False, 1e-10), ("c3", 31, True, 1e-6)]
    first = None
    for name, n, fp32, tol in cases:
        s = WL.workload(name, n_override=n).systems[0]
        a, f = cuda(s.a), cuda(s.f)
        _say("noalloc", name, n, "fp32" if fp32 else "fp64")
        z, info = csl.minres_solve_noalloc(a, s.lam.real, s.lam.imag, f, pinv_fp32=fp32,
                                           timeout_ms=30000)
        assert info["status"] == 0 and info["relres_true"] <= 1e-8, info
        zh, ih = _handle_solve(csl, a, s.lam, f, fp32, info["iters"])
        e = rel(z, zh)
        _say("  iters", info["iters"], ih["iters"], "vs handle path", e)
        assert e <= tol
        if first is None:
            first = (s, z.clone(), info)
    # the first case again, after the array held the other two systems
    s, z0, i0 = first
    z, info = csl.minres_solve_noalloc(cuda(s.a), s.lam.real, s.lam.imag, cuda(s.f),
                                       timeout_ms=30000)
    assert info == i0 and torch.equal(z, z0)


def test_noalloc_refuses_what_it_cannot_hold(csl):
    g = WL.rng(3)
    for shape in ((1023, 1023), (127, 127, 127), (100, 63)):
        a = torch.ones(shape, dtype=torch.float64, device="cuda")
        f = cuda(WL.complex_normal(g, shape))
        with pytest.raises(csl.CSLError, match="ERR_ARG"):
            csl.minres_solve_noalloc(a, 1.0, 1.0, f)
    # a valid call still works afterwards
    s = WL.workload("c1").systems[0]
    z, info = csl.minres_solve_noalloc(cuda(s.a), s.lam.real, s.lam.imag, cuda(s.f))
    assert info["status"] == 0 and info["relres_true"] <= 1e-8
