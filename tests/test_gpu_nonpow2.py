"""GPU parity on grids whose n + 1 is not a power of two (3 <= n <= 1022):
such axes have no FFT here and take the dense sine matrix on the matrix
cores; power-of-two axes of the same grid keep their engine choice.  Lines
longer than 511 points need the 64 KiB LDS variant of the solver.

Bars as in the other parity tests: A and FP64 P^{-1} 1e-13; FP32 P^{-1} on
the matrix cores 4 * 3 * sqrt(n_max) * 2^-24 (three FP32 dot products of up
to n_max terms in sequence; 8.1e-6 at 127, 2.3e-5 at 1022); MINRES iterates
against the oracle at the same iteration count 1e-10; FP32-preconditioner
solutions by the oracle's own residual (tol, 1%).
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import csl_oracle as O

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


def _crand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def _coef(shape, seed, lo=0.5, hi=2.0):
    return np.random.default_rng(seed).uniform(lo, hi, shape)


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _pow2(n):
    return ((n + 1) & n) == 0


SHAPES = [((5, 9), None), ((12, 12), None), ((20, 31), [1.0, 2.0]), ((100, 63), None),
          ((63, 100), None), ((127, 45), None), ((17, 33, 12), None), ((9, 15, 100), [1.0, 0.5, 2.0]),
          # past 127 points: larger sine matrices, and past 511 the 64 KiB LDS tiles
          ((200, 45), None), ((45, 300), [1.0, 3.0]), ((129, 255), None), ((1000, 9), None),
          ((9, 1022), None), ((600, 600), None), ((150, 20, 33), None), ((7, 31, 700), None)]


def _fp32_tol(shape):
    return 4 * 3 * math.sqrt(max(max(shape), 127)) * 2.0 ** -24


@pytest.mark.parametrize("shape,lengths", SHAPES)
def test_operators(csl, shape, lengths):
    _say("non-power-of-two operators", shape)
    a = _coef(shape, 1)
    x = _crand(shape, 2)
    alpha, beta = -37.5, 12.25
    for fp32 in (False, True):
        p = csl.Problem(cuda(a), alpha, beta, lengths=lengths, pinv_fp32=fp32)
        eng = p.dst_engines
        for ax, n in enumerate(shape):
            if not _pow2(n):
                assert eng[ax] == "gemm", (shape, eng)
        if not fp32:
            y = csl.apply_A(p, cuda(x)).cpu().numpy()
            assert rel(y, O.apply_A(O.build_K(a, lengths), alpha, beta, x)) <= 1e-13
        y = csl.apply_Pinv(p, cuda(x)).cpu().numpy()
        ref = O.apply_Pinv(x, p.abar, alpha, beta, lengths)
        _say("  P^-1", "fp32" if fp32 else "fp64", rel(y, ref))
        assert rel(y, ref) <= (_fp32_tol(shape) if fp32 else 1e-13), (fp32, rel(y, ref))
        p.close()


@pytest.mark.parametrize("shape,lengths", SHAPES)
def test_solve(csl, shape, lengths):
    _say("non-power-of-two solve", shape)
    a = _coef(shape, 3)
    f = _crand(shape, 4)
    lam = complex(20.0, 40.0)
    p = csl.Problem(cuda(a), lam.real, lam.imag, lengths=lengths)
    z, info = csl.minres_solve(p, cuda(f), timeout_ms=30000)
    zg = z.cpu().numpy()
    po = O.Problem(a, lam.real, lam.imag, lengths=lengths)
    zo, io = po.solve(f)
    _say(info, io["iters"])
    assert info["status"] == 0
    if info["iters"] == io["iters"]:
        assert rel(zg, zo) <= 1e-10
    else:
        assert abs(info["iters"] - io["iters"]) <= 1
        zf, _ = po.solve(f, fixed_iters=info["iters"])
        assert rel(zg, zf) <= 1e-10
    # FP32 preconditioner: the oracle's own residual of the GPU solution, and
    # the solution element by element against the FP64 oracle's iterate after
    # the GPU's number of steps (1e-6)
    p32 = csl.Problem(cuda(a), lam.real, lam.imag, lengths=lengths, pinv_fp32=True)
    z32, i32 = csl.minres_solve(p32, cuda(f), timeout_ms=30000)
    z32 = z32.cpu().numpy()
    r = f - O.apply_A(po.K, lam.real, lam.imag, np.conj(z32))
    assert i32["status"] == 0 and np.linalg.norm(r) / np.linalg.norm(f) <= 1.01e-8
    z32o, _ = po.solve(f, fixed_iters=i32["iters"])
    _say("  fp32 vs oracle", rel(z32, z32o))
    assert rel(z32, z32o) <= 1e-6
    p.close()
    p32.close()


def test_mixed_batch_and_engine_rules(csl):
    shapes = [(5, 9), (63, 63), (100, 63), (17, 33, 12), (31, 31)]
    probs, fs, refs = [], [], []
    for j, shape in enumerate(shapes):
        a = _coef(shape, 10 + j)
        f = _crand(shape, 20 + j)
        lam = complex(5.0 + j, 30.0)
        p = csl.Problem(cuda(a), lam.real, lam.imag)
        probs.append(p)
        fs.append(cuda(f))
        refs.append((a, lam, f, p.abar))
    b = csl.Batch(probs, timeout_ms=30000)
    assert b.schedule["block_threads"] == 256   # the matrix-core axes need the 256-thread solver
    zs, infos = b.solve(fs)
    for (a, lam, f, abar), z, info in zip(refs, zs, infos):
        po = O.Problem(a, lam.real, lam.imag)
        assert abar == pytest.approx(po.abar, rel=1e-14)
        zo, io = po.solve(f)
        assert info["status"] == 0 and abs(info["iters"] - io["iters"]) <= 1
        zf = zo if info["iters"] == io["iters"] else po.solve(f, fixed_iters=info["iters"])[0]
        assert rel(z.cpu().numpy(), zf) <= 1e-10
    b.close()
    with pytest.raises(csl.CSLError, match="ERR_ARG"):
        csl.Batch(probs, block_threads=512)
    for p in probs:
        p.close()
    a = cuda(_coef((20, 31), 1))
    with pytest.raises(csl.CSLError, match="ERR_ARG"):
        csl.Problem(a, 1.0, 1.0, dst="fft")
    p = csl.Problem(a, 1.0, 1.0, dst="gemm")
    assert p.dst_engines == ("gemm", "gemm")
    p.close()


def test_adjoint_non_power_of_two(csl):
    shape = (20, 45)
    a = _coef(shape, 5)
    f = _crand(shape, 6)
    zt = _crand(shape, 7)
    lam = complex(-10.0, 60.0)
    p = csl.Problem(cuda(a), lam.real, lam.imag)
    z, _ = csl.minres_solve(p, cuda(f), tol=1e-12)
    g, _ = csl.minres_adjoint(p, z, 2.0 * (z - cuda(zt)), tol=1e-12)
    po = O.Problem(a, lam.real, lam.imag)
    zo = po.direct(f)
    yo, _ = O.adjoint_solve(po, 2.0 * (zo - zt), direct=True)
    go = O.adjoint_gradients(a, lam.real, lam.imag, zo, yo)
    assert rel(g["f"].cpu().numpy(), go["f"]) <= 1e-9
    assert rel(g["a"].cpu().numpy(), go["a"]) <= 1e-9
    assert g["alpha"].item() == pytest.approx(go["alpha"], rel=1e-9)
    assert g["beta"].item() == pytest.approx(go["beta"], rel=1e-9)
    p.close()


def test_batch_with_long_sine_matrix_lines(csl):
    # lines past 511 points take the 64 KiB tiles; the batch shares one
    # launch with short-line and power-of-two systems
    shapes = [(1000, 9), (9, 600), (63, 63), (200, 45), (15, 31, 700)]
    probs, refs = [], []
    for j, shape in enumerate(shapes):
        a = _coef(shape, 40 + j)
        f = _crand(shape, 50 + j)
        lam = complex(8.0 + j, 35.0)
        p = csl.Problem(cuda(a), lam.real, lam.imag, pinv_fp32=(j % 2 == 1))
        probs.append(p)
        refs.append((a, lam, f, p.abar, p.pinv_fp32))
    b = csl.Batch(probs, timeout_ms=60000)
    zs, infos = b.solve([cuda(r[2]) for r in refs])
    for (a, lam, f, abar, fp32), z, info in zip(refs, zs, infos):
        po = O.Problem(a, lam.real, lam.imag)
        assert abar == pytest.approx(po.abar, rel=1e-14)
        assert info["status"] == 0
        zg = z.cpu().numpy()
        if fp32:
            r = f - O.apply_A(po.K, lam.real, lam.imag, np.conj(zg))
            assert np.linalg.norm(r) / np.linalg.norm(f) <= 1.01e-8
            # FP32 preconditioner on long sine-matrix lines: element by
            # element against the FP64 oracle after the GPU's steps (1e-6)
            zx, _ = po.solve(f, fixed_iters=info["iters"])
            _say(a.shape, "fp32", info["iters"], rel(zg, zx))
            assert rel(zg, zx) <= 1e-6
            continue
        zo, io = po.solve(f)
        assert abs(info["iters"] - io["iters"]) <= 1
        zf = zo if info["iters"] == io["iters"] else po.solve(f, fixed_iters=info["iters"])[0]
        _say(a.shape, info["iters"], rel(zg, zf))
        assert rel(zg, zf) <= 1e-10
    b.close()
    for p in probs:
        p.close()
