"""GPU parity of the matrix-core sine transform (dense DST-I matrix product
on MFMA) against the CPU oracle, and its agreement with the FFT engine.

Tolerances (relative 2-norm):
  FP64 P^{-1}: 1e-13, as for the FFT: each output of a transform is a dot
    product of n <= 127 terms, error O(sqrt(n) eps) = O(1e-15).
  FP32 P^{-1}: three FP32 products of length n <= 127 in sequence, each
    adding O(sqrt(n) 2^-24) relative error: 4 * 3 * sqrt(127) * 2^-24
    = 8.1e-6 bounds it.
  MINRES iterates: as for the FFT path (1e-10 FP64 against the oracle).
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import csl_oracle as O
from paper_2408_00488_amd import workloads as WL

pytestmark = pytest.mark.gpu

FP32_TOL = 4 * 3 * math.sqrt(127) * 2.0 ** -24


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


def _eligible(n):
    return 15 <= n <= 127


# axes of n = 7 and n >= 255 stay on the FFT: mixed engines within a system
SHAPES = [((15, 31), [1.0, 2.0]), ((63, 63), None), ((127, 127), None), ((3, 127), None),
          ((127, 511), None), ((255, 63), None), ((7, 15, 31), [0.5, 1.0, 2.0]),
          ((31, 31, 31), None), ((15, 127, 63), None)]


@pytest.mark.parametrize("shape,lengths", SHAPES)
@pytest.mark.parametrize("fp32", [False, True])
def test_apply_Pinv_gemm(csl, shape, lengths, fp32):
    _say("apply_Pinv gemm", shape, fp32)
    a = _coef(shape, 13)
    x = _crand(shape, 14)
    alpha, beta = -120.0, 7.5
    p = csl.Problem(cuda(a), alpha, beta, lengths=lengths, pinv_fp32=fp32, dst="gemm")
    assert p.dst_engines == tuple("gemm" if _eligible(n) else "fft" for n in shape)
    y = csl.apply_Pinv(p, cuda(x)).cpu().numpy()
    ref = O.apply_Pinv(x, p.abar, alpha, beta, lengths)
    assert rel(y, ref) <= (FP32_TOL if fp32 else 1e-13)


def test_engine_selection(csl):
    a = cuda(_coef((63, 255), 15))
    assert csl.Problem(a, 1.0, 1.0, dst="fft").dst_engines == ("fft", "fft")
    assert csl.Problem(a, 1.0, 1.0, dst="gemm").dst_engines == ("gemm", "fft")
    auto = csl.Problem(a, 1.0, 1.0).dst_engines
    assert auto[1] == "fft" and auto[0] in ("fft", "gemm")
    # the timed choice is cached per shape and precision: a second problem agrees
    assert csl.Problem(a, 2.0, -1.0).dst_engines == auto
    small = cuda(_coef((7, 7), 16))
    assert csl.Problem(small, 1.0, 1.0, dst="gemm").dst_engines == ("fft", "fft")
    with pytest.raises(KeyError):
        csl.Problem(a, 1.0, 1.0, dst="dense")


@pytest.mark.parametrize("n", [31, 63, 127])
def test_solve_gemm_matches_oracle_and_fft(csl, n):
    w = WL.workload("c1", n_override=n)
    s = w.systems[0]
    _say("solve gemm c1", n)
    pg = csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, dst="gemm")
    pf = csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, dst="fft")
    assert pg.dst_engines == ("gemm", "gemm")
    zg, ig = csl.minres_solve(pg, cuda(s.f), raise_on_error=False, timeout_ms=30000)
    zf, if_ = csl.minres_solve(pf, cuda(s.f), raise_on_error=False, timeout_ms=30000)
    assert ig["status"] == 0 and if_["status"] == 0
    assert ig["relres_true"] <= 1e-8
    po = O.Problem(s.a, s.lam.real, s.lam.imag)
    zo, io = po.solve(s.f, tol=1e-8)
    zg = zg.cpu().numpy()
    if ig["iters"] == io["iters"]:
        assert rel(zg, zo) <= 1e-10
    else:
        assert abs(ig["iters"] - io["iters"]) <= 1
        zx, _ = po.solve(s.f, fixed_iters=ig["iters"])
        assert rel(zg, zx) <= 1e-10
    assert abs(ig["iters"] - if_["iters"]) <= 1
    assert rel(zg, zf.cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("shape", [(31, 31, 31), (15, 63, 127)])
def test_solve_3d_gemm(csl, shape):
    _say("solve 3-D gemm", shape)
    a = _coef(shape, 17, 1.0, 3.0)
    f = _crand(shape, 18)
    lam = 10 + 100j
    p = csl.Problem(cuda(a), lam.real, lam.imag, dst="gemm", pinv_fp32=True)
    z, info = csl.minres_solve(p, cuda(f), raise_on_error=False, timeout_ms=30000)
    assert info["status"] == 0 and info["relres_true"] <= 1e-8
    po = O.Problem(a, lam.real, lam.imag)
    zg = z.cpu().numpy()
    r = f - O.apply_A(po.K, lam.real, lam.imag, np.conj(zg))
    # the user solution z solves (K + lambda I) z = f; apply_A acts on conj
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-8
    # element by element against the FP64 oracle's iterate after the GPU's
    # number of steps (FP32 preconditioner form: 1e-6)
    zx, _ = po.solve(f, fixed_iters=info["iters"])
    _say("  vs oracle", info["iters"], rel(zg, zx))
    assert rel(zg, zx) <= 1e-6


def test_batch_gemm_and_fft_mixed(csl):
    w = WL.workload("c4", count_override=8)
    probs = []
    for j, s in enumerate(w.systems):
        probs.append(csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=(j % 2 == 1),
                                 dst=("gemm" if j % 4 < 2 else "fft")))
    _say("batch gemm mix", [p.dst_engines for p in probs])
    F = [cuda(s.f) for s in w.systems]
    b = csl.Batch(probs, timeout_ms=30000)
    zs, infos = b.solve(F)
    first = [z.cpu().numpy().copy() for z in zs]
    for k in range(3):
        zs2, infos2 = b.solve(F)
        for z1, z2 in zip(first, zs2):
            assert np.array_equal(z1, z2.cpu().numpy())
    for s, z, info, p in zip(w.systems, first, infos, probs):
        assert info["status"] == 0 and info["relres_true"] <= 1e-8, info
        zo = O.Problem(s.a, s.lam.real, s.lam.imag).direct(s.f)
        assert rel(z, zo) <= 1e-6


def test_tune_keeps_forced_engines_and_may_move_auto_ones(csl):
    # problem_tune may move an automatically chosen matrix-core axis to the
    # FFT (never a forced one, never an axis without an FFT); the tuned
    # problem still solves to the oracle's result
    shape = (31, 31, 31)
    a = _coef(shape, 7)
    f = _crand(shape, 8)
    lam = complex(12.0, 30.0)
    forced = csl.Problem(cuda(a), lam.real, lam.imag, dst="gemm", pinv_fp32=True)
    forced.tune(cuda(f))
    assert forced.dst_engines == ("gemm", "gemm", "gemm")
    auto = csl.Problem(cuda(a), lam.real, lam.imag, pinv_fp32=True)
    before = auto.dst_engines
    t = auto.tune(cuda(f))
    after = auto.dst_engines
    _say("auto engines", before, "->", after, t)
    assert all(e2 == e1 or e2 == "fft" for e1, e2 in zip(before, after))
    po = O.Problem(a, lam.real, lam.imag)
    for p in (forced, auto):
        z, info = csl.minres_solve(p, cuda(f), timeout_ms=30000)
        zg = z.cpu().numpy()
        r = f - O.apply_A(po.K, lam.real, lam.imag, np.conj(zg))
        assert info["status"] == 0 and np.linalg.norm(r) / np.linalg.norm(f) <= 1.01e-8
        # tuner-moved (auto) and forced engines: element by element against the
        # FP64 oracle after the GPU's number of steps
        zx, _ = po.solve(f, fixed_iters=info["iters"])
        _say("  ", p.dst_engines, "vs oracle", rel(zg, zx))
        assert rel(zg, zx) <= 1e-6
    mixed = csl.Problem(cuda(_coef((20, 63), 9)), lam.real, lam.imag)
    mixed.tune(cuda(_crand((20, 63), 10)))
    assert mixed.dst_engines[0] == "gemm"   # n + 1 = 21 has no FFT
    for p in (forced, auto, mixed):
        p.close()
