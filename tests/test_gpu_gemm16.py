"""GPU parity of the FP16 split-product sine-matrix engine (dst "gemm16":
every line scaled by a power of two, matrix and line split into FP16 high
and low parts, three FP16 matrix-core products accumulated in FP32) against
the CPU oracle, in the stand-alone preconditioner and inside MINRES.

Tolerances (relative 2-norm):
  P^{-1}: 1e-6, the FP32 preconditioner's bar (the split keeps each operand
    to about 2^-22 relative; every output is an FP32 sum of at most 64
    products per parity block).
  MINRES iterates against the FP64 oracle after the GPU's number of steps:
    1e-6 (the FP32 preconditioner form).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import csl_oracle as O
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


def _crand(shape, seed, scale=1.0):
    g = np.random.default_rng(seed)
    return scale * (g.standard_normal(shape) + 1j * g.standard_normal(shape))


def _coef(shape, seed, lo=0.5, hi=2.0):
    return np.random.default_rng(seed).uniform(lo, hi, shape)


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _engine(n):
    return "gemm16" if (15 <= n <= 127 or ((n + 1) & n) != 0) else "fft"


SHAPES = [((15, 31), [1.0, 2.0]), ((63, 63), None), ((127, 127), None), ((100, 63), None),
          ((127, 255), None), ((7, 15, 31), [0.5, 1.0, 2.0]), ((31, 31, 31), None),
          ((15, 127, 63), None), ((20, 45), None)]


@pytest.mark.parametrize("shape,lengths", SHAPES)
def test_apply_Pinv_gemm16(csl, shape, lengths):
    a = _coef(shape, 13)
    alpha, beta = -120.0, 7.5
    p = csl.Problem(cuda(a), alpha, beta, lengths=lengths, pinv_fp32=True, dst="gemm16")
    assert p.dst_engines == tuple(_engine(n) for n in shape)
    # magnitudes far from 1 in both directions: the per-line scaling keeps
    # the FP16 parts in range
    for k, scale in enumerate((1.0, 1e-12, 1e9)):
        x = _crand(shape, 14 + k, scale)
        y = csl.apply_Pinv(p, cuda(x)).cpu().numpy()
        ref = O.apply_Pinv(x, p.abar, alpha, beta, lengths)
        e = rel(y, ref)
        _say("apply_Pinv gemm16", shape, scale, e)
        assert e <= 1e-6


def test_gemm16_needs_fp32_preconditioner(csl):
    a = cuda(_coef((63, 63), 1))
    with pytest.raises(csl.CSLError, match="ERR_ARG"):
        csl.Problem(a, 1.0, 1.0, pinv_fp32=False, dst="gemm16")


@pytest.mark.parametrize("shape", [(63, 63), (127, 127), (31, 31, 31), (100, 63)])
def test_solve_gemm16_matches_oracle(csl, shape):
    a = _coef(shape, 17, 1.0, 3.0)
    f = _crand(shape, 18)
    lam = complex(10.0, 100.0) if len(shape) == 3 else complex(-60.0, 25.0)
    p = csl.Problem(cuda(a), lam.real, lam.imag, pinv_fp32=True, dst="gemm16")
    assert "gemm16" in p.dst_engines and p.schedule["block_threads"] == 256
    z, info = csl.minres_solve(p, cuda(f), timeout_ms=30000)
    assert info["status"] == 0 and info["relres_true"] <= 1e-8
    po = O.Problem(a, lam.real, lam.imag)
    zg = z.cpu().numpy()
    zx, _ = po.solve(f, fixed_iters=info["iters"])
    _, io = po.solve(f)
    e = rel(zg, zx)
    _say("solve gemm16", shape, info["iters"], io["iters"], e)
    assert abs(info["iters"] - io["iters"]) <= 2
    assert e <= 1e-6
    # tuning keeps the forced engine
    p.tune(cuda(f))
    assert "gemm16" in p.dst_engines
    z2, info2 = csl.minres_solve(p, cuda(f), timeout_ms=30000)
    assert rel(z2.cpu().numpy(), zx if info2["iters"] == info["iters"]
               else po.solve(f, fixed_iters=info2["iters"])[0]) <= 1e-6


def test_batch_gemm16_with_other_engines(csl):
    # FP16-engine systems share a launch with FFT and FP32 / FP64 matrix-core
    # ones (the FP16 solver instance carries all of them); clones keep the
    # engine
    w = WL.workload("c4", count_override=8)
    probs = []
    dsts = ["gemm16", "fft", "gemm16", "gemm", "gemm16", "fft", "gemm16", "gemm"]
    for j, (s, dst) in enumerate(zip(w.systems, dsts)):
        fp32 = dst == "gemm16" or j in (1, 7)
        probs.append(csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=fp32, dst=dst))
    probs.append(probs[0].clone())
    assert probs[-1].dst_engines == probs[0].dst_engines
    systems = list(w.systems) + [w.systems[0]]
    F = [cuda(s.f) for s in systems]
    b = csl.Batch(probs, timeout_ms=30000)
    zs, infos = b.solve(F)
    _say("gemm16 batch", [p.dst_engines for p in probs], [i["iters"] for i in infos])
    for s, p, z, info in zip(systems, probs, zs, infos):
        assert info["status"] == 0 and info["relres_true"] <= 1e-8
        po = O.Problem(s.a, s.lam.real, s.lam.imag)
        zx, _ = po.solve(s.f, fixed_iters=info["iters"])
        assert rel(z.cpu().numpy(), zx) <= (1e-6 if p.pinv_fp32 else 1e-10)
    zs2, infos2 = b.solve(F)
    assert infos2 == infos
    for z1, z2 in zip(zs, zs2):
        assert torch.equal(z1, z2)
