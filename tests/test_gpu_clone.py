"""GPU: problem_clone and several right-hand sides of one shifted system
solved as a batch of clones.

- A clone has the same abar, engines, precision and schedule, and solves a
  right-hand side bitwise like the original (same descriptor, same tiling).
- A batch of the original and its clones on different right-hand sides
  gives every solution of the oracle's MINRES at the same iteration count
  (relative 1e-10).
- The clone owns its coefficient copy: it keeps working after the
  original is destroyed.
"""
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


@pytest.mark.parametrize("shape,kw", [((63, 63), {}), ((31, 63), dict(dst="gemm")),
                                      ((15, 31, 15), dict(pinv_fp32=True)),
                                      ((20, 45), dict(abar_rule="geomean"))])
def test_clone_matches_original(csl, shape, kw):
    a = _coef(shape, 1)
    f = cuda(_crand(shape, 2))
    p = csl.Problem(cuda(a), 12.0, 30.0, **kw)
    p.set_schedule(4096, 65536, 0)
    q = p.clone()
    assert q.abar == p.abar and q.dst_engines == p.dst_engines and q.pinv_fp32 == p.pinv_fp32
    assert q.schedule == p.schedule
    z1, i1 = csl.minres_solve(p, f)
    z2, i2 = csl.minres_solve(q, f)
    assert i1 == i2 and torch.equal(z1, z2)
    p.close()
    z3, i3 = csl.minres_solve(q, f)
    assert i3 == i1 and torch.equal(z3, z1)
    q.close()


def test_many_right_hand_sides_as_a_batch(csl):
    shape, lam, count = (63, 63), complex(-20.0, 45.0), 16
    a = _coef(shape, 3)
    p = csl.Problem(cuda(a), lam.real, lam.imag)
    probs = [p] + [p.clone() for _ in range(count - 1)]
    fs_h = [_crand(shape, 100 + j) for j in range(count)]
    b = csl.Batch(probs, timeout_ms=30000)
    zs, infos = b.solve([cuda(f) for f in fs_h])
    po = O.Problem(a, lam.real, lam.imag)
    worst = 0.0
    for f, z, info in zip(fs_h, zs, infos):
        zo, io = po.solve(f)
        assert info["status"] == 0 and abs(info["iters"] - io["iters"]) <= 1
        zf = zo if info["iters"] == io["iters"] else po.solve(f, fixed_iters=info["iters"])[0]
        worst = max(worst, rel(z.cpu().numpy(), zf))
    _say("16 right-hand sides, worst difference", worst)
    assert worst <= 1e-10
    b.close()
    for q in probs:
        q.close()
