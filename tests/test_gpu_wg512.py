"""GPU parity of the persistent solver's 512-thread instances (eight waves per
workgroup, for systems whose sine transforms all run on the FFT: one for
batches of 2-D systems, one for any dimension) against the CPU oracle and
against the 256-thread instance, and the rules that choose between them.

Tolerances (relative 2-norm), as for the 256-thread solver:
  MINRES iterates against the FP64 oracle at a matched iteration count:
    1e-10 with the FP64 preconditioner (the target is 1e-8), 1e-6 with the
    FP32 one.
  512 against 256 threads: each element goes through the same arithmetic,
    but the inner-product partials are summed over twice the threads, so
    the Lanczos scalars differ by rounding only: 1e-10 (FP64 P^{-1}).
  With the FP32 preconditioner the Krylov space itself is perturbed at the
    FP32 level, so on small grids, where the FP64 method terminates
    exactly after as many steps as the block system has unknowns, the
    iteration counts can differ (3 x 3: 22 against 18).  Those solutions
    are compared element by element with the FP64 oracle's iterate after
    the GPU's number of steps, at 1e-6, and their residual under the
    oracle's K is checked against the tolerance as well.
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


def _oracle_relres(po, lam, f, z):
    # the block operator acts on conj(z), z the solution of (K + lambda I) z = f
    r = f - O.apply_A(po.K, lam.real, lam.imag, np.conj(z))
    return float(np.linalg.norm(r) / np.linalg.norm(f))


def _vs_oracle_fp32(po, f, zg, info):
    # the FP64 oracle's iterate after the GPU's number of steps
    zf, _ = po.solve(f, fixed_iters=info["iters"])
    return rel(zg, zf)


def _vs_oracle(po, f, zg, info, zo, io):
    if info["iters"] == io["iters"]:
        return rel(zg, zo)
    assert abs(info["iters"] - io["iters"]) <= 1, (info, io)
    zf, _ = po.solve(f, fixed_iters=info["iters"])
    return rel(zg, zf)


def test_selection_rules(csl):
    a2 = cuda(_coef((63, 63), 1))
    a3 = cuda(_coef((7, 15, 31), 2))
    p2 = csl.Problem(a2, -40.0, 3.0, dst="fft")
    p3 = csl.Problem(a3, -40.0, 3.0, dst="fft")
    p3g = csl.Problem(a3, -40.0, 3.0, dst="gemm")
    pg = csl.Problem(a2, -40.0, 3.0, dst="gemm")
    assert pg.dst_engines == ("gemm", "gemm")
    assert p3g.dst_engines == ("fft", "gemm", "gemm")
    assert p2.schedule["block_threads"] == 512
    assert p3.schedule["block_threads"] == 512
    assert pg.schedule["block_threads"] == 256
    assert p3g.schedule["block_threads"] == 256
    # a GEMM axis next to an FFT one also keeps the 256-thread solver
    pm = csl.Problem(cuda(_coef((127, 511), 3)), 5.0, 5.0, dst="gemm")
    assert pm.dst_engines == ("gemm", "fft") and pm.schedule["block_threads"] == 256
    for p in (p3g, pg, pm):
        with pytest.raises(csl.CSLError):
            p.set_schedule(0, 0, 512)
    p2.set_schedule(0, 0, 256)
    assert p2.schedule["block_threads"] == 256
    p2.set_schedule(0, 0, 0)
    assert p2.schedule["block_threads"] == 512
    b = csl.Batch([p2, csl.Problem(a2, 10.0, -3.0, pinv_fp32=True, dst="fft")])
    assert b.schedule["block_threads"] == 512
    assert csl.Batch([p2], block_threads=256).schedule["block_threads"] == 256
    # 2-D and 3-D FFT systems together: the any-dimension 512-thread instance
    assert csl.Batch([p2, p3]).schedule["block_threads"] == 512
    assert csl.Batch([p2, p3g]).schedule["block_threads"] == 256
    with pytest.raises(csl.CSLError):
        csl.Batch([p2, p3g], block_threads=512)
    with pytest.raises(csl.CSLError):
        csl.Batch([p2], block_threads=128)


# ragged grids (rows and columns of unequal length), the smallest grid
# (n = 3), lines of the longest FFT (n = 1023) and domain lengths != 1
SHAPES = [((3, 3), None), ((3, 7), [2.0, 0.5]), ((15, 31), [1.0, 2.0]), ((63, 63), None),
          ((3, 511), None), ((511, 3), None), ((1023, 7), None), ((127, 255), None)]


@pytest.mark.parametrize("shape,lengths", SHAPES)
@pytest.mark.parametrize("fp32", [False, True])
def test_single_solve_both_instances(csl, shape, lengths, fp32):
    _say("wg512 single", shape, lengths, fp32)
    a = _coef(shape, 21)
    f = _crand(shape, 22)
    lam = -150.0 + 20.0j
    p = csl.Problem(cuda(a), lam.real, lam.imag, pinv_fp32=fp32, lengths=lengths, dst="fft")
    po = O.Problem(a, lam.real, lam.imag, lengths=lengths)
    zo, io = po.solve(f, tol=1e-8)
    out = {}
    for bt in (512, 256):
        p.set_schedule(0, 0, bt)
        assert p.schedule["block_threads"] == bt
        z, info = csl.minres_solve(p, cuda(f), raise_on_error=False, timeout_ms=30000)
        zg = z.cpu().numpy()
        _say(" ", bt, info, io["iters"])
        assert info["status"] == 0 and info["relres_true"] <= 1e-8
        if fp32:
            assert _oracle_relres(po, lam, f, zg) <= 1.01e-8
            e32 = _vs_oracle_fp32(po, f, zg, info)
            _say("   fp32 vs oracle", e32)
            assert e32 <= 1e-6
        else:
            assert _vs_oracle(po, f, zg, info, zo, io) <= 1e-10
        out[bt] = (zg, info)
    if not fp32:
        assert abs(out[512][1]["iters"] - out[256][1]["iters"]) <= 1
        if out[512][1]["iters"] == out[256][1]["iters"]:
            assert rel(out[512][0], out[256][0]) <= 1e-10


SHAPES3 = [((7, 15, 31), [0.5, 1.0, 2.0]), ((15, 15, 15), None), ((31, 31, 31), None),
           ((3, 63, 7), None)]


@pytest.mark.parametrize("shape,lengths", SHAPES3)
@pytest.mark.parametrize("fp32", [False, True])
def test_single_solve_3d_both_instances(csl, shape, lengths, fp32):
    _say("wg512x single", shape, lengths, fp32)
    a = _coef(shape, 31, 1.0, 3.0)
    f = _crand(shape, 32)
    lam = 10.0 + 100.0j
    p = csl.Problem(cuda(a), lam.real, lam.imag, pinv_fp32=fp32, lengths=lengths, dst="fft")
    po = O.Problem(a, lam.real, lam.imag, lengths=lengths)
    zo, io = po.solve(f, tol=1e-8)
    out = {}
    for bt in (512, 256):
        p.set_schedule(0, 0, bt)
        assert p.schedule["block_threads"] == bt
        z, info = csl.minres_solve(p, cuda(f), raise_on_error=False, timeout_ms=30000)
        zg = z.cpu().numpy()
        _say(" ", bt, info, io["iters"])
        assert info["status"] == 0 and info["relres_true"] <= 1e-8
        if fp32:
            assert _oracle_relres(po, lam, f, zg) <= 1.01e-8
            e32 = _vs_oracle_fp32(po, f, zg, info)
            _say("   fp32 vs oracle", e32)
            assert e32 <= 1e-6
        else:
            assert _vs_oracle(po, f, zg, info, zo, io) <= 1e-10
        out[bt] = (zg, info)
    if not fp32 and out[512][1]["iters"] == out[256][1]["iters"]:
        assert rel(out[512][0], out[256][0]) <= 1e-10


def test_batch_2d_and_3d_on_512(csl):
    # the any-dimension instance carries 2-D and 3-D systems in one launch
    cases = [((31, 31, 31), 10 + 100j, False), ((63, 63), -50 + 20j, False),
             ((15, 31, 15), 5 + 50j, True), ((127, 63), 30 - 40j, True)]
    probs, fs, ref = [], [], []
    for k, (shape, lam, fp32) in enumerate(cases):
        a = _coef(shape, 40 + k, 1.0, 3.0)
        f = _crand(shape, 50 + k)
        p = csl.Problem(cuda(a), lam.real, lam.imag, pinv_fp32=fp32, dst="fft")
        probs.append(p)
        fs.append(cuda(f))
        ref.append((a, f, lam, fp32, O.Problem(a, lam.real, lam.imag)))
    b = csl.Batch(probs, timeout_ms=30000)
    assert b.schedule["block_threads"] == 512
    zs, infos = b.solve(fs)
    _say("wg512x batch", [i["iters"] for i in infos])
    for (a, f, lam, fp32, po), z, info in zip(ref, zs, infos):
        assert info["status"] == 0 and info["relres_true"] <= 1e-8
        zg = z.cpu().numpy()
        if fp32:
            assert _oracle_relres(po, lam, f, zg) <= 1.01e-8
            e32 = _vs_oracle_fp32(po, f, zg, info)
            _say("   fp32 vs oracle", e32)
            assert e32 <= 1e-6
        else:
            zo, io = po.solve(f, tol=1e-8)
            assert _vs_oracle(po, f, zg, info, zo, io) <= 1e-10
    zs2, infos2 = b.solve(fs)
    assert infos2 == infos
    for z1, z2 in zip(zs, zs2):
        assert torch.equal(z1, z2)


@pytest.mark.parametrize("fp32", [False, True])
def test_iterate_after_k_steps_512(csl, fp32):
    # every k exercises a different form of the paired w/x updates
    s = WL.workload("c1", n_override=31).systems[0]
    p = csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=fp32, dst="fft")
    p.set_schedule(0, 0, 512)
    po = O.Problem(s.a, s.lam.real, s.lam.imag)
    f = cuda(s.f)
    for k in range(1, 8):
        z, info = csl.minres_solve(p, f, maxit=k, tol=1e-30, raise_on_error=False)
        assert info["iters"] == k and info["status_name"] == "ERR_NOT_CONVERGED", info
        zo, io = po.solve(s.f, fixed_iters=k)
        assert rel(z.cpu().numpy(), zo) <= (1e-6 if fp32 else 1e-12), k
        assert info["relres_est"] == pytest.approx(io["relres_est"], rel=1e-5 if fp32 else 1e-9)


def test_status_paths_512(csl):
    n = 15
    a = WL.coef_c1(n)
    f = _crand((n, n), 13)
    p = csl.Problem(cuda(a), -50.0, 2.0, dst="fft")
    assert p.schedule["block_threads"] == 512
    z, info = csl.minres_solve(p, cuda(f), maxit=2, raise_on_error=False)
    assert info["status"] == 3 and info["iters"] == 2
    zo, _ = O.Problem(a, -50.0, 2.0).solve(f, maxit=2)
    assert rel(z.cpu().numpy(), zo) <= 1e-12
    z, info = csl.minres_solve(p, torch.zeros((n, n), dtype=torch.complex128, device="cuda"))
    assert info["status"] == 0 and info["iters"] == 0 and not z.abs().sum().item()
    bad = f.copy()
    bad[3, 4] = np.nan
    z, info = csl.minres_solve(p, cuda(bad), raise_on_error=False)
    assert info["status"] == 5


def test_batch_both_instances_and_replays(csl):
    w = WL.workload("c4", count_override=8)
    probs = [csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=(j % 2 == 1), dst="fft")
             for j, s in enumerate(w.systems)]
    fs = [cuda(s.f) for s in w.systems]
    res = {}
    for bt in (512, 256):
        b = csl.Batch(probs, block_threads=bt, timeout_ms=30000)
        assert b.schedule["block_threads"] == bt
        zs, infos = b.solve(fs)
        _say("wg512 batch", bt, [i["iters"] for i in infos])
        for j, (s, p, z, info) in enumerate(zip(w.systems, probs, zs, infos)):
            assert info["status"] == 0 and info["relres_true"] <= 1e-8
            po = O.Problem(s.a, s.lam.real, s.lam.imag)
            if j % 2:
                assert _oracle_relres(po, s.lam, s.f, z.cpu().numpy()) <= 1.01e-8
                assert _vs_oracle_fp32(po, s.f, z.cpu().numpy(), info) <= 1e-6
            else:
                zo, io = po.solve(s.f)
                assert _vs_oracle(po, s.f, z.cpu().numpy(), info, zo, io) <= 1e-10
        first = [z.clone() for z in zs]
        for _ in range(3):
            zs2, infos2 = b.solve(fs)
            torch.cuda.synchronize()
            assert infos2 == infos
            for z1, z2 in zip(first, zs2):
                assert torch.equal(z1, z2)
        res[bt] = ([z.cpu().numpy() for z in first], infos)
        b.close()
    for j, (z5, z2, i5, i2) in enumerate(zip(res[512][0], res[256][0], res[512][1], res[256][1])):
        if j % 2 == 0 and i5["iters"] == i2["iters"]:
            assert rel(z5, z2) <= 1e-10


def test_tuners_consider_both_sizes(csl):
    w = WL.workload("c4", count_override=4)
    probs = [csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=True, dst="fft")
             for s in w.systems]
    fs = [cuda(s.f) for s in w.systems]
    b = csl.Batch(probs)
    t = b.tune(fs)
    _say("batch tune", t)
    assert t["block_threads"] in (256, 512) and t["candidates"] >= 20
    assert b.schedule["block_threads"] == t["block_threads"]
    zs, infos = b.solve(fs)
    assert all(i["status"] == 0 and i["relres_true"] <= 1e-8 for i in infos)
    p = probs[-1]
    tp = p.tune(fs[-1])
    _say("problem tune", tp)
    assert tp["block_threads"] in (256, 512) and p.schedule == dict(tp, candidates=0, ms=0.0,
                                                                      ms_default=0.0)
    z, info = csl.minres_solve(p, fs[-1])
    assert info["status"] == 0 and rel(z.cpu().numpy(), zs[-1].cpu().numpy()) <= 1e-6
