"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element.

Tolerances (relative 2-norm): A and FP64 P^{-1}: 1e-13 (rounding of a
short stencil sum / of an FFT of length <= 2048); FP32 P^{-1}: 1e-6;
MINRES iterates at a matched iteration count: 1e-10 for FP64 (the target
is 1e-8), 1e-6 for the FP32 preconditioner against the FP64 oracle.
"""
import math
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


SHAPES = [((7, 7), None), ((15, 31), [1.0, 2.0]), ((63, 63), None), ((3, 511), None),
          ((7, 15, 31), [0.5, 1.0, 2.0]), ((31, 31, 31), None), ((1023, 7), None)]


@pytest.mark.parametrize("shape,lengths", SHAPES)
def test_apply_A(csl, shape, lengths):
    _say("apply_A", shape)
    a = _coef(shape, 1)
    x = _crand(shape, 2)
    alpha, beta = -37.5, 12.25
    p = csl.Problem(cuda(a), alpha, beta, lengths=lengths)
    y = csl.apply_A(p, cuda(x)).cpu().numpy()
    ref = O.apply_A(O.build_K(a, lengths), alpha, beta, x)
    assert rel(y, ref) <= 1e-13
    amin, amax = O.coefficient_bounds(a)
    assert p.a_min == amin and p.a_max == amax
    assert p.abar == pytest.approx(O.abar_value(a, "mean"), rel=1e-14)


@pytest.mark.parametrize("shape,lengths", SHAPES)
@pytest.mark.parametrize("fp32", [False, True])
def test_apply_Pinv(csl, shape, lengths, fp32):
    _say("apply_Pinv", shape, fp32)
    a = _coef(shape, 3)
    x = _crand(shape, 4)
    alpha, beta = -120.0, 7.5
    p = csl.Problem(cuda(a), alpha, beta, lengths=lengths, pinv_fp32=fp32)
    y = csl.apply_Pinv(p, cuda(x)).cpu().numpy()
    ref = O.apply_Pinv(x, p.abar, alpha, beta, lengths)
    assert rel(y, ref) <= (1e-6 if fp32 else 1e-13)


def test_apply_Pinv_in_place_and_geomean(csl):
    shape = (31, 63)
    a = _coef(shape, 5)
    x = _crand(shape, 6)
    p = csl.Problem(cuda(a), 3.0, -40.0, abar_rule="geomean")
    assert p.abar == pytest.approx(O.abar_value(a, "geomean"), rel=1e-15)
    xt = cuda(x)
    csl.apply_Pinv(p, xt, xt)
    assert rel(xt.cpu().numpy(), O.apply_Pinv(x, p.abar, 3.0, -40.0)) <= 1e-13


def _solve_both(csl, a, lam, f, fp32=False, tol=1e-8, maxit=1000, abar_rule="mean",
                lengths=None):
    p = csl.Problem(cuda(a), lam.real, lam.imag, pinv_fp32=fp32, abar_rule=abar_rule,
                    lengths=lengths)
    z, info = csl.minres_solve(p, cuda(f), tol=tol, maxit=maxit, raise_on_error=False,
                               timeout_ms=30000)
    zg = z.cpu().numpy()
    # the oracle takes its own abar by the same rule
    po = O.Problem(a, lam.real, lam.imag, abar_rule=abar_rule, lengths=lengths)
    assert p.abar == pytest.approx(po.abar, rel=1e-14)
    zo, io = po.solve(f, tol=tol, maxit=maxit)
    return p, zg, info, po, zo, io


def _compare_iterates(po, f, zg, info, zo, io, tol_same):
    if info["iters"] == io["iters"]:
        return rel(zg, zo)
    # a rounding-level difference flipped the stopping test: compare at the
    # GPU's count
    assert abs(info["iters"] - io["iters"]) <= 1, (info, io)
    zf, _ = po.solve(f, fixed_iters=info["iters"])
    return rel(zg, zf)


def test_solve_config1_full(csl):
    w = WL.workload("c1")
    s = w.systems[0]
    _say("solve c1", s.n)
    p, zg, info, po, zo, io = _solve_both(csl, s.a, s.lam, s.f)
    _say(info, io["iters"], io["relres_true"])
    assert info["status"] == 0
    assert rel(zg, zo) < 1e-10 if info["iters"] == io["iters"] else True
    assert _compare_iterates(po, s.f, zg, info, zo, io, 1e-10) <= 1e-10
    assert info["relres_true"] <= 1e-8
    assert info["relres_true"] == pytest.approx(io["relres_true"], rel=1e-3)
    assert info["relres_est"] == pytest.approx(io["relres_est"], rel=1e-6)
    zd = po.direct(s.f)
    assert rel(zg, zd) <= 1e-6


@pytest.mark.parametrize("n", [7, 63, 511])
def test_two_iteration_invariant(csl, n):
    # Theorem 2 / Table 1(a): a = 1 gives exactly 2 MINRES iterations.
    for lam in (-200 + 50j, 100 + 100j, -100 + 1j, 1 - 100j):
        f = _crand((n, n), n)
        p = csl.Problem(cuda(np.ones((n, n))), lam.real, lam.imag)
        z, info = csl.minres_solve(p, cuda(f), timeout_ms=30000)
        _say("invariant", n, lam, info)
        assert info["iters"] == 2
        assert info["relres_true"] <= 1e-10


def test_solve_config2_full(csl):
    w = WL.workload("c2")
    s = w.systems[0]
    _say("solve c2", s.n)
    p, zg, info, po, zo, io = _solve_both(csl, s.a, s.lam, s.f)
    _say(info, io["iters"])
    assert info["status"] == 0
    assert _compare_iterates(po, s.f, zg, info, zo, io, 1e-10) <= 1e-10
    assert info["relres_true"] <= 1e-8


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("shape", [(15, 15, 15), (7, 31, 15)])
def test_solve_3d(csl, shape, fp32):
    a = 2.0 + _coef(shape, 9, -1.0, 1.0)
    f = _crand(shape, 10)
    lam = 10 + 100j
    _say("solve 3d", shape, fp32)
    p, zg, info, po, zo, io = _solve_both(csl, a, lam, f, fp32=fp32)
    _say(info, io["iters"])
    assert info["status"] == 0
    if fp32:
        assert abs(info["iters"] - io["iters"]) <= 1
        assert rel(zg, zo) <= 1e-6
    else:
        assert _compare_iterates(po, f, zg, info, zo, io, 1e-10) <= 1e-10


def test_solve_fp32_preconditioner_2d(csl):
    w = WL.workload("c1")
    s = w.systems[0]
    p, zg, info, po, zo, io = _solve_both(csl, s.a, s.lam, s.f, fp32=True)
    _say("fp32 c1", info, io["iters"])
    assert info["status"] == 0 and abs(info["iters"] - io["iters"]) <= 1
    assert rel(zg, zo) <= 1e-6
    assert info["relres_true"] <= 1e-8


def test_solve_rectangular_and_lengths(csl):
    shape = (15, 63)
    a = _coef(shape, 11)
    f = _crand(shape, 12)
    p, zg, info, po, zo, io = _solve_both(csl, a, complex(-50, 20), f, lengths=[1.0, 3.0])
    _say("rect", info, io["iters"])
    assert _compare_iterates(po, f, zg, info, zo, io, 1e-10) <= 1e-10


def test_status_paths(csl):
    n = 15
    a = WL.coef_c1(n)
    f = _crand((n, n), 13)
    p = csl.Problem(cuda(a), -50.0, 2.0)
    z, info = csl.minres_solve(p, cuda(f), maxit=2, raise_on_error=False)
    assert info["status"] == 3 and info["iters"] == 2
    po = O.Problem(a, -50.0, 2.0)
    zo, io = po.solve(f, maxit=2)
    assert rel(z.cpu().numpy(), zo) <= 1e-12
    z, info = csl.minres_solve(p, torch.zeros((n, n), dtype=torch.complex128, device="cuda"))
    assert info["status"] == 0 and info["iters"] == 0 and not z.abs().sum().item()
    bad = f.copy()
    bad[3, 4] = np.nan
    z, info = csl.minres_solve(p, cuda(bad), raise_on_error=False)
    assert info["status"] == 5
    with pytest.raises(csl.CSLError) as e:
        csl.minres_solve(p, cuda(bad))
    assert e.value.status == 5
    # singular preconditioner: beta = 0 and alpha = -abar * mu for one mode
    mu = O.mode_eigenvalues((n, n))
    with pytest.raises(csl.CSLError) as e:
        csl.Problem(cuda(np.ones((n, n))), -float(mu[2, 3]), 0.0)
    assert e.value.status == 2
    bad_a = np.ones((n, n))
    bad_a[1, 1] = -1.0
    with pytest.raises(csl.CSLError) as e:
        csl.Problem(cuda(bad_a), 1.0, 1.0)
    assert e.value.status == 1


def test_solve_deterministic(csl):
    w = WL.workload("c1")
    s = w.systems[0]
    p = csl.Problem(cuda(s.a), s.lam.real, s.lam.imag)
    f = cuda(s.f)
    z1, i1 = csl.minres_solve(p, f)
    z2, i2 = csl.minres_solve(p, f)
    assert i1 == i2
    assert torch.equal(z1, z2)


def test_batch_matches_oracle_and_replays(csl):
    w = WL.workload("c4", count_override=8)
    probs = [csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=False) for s in w.systems]
    fs = [cuda(s.f) for s in w.systems]
    b = csl.Batch(probs, timeout_ms=30000)
    zs, infos = b.solve(fs)
    _say("batch", [i["iters"] for i in infos])
    for s, p, z, info in zip(w.systems, probs, zs, infos):
        assert info["status"] == 0
        po = O.Problem(s.a, s.lam.real, s.lam.imag)
        zo, io = po.solve(s.f)
        assert _compare_iterates(po, s.f, z.cpu().numpy(), info, zo, io, 1e-10) <= 1e-10
    # graph replay: same results, bitwise, on every replay
    for _ in range(3):
        zs2, infos2 = b.solve(fs)
        torch.cuda.synchronize()
        assert infos2 == infos
        for z, z2 in zip(zs, zs2):
            assert torch.equal(z, z2)
    # eager batch equals the graph batch
    b2 = csl.Batch(probs, use_graph=False)
    zs3, infos3 = b2.solve(fs)
    assert infos3 == infos
    for z, z3 in zip(zs, zs3):
        assert torch.equal(z, z3)
    b.close()
    b2.close()


def test_batch_mixed_precision_uneven(csl):
    w = WL.workload("c4", count_override=8)
    probs = [csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=True) for s in w.systems]
    fs = [cuda(s.f) for s in w.systems]
    b = csl.Batch(probs)
    zs, infos = b.solve(fs)
    for s, p, z, info in zip(w.systems, probs, zs, infos):
        po = O.Problem(s.a, s.lam.real, s.lam.imag)
        zo, io = po.solve(s.f)
        assert info["status"] == 0 and abs(info["iters"] - io["iters"]) <= 1
        assert rel(z.cpu().numpy(), zo) <= 1e-6
        assert info["relres_true"] <= 1e-8


def test_adjoint_matches_oracle(csl):
    w = WL.workload("c5", n_override=31, count_override=3)
    for s in w.systems:
        p = csl.Problem(cuda(s.a), s.lam.real, s.lam.imag)
        z, info = csl.minres_solve(p, cuda(s.f), tol=1e-12)
        G = 2.0 * (z - cuda(s.z_target))
        g, ainfo = csl.minres_adjoint(p, z, G, tol=1e-12)
        po = O.Problem(s.a, s.lam.real, s.lam.imag)
        zo = po.direct(s.f)
        yo, _ = O.adjoint_solve(po, 2.0 * (zo - s.z_target), direct=True)
        go = O.adjoint_gradients(s.a, s.lam.real, s.lam.imag, zo, yo)
        _say("adjoint", s.lam, ainfo)
        assert rel(g["f"].cpu().numpy(), go["f"]) <= 1e-9
        assert rel(g["a"].cpu().numpy(), go["a"]) <= 1e-9
        assert g["alpha"].item() == pytest.approx(go["alpha"], rel=1e-9)
        assert g["beta"].item() == pytest.approx(go["beta"], rel=1e-9)


def test_autograd_function(csl):
    n = 15
    a = torch.tensor(WL.coef_c1(n), dtype=torch.float64, device="cuda", requires_grad=True)
    al = torch.tensor(-30.0, dtype=torch.float64, device="cuda", requires_grad=True)
    be = torch.tensor(45.0, dtype=torch.float64, device="cuda", requires_grad=True)
    f = cuda(_crand((n, n), 21)).requires_grad_(True)
    zt = cuda(_crand((n, n), 22))
    z = csl.solve(f, a, al, be, tol=1e-12)
    loss = (z - zt).abs().pow(2).sum()
    loss.backward()
    po = O.Problem(WL.coef_c1(n), -30.0, 45.0)
    zo = po.direct(_crand((n, n), 21))
    yo, _ = O.adjoint_solve(po, 2.0 * (zo - _crand((n, n), 22)), direct=True)
    go = O.adjoint_gradients(WL.coef_c1(n), -30.0, 45.0, zo, yo)
    assert rel(a.grad.cpu().numpy(), go["a"]) <= 1e-9
    assert rel(f.grad.cpu().numpy(), go["f"]) <= 1e-9
    assert al.grad.item() == pytest.approx(go["alpha"], rel=1e-9)
    assert be.grad.item() == pytest.approx(go["beta"], rel=1e-9)


@pytest.mark.parametrize("tile_elems", [256, 1024])
def test_small_tiles_long_lines(csl, tile_elems):
    # lines of 2048 (n = 1023) with small tiles: the twiddle staging for the
    # long lines must still get its LDS
    shape = (1023, 15)
    _say("small tiles long lines", tile_elems)
    a = _coef(shape, 21)
    x = _crand(shape, 22)
    p = csl.Problem(cuda(a), -10.0, 30.0, tile_elems=tile_elems)
    y = csl.apply_Pinv(p, cuda(x)).cpu().numpy()
    assert rel(y, O.apply_Pinv(x, p.abar, -10.0, 30.0)) <= 1e-13
    f = _crand(shape, 23)
    z, info = csl.minres_solve(p, cuda(f), raise_on_error=False, timeout_ms=30000)
    assert info["status"] == 0 and info["relres_true"] <= 1e-8


def test_batch_lds_budget_and_tuner(csl):
    # the same batch with 32 KiB and 64 KiB line budgets, then autotuned:
    # schedules change chunk sizes (summation order), not the method
    w = WL.workload("c4", count_override=8)
    probs = [csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=(j % 2 == 0))
             for j, s in enumerate(w.systems)]
    F = [cuda(s.f) for s in w.systems]
    _say("batch lds budgets")
    ref = None
    for lds in (0, 65536):
        b = csl.Batch(probs, lds_bytes=lds, timeout_ms=30000)
        zs, infos = b.solve(F)
        assert all(i["status"] == 0 and i["relres_true"] <= 1e-8 for i in infos), infos
        zc = [z.cpu().numpy() for z in zs]
        if ref is None:
            ref = zc
        else:
            for a_, b_ in zip(zc, ref):
                assert rel(a_, b_) <= 1e-9
        b.close()
    b = csl.Batch(probs, timeout_ms=30000)
    t = b.tune(F)
    _say("tuned", t)
    assert t["candidates"] >= 2 and t["lds_bytes"] in (32768, 65536) and t["tile_points"] > 0
    assert t["ms"] <= t["ms_default"] * 1.0000001
    zs, infos = b.solve(F)
    assert all(i["status"] == 0 and i["relres_true"] <= 1e-8 for i in infos), infos
    for z, r in zip(zs, ref):
        assert rel(z.cpu().numpy(), r) <= 1e-9
    # replays of the recaptured graph agree bitwise
    z1 = [z.cpu().numpy().copy() for z in zs]
    zs2, _ = b.solve(F)
    for a_, b_ in zip(z1, zs2):
        assert np.array_equal(a_, b_.cpu().numpy())
    with pytest.raises(csl.CSLError):
        csl.Batch(probs, lds_bytes=12345)


def test_problem_schedule_and_tuner(csl):
    # single-solve schedules change the tile grouping and the LDS budget
    # (summation order), not the method
    s = WL.workload("c2", n_override=255).systems[0]
    p = csl.Problem(cuda(s.a), s.lam.real, s.lam.imag)
    f = cuda(s.f)
    ref, info0 = csl.minres_solve(p, f)
    r0 = ref.cpu().numpy()
    for tp, lds in ((1, 0), (0, 65536), (4096, 0), (16384, 65536)):
        p.set_schedule(tp, lds)
        z, info = csl.minres_solve(p, f)
        assert info["status"] == 0 and abs(info["iters"] - info0["iters"]) <= 1
        assert rel(z.cpu().numpy(), r0) <= 1e-9
        y = csl.apply_Pinv(p, f).cpu().numpy()
        assert rel(y, O.apply_Pinv(s.f, p.abar, s.lam.real, s.lam.imag)) <= 1e-13
    t = p.tune(f)
    _say("problem tune", t)
    assert t["candidates"] >= 2 and t["ms"] <= t["ms_default"] * 1.0000001
    z, info = csl.minres_solve(p, f)
    assert info["status"] == 0 and rel(z.cpu().numpy(), r0) <= 1e-9
    with pytest.raises(csl.CSLError):
        p.set_schedule(0, 1000)
    with pytest.raises(csl.CSLError):
        p.set_schedule(0, 0, 384)


@pytest.mark.parametrize("fp32", [False, True])
def test_iterate_after_k_steps(csl, fp32):
    # stopping at every k exercises the paired w/x updates in all their
    # forms: a deferred step applied alone (odd k) or with its successor
    # (even k), against the oracle's iterate after exactly k steps
    s = WL.workload("c1", n_override=31).systems[0]
    p = csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=fp32)
    po = O.Problem(s.a, s.lam.real, s.lam.imag)
    f = cuda(s.f)
    for k in range(1, 8):
        z, info = csl.minres_solve(p, f, maxit=k, tol=1e-30, raise_on_error=False)
        assert info["iters"] == k and info["status_name"] == "ERR_NOT_CONVERGED", info
        zo, io = po.solve(s.f, fixed_iters=k)
        assert rel(z.cpu().numpy(), zo) <= (1e-6 if fp32 else 1e-12), k
        assert info["relres_est"] == pytest.approx(io["relres_est"], rel=1e-5 if fp32 else 1e-9)
