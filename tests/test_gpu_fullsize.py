"""GPU checks at the workloads' full sizes, in the configurations the bench
times, against the CPU oracle:

- the 3-D n = 127 system (FP64 and FP32 preconditioner) and all 64 systems
  of the batched-shift workload: the GPU iterate element by element against
  the oracle's MINRES iterate after the same number of steps, with the
  oracle taking its own abar; and the residual ||f - (K + lambda I) z|| / ||f||
  of the GPU solution under the oracle's K against the tolerance;
- the adjoint workload (16 shifts, n = 255, 65025 coefficient parameters):
  the GPU gradients of four systems element by element against the oracle's
  gradients from direct solves; the directional derivative along a random
  direction in a of L = sum ||z_j - zt_j||^2 against central differences of
  the oracle's direct solves (step 1e-5); and directional derivatives in
  alpha, beta and f against central differences of GPU solves at tol 1e-12.

Tolerances: iterates against the oracle after the same number of steps,
1e-10 with the FP64 preconditioner (the target is 1e-8) and 1e-6 with the
FP32 one; residual <= tol (1e-8); reported vs oracle residual within 5% plus
1e-12 (two FP64 evaluations of a quantity of size 1e-8 with summation errors
of O(1e-16 ||f||)); gradients against the direct-solve ones 1e-9 (the GPU
solves run at tol 1e-13); finite differences relative 1e-5.
"""
import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import csl_oracle as O
from paper_2408_00488_amd import workloads as WL

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


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
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _oracle_relres(K, lam, f, z):
    r = np.ravel(f) - (K @ np.ravel(z) + lam * np.ravel(z))
    return float(np.linalg.norm(r) / np.linalg.norm(f))


def _vs_oracle_iterate(po, f, zg, info, zo, io):
    """Relative difference of the GPU iterate from the oracle's after the
    GPU's number of steps (the oracle's own run when the counts agree)."""
    if info["iters"] == io["iters"]:
        return rel(zg, zo)
    zf, _ = po.solve(f, fixed_iters=info["iters"])
    return rel(zg, zf)


@pytest.mark.timeout(900)
def test_c3_full_size_fp32_and_fp64(csl):
    w = WL.workload("c3")
    s = w.systems[0]
    _say("c3 full", s.a.shape)
    po = O.Problem(s.a, s.lam.real, s.lam.imag)
    zo, io = po.solve(s.f)
    _say("c3 oracle", io["iters"], io["relres_true"])
    for fp32 in (True, False):
        p = csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=fp32)
        assert p.abar == pytest.approx(po.abar, rel=1e-14)
        z, info = csl.minres_solve(p, cuda(s.f), timeout_ms=60000)
        zc = z.cpu().numpy()
        rr = _oracle_relres(po.K, s.lam, s.f, zc)
        e = _vs_oracle_iterate(po, s.f, zc, info, zo, io)
        _say("c3", "fp32" if fp32 else "fp64", info, "oracle relres", rr, "vs oracle", e)
        assert info["status"] == 0
        assert rr <= 1e-8
        assert abs(info["relres_true"] - rr) <= 0.05 * rr + 1e-12
        assert abs(info["iters"] - io["iters"]) <= (2 if fp32 else 1)
        assert e <= (1e-6 if fp32 else 1e-10)
        p.close()


@pytest.mark.timeout(900)
def test_c4_full_batch_vs_oracle(csl):
    w = WL.workload("c4")
    probs = [csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=True) for s in w.systems]
    F = [cuda(s.f) for s in w.systems]
    b = csl.Batch(probs, timeout_ms=60000)
    t = b.tune(F)
    _say("c4 schedule", t)
    zs, infos = b.solve(F)
    worst_rr, worst_e = 0.0, 0.0
    for j, (s, p, z, info) in enumerate(zip(w.systems, probs, zs, infos)):
        po = O.Problem(s.a, s.lam.real, s.lam.imag)
        assert p.abar == pytest.approx(po.abar, rel=1e-14)
        zo, io = po.solve(s.f)
        zc = z.cpu().numpy()
        rr = _oracle_relres(po.K, s.lam, s.f, zc)
        e = _vs_oracle_iterate(po, s.f, zc, info, zo, io)
        assert info["status"] == 0 and rr <= 1e-8, (j, s.n, s.lam, info, rr)
        assert abs(info["relres_true"] - rr) <= 0.05 * rr + 1e-12
        assert abs(info["iters"] - io["iters"]) <= 2, (j, info, io["iters"])
        assert e <= 1e-6, (j, s.n, e)
        worst_rr, worst_e = max(worst_rr, rr), max(worst_e, e)
        if j % 8 == 7:
            _say("c4 systems", j + 1, "worst oracle relres", worst_rr, "worst vs oracle", worst_e)
    _say("c4 iterations", sorted({i["iters"] for i in infos}))


def _c5_direct_loss_difference(w, ap, am):
    """L(a+) - L(a-) for L = sum_j ||z_j - zt_j||^2 with the oracle's direct
    solves, summed as sum_j Re<z+ - z-, z+ + z- - 2 zt> (the same number as the
    difference of the two losses, without the cancellation of the large
    ||zt||^2 terms)."""
    tot = 0.0
    for s in w.systems:
        zp = O.Problem(ap, s.lam.real, s.lam.imag).direct(s.f)
        zm = O.Problem(am, s.lam.real, s.lam.imag).direct(s.f)
        tot += float(np.real(np.vdot(zp - zm, zp + zm - 2.0 * s.z_target)))
    return tot


@pytest.mark.timeout(900)
def test_c5_full_size_adjoint(csl):
    w = WL.workload("c5")
    a = w.systems[0].a
    n = a.shape[0]
    at = cuda(a)
    g = np.random.default_rng(55)
    tol = 1e-13
    lams = [s.lam for s in w.systems]
    fs = [cuda(s.f) for s in w.systems]
    # adjoint gradients: summed over the 16 systems for a, and per system for
    # the four compared with the oracle one by one
    ga = torch.zeros_like(at)
    gf, galpha, gbeta, ga_each = [], [], [], []
    for j, s in enumerate(w.systems):
        p = csl.Problem(at, s.lam.real, s.lam.imag)
        z, _ = csl.minres_solve(p, cuda(s.f), tol=tol, timeout_ms=60000)
        G = 2.0 * (z - cuda(s.z_target))
        gaj = torch.zeros_like(at)
        gr, _ = csl.minres_adjoint(p, z, G, tol=tol, ga=gaj, timeout_ms=60000)
        ga += gaj
        ga_each.append(gaj.cpu().numpy() if j < 4 else None)
        gf.append(gr["f"])
        galpha.append(gr["alpha"].item())
        gbeta.append(gr["beta"].item())
        p.close()
    _say("c5 adjoint done", n, len(w.systems))
    # the first four systems against the oracle's gradients from direct solves
    for j in range(4):
        s = w.systems[j]
        po = O.Problem(a, s.lam.real, s.lam.imag)
        zd = po.direct(s.f)
        yd, _ = O.adjoint_solve(po, 2.0 * (zd - s.z_target), direct=True)
        go = O.adjoint_gradients(a, s.lam.real, s.lam.imag, zd, yd)
        ef, ea = rel(gf[j].cpu().numpy(), go["f"]), rel(ga_each[j], go["a"])
        _say("c5 system", j, "grad f", ef, "grad a", ea, "alpha", galpha[j], go["alpha"],
             "beta", gbeta[j], go["beta"])
        assert ef <= 1e-9 and ea <= 1e-9
        assert galpha[j] == pytest.approx(go["alpha"], rel=1e-9)
        assert gbeta[j] == pytest.approx(go["beta"], rel=1e-9)
    # a random direction in a: central differences of the oracle's direct
    # solves against the summed adjoint gradient
    h = 1e-5
    da = g.standard_normal(a.shape)
    da = da / np.linalg.norm(da) * np.linalg.norm(a)
    fd = _c5_direct_loss_difference(w, a + h * da, a - h * da) / (2 * h)
    an = float(torch.sum(ga * cuda(da)).item())
    _say("dL/da . d (random): fd", fd, "adjoint", an)
    assert an == pytest.approx(fd, rel=1e-5)
    # alpha and beta of system 3, and a direction in f of system 7, by central
    # differences of GPU solves
    hg = 1e-6
    for j, kind in ((3, "alpha"), (3, "beta")):
        # only system j depends on its shift: difference its own loss term,
        # with a step relative to |lambda_j|
        hs = hg * abs(lams[j])
        dl = complex(hs, 0) if kind == "alpha" else complex(0, hs)
        sj = w.systems[j]

        def lj(lam):
            p = csl.Problem(at, lam.real, lam.imag)
            z, _ = csl.minres_solve(p, fs[j], tol=1e-12, timeout_ms=60000)
            return float((z - cuda(sj.z_target)).abs().pow(2).sum().item())

        fdj = (lj(lams[j] + dl) - lj(lams[j] - dl)) / (2 * hs)
        anj = galpha[j] if kind == "alpha" else gbeta[j]
        _say(kind, j, fdj, anj)
        assert anj == pytest.approx(fdj, rel=1e-5)
    j = 7
    sj = w.systems[j]
    df = g.standard_normal(sj.f.shape) + 1j * g.standard_normal(sj.f.shape)
    df = df / np.linalg.norm(df) * np.linalg.norm(sj.f)

    def lf(f):
        p = csl.Problem(at, sj.lam.real, sj.lam.imag)
        z, _ = csl.minres_solve(p, cuda(f), tol=1e-12, timeout_ms=60000)
        return float((z - cuda(sj.z_target)).abs().pow(2).sum().item())

    fdf = (lf(sj.f + hg * df) - lf(sj.f - hg * df)) / (2 * hg)
    # torch convention: dL/d(Re f) + i dL/d(Im f); directional derivative = Re <grad, df>
    anf = float(np.real(np.vdot(gf[j].cpu().numpy(), df)))
    _say("dL/df . d", fdf, anf)
    assert anf == pytest.approx(fdf, rel=1e-5)


def _crand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def test_iterations_flat_in_n_table2a(csl):
    # Theorem 4 at the sizes of Table 2(a) that the grid rules admit (n = 63,
    # 255, 1023), Example 2's coefficient on the unit square and the
    # geometric-mean abar: for each of the table's shifts the GPU count is the
    # printed 14 at n = 255 and 1023, and at n = 63 (where the count depends
    # on the random right-hand side: 14 for most seeds, 12 for some) it is 12
    # or 14 and equals the oracle's within one step; every solution meets the
    # tolerance under the oracle's K.
    gold = json.load(open(os.path.join(GOLD, "table2a_iterations.json")))
    for alpha, beta in gold["shifts_alpha_beta"]:
        lam = complex(alpha, beta)
        its = []
        for n in (63, 255, 1023):
            a = WL.coef_paper_ex2(n)
            f = _crand((n, n), 7)
            p = csl.Problem(cuda(a), alpha, beta, abar_rule="geomean")
            z, info = csl.minres_solve(p, cuda(f), timeout_ms=60000)
            zc = z.cpu().numpy()
            rr = _oracle_relres(O.build_K(a), lam, f, zc)
            _say("table 2(a)", lam, n, info["iters"], rr)
            assert info["status"] == 0 and rr <= 1e-8
            if n == 63:
                _, io = O.Problem(a, alpha, beta, abar_rule="geomean").solve(f)
                assert abs(io["iters"] - info["iters"]) <= 1, (io["iters"], info)
            its.append(info["iters"])
            p.close()
        assert its[1:] == [gold["iterations"]] * 2, (lam, its)
        assert its[0] in (gold["iterations"] - 2, gold["iterations"]), (lam, its)


def test_iterations_flat_in_n_3d(csl):
    # the same property in 3-D on the c3 coefficient and shift, n = 15 .. 127,
    # with the FP32 preconditioner
    lam = complex(10.0, 100.0)
    its = []
    for n in (15, 31, 63, 127):
        a = WL.coef_c3(n)
        f = _crand((n, n, n), 9)
        p = csl.Problem(cuda(a), lam.real, lam.imag, pinv_fp32=True)
        z, info = csl.minres_solve(p, cuda(f), timeout_ms=60000)
        rr = _oracle_relres(O.build_K(a), lam, f, z.cpu().numpy())
        _say("3-D", n, info["iters"], rr)
        assert info["status"] == 0 and rr <= 1e-8
        its.append(info["iters"])
        p.close()
    assert max(its) - min(its) <= 2, its
