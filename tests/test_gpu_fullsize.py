"""GPU checks at the workloads' full sizes, in the configurations the bench
times, through properties the oracle can evaluate at any size:

- residuals ||f - (K + lambda I) z|| / ||f|| of the GPU solutions with the
  oracle's own K (a sparse matrix assembled face by face), against the tol;
- the GPU's reported relres against that oracle residual (same quantity);
- for the adjoint (16 shifts, n = 255, 65025 coefficient parameters):
  directional central differences of L = sum ||z_j - zt_j||^2 along random
  directions in a, alpha, beta and f, each difference from two GPU solves at
  tol 1e-12, against the adjoint gradients.

Tolerances: residual <= tol (1e-8); reported vs oracle residual within 5%
plus 1e-12 (two FP64 evaluations of a quantity of size 1e-8 with summation
errors of O(1e-16 ||f||)); finite differences: relative 1e-5 (central
difference truncation, of order step^2, and the solve noise 1e-12 / step,
about 1e-6 relative at a relative step of 1e-6).
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


def _oracle_relres(K, lam, f, z):
    r = np.ravel(f) - (K @ np.ravel(z) + lam * np.ravel(z))
    return float(np.linalg.norm(r) / np.linalg.norm(f))


def test_c3_full_size_fp32_and_fp64(csl):
    w = WL.workload("c3")
    s = w.systems[0]
    _say("c3 full", s.a.shape)
    K = O.build_K(s.a)
    for fp32 in (True, False):
        p = csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=fp32)
        z, info = csl.minres_solve(p, cuda(s.f), timeout_ms=60000)
        zc = z.cpu().numpy()
        rr = _oracle_relres(K, s.lam, s.f, zc)
        _say("c3", "fp32" if fp32 else "fp64", info, rr)
        assert info["status"] == 0
        assert rr <= 1e-8
        assert abs(info["relres_true"] - rr) <= 0.05 * rr + 1e-12


def test_c4_full_batch_residuals(csl):
    w = WL.workload("c4")
    probs = [csl.Problem(cuda(s.a), s.lam.real, s.lam.imag, pinv_fp32=True) for s in w.systems]
    F = [cuda(s.f) for s in w.systems]
    b = csl.Batch(probs, timeout_ms=60000)
    t = b.tune(F)
    _say("c4 schedule", t)
    zs, infos = b.solve(F)
    Ks = {}
    worst = 0.0
    for s, z, info in zip(w.systems, zs, infos):
        if s.n not in Ks:
            Ks[s.n] = O.build_K(s.a)
        rr = _oracle_relres(Ks[s.n], s.lam, s.f, z.cpu().numpy())
        assert info["status"] == 0 and rr <= 1e-8, (s.n, s.lam, info, rr)
        assert abs(info["relres_true"] - rr) <= 0.05 * rr + 1e-12
        worst = max(worst, rr)
    _say("c4 worst oracle relres", worst, "iterations", sorted({i["iters"] for i in infos}))


def test_c5_full_size_adjoint_directional_fd(csl):
    w = WL.workload("c5")
    a = w.systems[0].a
    n = a.shape[0]
    at = cuda(a)
    g = np.random.default_rng(55)
    tol = 1e-12

    def loss(a_dev, lams, fs):
        tot = 0.0
        for s, lam, f in zip(w.systems, lams, fs):
            p = csl.Problem(a_dev, lam.real, lam.imag)
            z, _ = csl.minres_solve(p, f, tol=tol, timeout_ms=60000)
            tot += float((z - cuda(s.z_target)).abs().pow(2).sum().item())
        return tot

    lams = [s.lam for s in w.systems]
    fs = [cuda(s.f) for s in w.systems]
    # adjoint gradients, summed over the 16 systems for a
    ga = torch.zeros_like(at)
    gf, galpha, gbeta = [], [], []
    for s in w.systems:
        p = csl.Problem(at, s.lam.real, s.lam.imag)
        z, _ = csl.minres_solve(p, cuda(s.f), tol=tol, timeout_ms=60000)
        G = 2.0 * (z - cuda(s.z_target))
        gr, _ = csl.minres_adjoint(p, z, G, tol=tol, ga=ga, timeout_ms=60000)
        gf.append(gr["f"])
        galpha.append(gr["alpha"].item())
        gbeta.append(gr["beta"].item())
    _say("c5 adjoint done", n, len(w.systems))
    h = 1e-6
    # direction in a: the adjoint gradient's own direction plus a random part.
    # A purely random direction in 65025 dimensions gives a derivative that
    # cancels down to the size of the finite-difference noise.
    gan = ga.cpu().numpy()
    rnd = g.standard_normal(a.shape)
    da = gan / np.linalg.norm(gan) + 0.5 * rnd / np.linalg.norm(rnd)
    da = da / np.linalg.norm(da) * np.linalg.norm(a)
    fd = (loss(cuda(a + h * da), lams, fs) - loss(cuda(a - h * da), lams, fs)) / (2 * h)
    an = float(torch.sum(ga * cuda(da)).item())
    _say("dL/da . d", fd, an)
    assert an == pytest.approx(fd, rel=1e-5)
    # alpha and beta of system 3, and a direction in f of system 7
    for j, kind in ((3, "alpha"), (3, "beta")):
        # only system j depends on its shift: difference its own loss term,
        # with a step relative to |lambda_j|
        hs = 1e-6 * abs(lams[j])
        dl = complex(hs, 0) if kind == "alpha" else complex(0, hs)
        sj = w.systems[j]

        def lj(lam):
            p = csl.Problem(at, lam.real, lam.imag)
            z, _ = csl.minres_solve(p, fs[j], tol=tol, timeout_ms=60000)
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
        z, _ = csl.minres_solve(p, cuda(f), tol=tol, timeout_ms=60000)
        return float((z - cuda(sj.z_target)).abs().pow(2).sum().item())

    fdf = (lf(sj.f + h * df) - lf(sj.f - h * df)) / (2 * h)
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
    # printed 14 at every n, every solution meets the tolerance under the
    # oracle's K, and at n = 63 the count equals the oracle's within one step.
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
                _, io = O.Problem(a, alpha, beta, abar_rule="given", abar=p.abar).solve(f)
                assert abs(io["iters"] - info["iters"]) <= 1, (io["iters"], info)
            its.append(info["iters"])
            p.close()
        assert its == [gold["iterations"]] * 3, (lam, its)


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
