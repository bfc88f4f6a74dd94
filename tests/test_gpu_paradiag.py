"""GPU parity of the alpha-circulant all-at-once layer (paradiag_*) against
the oracle, through the C ABI.

- The step transform (alpha^(k/L) scaling and the DFT over the L steps, and
  its inverse) element by element against the oracle's: relative 1e-13 (an
  FP64 FFT of length <= 1024 and one exp per step), on point counts that
  leave a ragged last workgroup.
- The shifts D_j against the oracle's closed form: relative 1e-14.
- The solve against a direct solve of kron(C, I) + kron(I, K) on small
  grids: with every mode at tolerance tol, the all-at-once residual is at
  most tol times cond(Gamma) = alpha^(-(L-1)/L) (the transform is unitary
  up to the Gamma scaling), and the error at most that times the modes'
  condition; checked as a residual bound and as a solution bound.
- Per mode, the GPU iteration counts within one of the oracle's MINRES.
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


@pytest.mark.parametrize("L,shape,alpha_c", [(8, (7, 7), 0.1), (64, (63, 63), 1e-2),
                                             (1024, (15, 31), 0.5), (16, (7, 15, 7), 1.0)])
def test_step_transform_and_shifts(csl, L, shape, alpha_c):
    _say("step transform", L, shape, alpha_c)
    tau = 0.05
    pd = csl.ParaDiag(cuda(_coef(shape, 1)), L, tau, alpha_c, dst="fft")
    x = _crand((L,) + shape, 2)
    y = pd.transform(cuda(x)).cpu().numpy()
    assert rel(y, O.paradiag_forward(x, alpha_c)) <= 1e-13
    xi = pd.transform(cuda(x), inverse=True).cpu().numpy()
    assert rel(xi, O.paradiag_inverse(x, alpha_c)) <= 1e-13
    back = pd.transform(cuda(y), inverse=True).cpu().numpy()
    assert rel(back, x) <= 1e-13
    D = O.alpha_circulant_shifts(L, tau, alpha_c)
    assert rel(np.array(pd.shifts), D) <= 1e-14
    pd.close()


@pytest.mark.parametrize("shape,L,alpha_c,fp32", [((15, 15), 8, 0.1, False),
                                                  ((7, 7, 7), 16, 0.05, False),
                                                  ((31, 31), 32, 1e-2, True),
                                                  ((20, 31), 8, 0.1, False)])
def test_paradiag_solve_against_all_at_once(csl, shape, L, alpha_c, fp32):
    _say("paradiag solve", shape, L, alpha_c, fp32)
    tau = 0.02
    a = _coef(shape, 3)
    R = _crand((L,) + shape, 4)
    tol = 1e-10
    pd = csl.ParaDiag(cuda(a), L, tau, alpha_c, pinv_fp32=fp32, tol=tol, timeout_ms=30000)
    U, infos = pd.solve(cuda(R))
    U = U.cpu().numpy()
    assert all(i["status"] == 0 for i in infos)
    A = O.all_at_once_matrix(O.build_K(a), L, tau, alpha_c)
    cond_gamma = alpha_c ** (-(L - 1) / L)
    res = np.linalg.norm(R.ravel() - A @ U.ravel()) / np.linalg.norm(R)
    _say("all-at-once residual", res, "bound", tol * cond_gamma)
    assert res <= 1.01 * tol * cond_gamma
    Ud, _ = O.paradiag_solve(a, L, tau, alpha_c, R)
    err = rel(U, Ud)
    _say("error against the direct solve", err)
    assert err <= 1e-6
    # per mode: the same MINRES as the oracle's, within one iteration
    if not fp32:
        _, io = O.paradiag_solve(a, L, tau, alpha_c, R, direct=False, tol=tol)
        for j, (gi, oi) in enumerate(zip(infos, io)):
            assert abs(gi["iters"] - oi["iters"]) <= 1, (j, gi, oi["iters"])
    # graph replays repeat the result bitwise
    U2, infos2 = pd.solve(cuda(R))
    assert infos2 == infos and np.array_equal(U2.cpu().numpy(), U)
    pd.close()


def test_paradiag_bench_size_residual_and_tuner(csl):
    # the measured configuration: 64 steps on a 2-D n = 255 grid, FP32
    # preconditioner, tol 1e-8
    n, L, tau, alpha_c = 255, 64, 1.0 / 64, 1e-2
    x = (np.arange(1, n + 1) / (n + 1.0))
    a = 1.0 + 0.5 * np.sin(2 * np.pi * x)[:, None] * np.sin(2 * np.pi * x)[None, :]
    R = _crand((L, n, n), 5)
    pd = csl.ParaDiag(cuda(a), L, tau, alpha_c, pinv_fp32=True, timeout_ms=60000)
    sched = pd.tune(cuda(R))
    assert sched["candidates"] >= 2
    U, infos = pd.solve(cuda(R))
    assert all(i["status"] == 0 for i in infos)
    its = [i["iters"] for i in infos]
    _say("bench-size modes: iterations", min(its), max(its))
    A = O.all_at_once_matrix(O.build_K(a), L, tau, alpha_c)
    Uc = U.cpu().numpy()
    res = np.linalg.norm(R.ravel() - A @ Uc.ravel()) / np.linalg.norm(R)
    _say("all-at-once residual", res)
    assert res <= 1.01 * 1e-8 * alpha_c ** (-(L - 1) / L)
    pd.close()


def test_paradiag_argument_checks(csl):
    a = cuda(_coef((7, 7), 6))
    for kw in (dict(steps=12, tau=0.1, alpha_c=0.1), dict(steps=4, tau=0.1, alpha_c=0.1),
               dict(steps=8, tau=0.0, alpha_c=0.1), dict(steps=8, tau=0.1, alpha_c=0.0),
               dict(steps=8, tau=0.1, alpha_c=1.5)):
        with pytest.raises(csl.CSLError, match="ERR_ARG"):
            csl.ParaDiag(a, **kw)
    pd = csl.ParaDiag(a, 8, 0.1, 0.1)
    r = cuda(_crand((8, 7, 7), 7))
    with pytest.raises(csl.CSLError, match="ERR_ARG"):
        pd.solve(r, u=r)
    with pytest.raises(ValueError):
        pd.solve(cuda(_crand((4, 7, 7), 7)))
    pd.close()
