"""Pins of the CPU oracle against facts fixed by the paper and by
mathematics (closed forms, dense linear algebra, brute force, the paper's
theorems and tables).  None of these re-types the oracle's own formula."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import csl_oracle as O
from paper_2408_00488_amd import workloads as WL

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_coef(shape, seed, lo=0.5, hi=2.0):
    g = np.random.default_rng(seed)
    return g.uniform(lo, hi, shape)


def _crand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


# ---------------------------------------------------------------- sine transform

@pytest.mark.parametrize("n", [1, 3, 7, 15, 31, 12, 100])
def test_dst_equals_dense_sine_matrix(n):
    # Section 2.3: W is the real symmetric orthogonal DST matrix.
    j = np.arange(1, n + 1)
    W = np.array([[math.sqrt(2.0 / (n + 1)) * math.sin(math.pi * p * q / (n + 1))
                   for q in j] for p in j])
    x = _crand(n, n)
    assert np.allclose(O.dst1(x), W @ x, atol=1e-13, rtol=0)
    assert np.allclose(W, W.T, atol=0)
    assert np.allclose(W @ W, np.eye(n), atol=1e-13)


@pytest.mark.parametrize("n", [3, 4, 12, 45, 200])
def test_dst_row_reflection(n):
    # The DST-I matrix satisfies W[n-1-m][k] = (-1)^k W[m][k] (0-based): the
    # even-k and odd-k partial sums E, O of row m give the transform at m
    # (E + O) and at n-1-m (E - O).  Brute-force sums, checked against the
    # oracle's DST.
    x = _crand(n, 3 * n)
    c = math.sqrt(2.0 / (n + 1))
    y = O.dst1(x)
    for m in range((n + 1) // 2):
        E = sum(c * math.sin(math.pi * (m + 1) * (k + 1) / (n + 1)) * x[k] for k in range(0, n, 2))
        Od = sum(c * math.sin(math.pi * (m + 1) * (k + 1) / (n + 1)) * x[k] for k in range(1, n, 2))
        assert abs(y[m] - (E + Od)) <= 1e-12
        assert abs(y[n - 1 - m] - (E - Od)) <= 1e-12


@pytest.mark.parametrize("n", [3, 7, 16, 31, 45])
def test_mu_closed_form_and_diagonalisation(n):
    # Section 2.3: W L W = Lambda with positive diagonal.
    h = 1.0 / (n + 1)
    L1 = O.laplacian_1d(n, h)
    mu = O.mu_1d(n, h)
    assert np.allclose(np.sort(mu), np.linalg.eigvalsh(L1), rtol=1e-12)
    W = O.sine_matrix(n)
    assert np.allclose(W @ L1 @ W, np.diag(mu), atol=1e-9 * mu.max())
    assert (mu > 0).all()


def test_dst_multiaxis_is_kronecker():
    x = _crand((5, 7, 3), 1)
    W0, W1, W2 = O.sine_matrix(5), O.sine_matrix(7), O.sine_matrix(3)
    ref = np.einsum("ia,jb,kc,abc->ijk", W0, W1, W2, x)
    assert np.allclose(O.dst1(x), ref, atol=1e-13)


# ---------------------------------------------------------------- stencil K

def _K_brute(a, lengths=None):
    """Pure-Python node-by-node assembly from the stencil definition."""
    shape = a.shape
    d = a.ndim
    hs = [(1.0 if lengths is None else lengths[k]) / (shape[k] + 1) for k in range(d)]
    M = a.size
    K = np.zeros((M, M))
    for p in np.ndindex(shape):
        ip = np.ravel_multi_index(p, shape)
        for ax in range(d):
            for step in (-1, 1):
                q = list(p)
                q[ax] += step
                if 0 <= q[ax] < shape[ax]:
                    aq = a[tuple(q)]
                    c = 2 * a[p] * aq / (a[p] + aq)
                    iq = np.ravel_multi_index(tuple(q), shape)
                    K[ip, iq] -= c / hs[ax] ** 2
                else:
                    c = a[p]
                K[ip, ip] += c / hs[ax] ** 2
    return K


@pytest.mark.parametrize("shape", [(4, 5), (3, 4, 5), (6,)])
def test_K_matches_brute_force(shape):
    a = _rand_coef(shape, 3)
    lengths = [1.0 + 0.25 * k for k in range(len(shape))]
    assert np.allclose(O.build_K(a, lengths).toarray(), _K_brute(a, lengths),
                       rtol=1e-13, atol=0)


@pytest.mark.parametrize("n", [5, 8])
def test_K_constant_is_textbook_laplacian(n):
    h = 1.0 / (n + 1)
    T = O.laplacian_1d(n, h)
    I = np.eye(n)
    L2 = np.kron(T, I) + np.kron(I, T)
    assert np.allclose(O.build_K(np.ones((n, n))).toarray(), L2, rtol=1e-14)
    L3 = np.kron(np.kron(T, I), I) + np.kron(np.kron(I, T), I) + np.kron(np.kron(I, I), T)
    assert np.allclose(O.build_K(np.ones((n, n, n))).toarray(), L3, rtol=1e-14)


@pytest.mark.parametrize("shape", [(7, 7), (5, 6, 4)])
def test_lemma3_bounds(shape):
    # Lemma 3 (i): a_min L <= K <= a_max L ; (ii) L >= c0 I.
    a = _rand_coef(shape, 7)
    K = O.build_K(a).toarray()
    L = O.build_K(np.ones(shape)).toarray()
    amin, amax = O.coefficient_bounds(a)
    assert np.allclose(K, K.T)
    tol = 1e-10 * np.abs(K).max()
    assert np.linalg.eigvalsh(K - amin * L).min() >= -tol
    assert np.linalg.eigvalsh(amax * L - K).min() >= -tol
    c0 = O.mode_eigenvalues(shape).min()
    assert np.linalg.eigvalsh(L).min() == pytest.approx(c0, rel=1e-10)


# ---------------------------------------------------------------- block form

def test_apply_A_matches_block_matrix_and_complex_system():
    n = 6
    a = _rand_coef((n, n), 11)
    K = O.build_K(a)
    alpha, beta = -30.0, 12.5
    x = _crand((n, n), 12)
    B = O.block_matrix(K, alpha, beta)
    y = O.apply_A(K, alpha, beta, x)
    assert np.allclose(O.to_block(y), B @ O.to_block(x), rtol=1e-14, atol=1e-10)
    # symmetric: <x, A y> = <A x, y>
    x2 = _crand((n, n), 13)
    assert O.rdot(x, O.apply_A(K, alpha, beta, x2)) == pytest.approx(
        O.rdot(O.apply_A(K, alpha, beta, x), x2), rel=1e-12)
    # unknown [Re z; -Im z] with rhs [Re f; Im f] solves (K + lambda I) z = f
    f = _crand((n, n), 14)
    Kc = (K + complex(alpha, beta) * sp.identity(n * n)).toarray()
    z = np.linalg.solve(Kc, f.ravel())
    u = np.concatenate([z.real, -z.imag])
    assert np.allclose(B @ u, O.to_block(f), atol=1e-9)


def test_paper_printed_orientation_reading():
    # Eq. (2) as printed maps [z1; z2] to [Im f; Re f] (so its printed rhs
    # [a; b] is swapped); its square equals ours, so |A| (Eq. (3)) agrees.
    n = 4
    a = _rand_coef((n, n), 21)
    K = O.build_K(a)
    alpha, beta = 5.0, -3.0
    f = _crand((n, n), 22)
    Kc = (K + complex(alpha, beta) * sp.identity(n * n)).toarray()
    z = np.linalg.solve(Kc, f.ravel())
    Bp = O.paper_block_matrix(K, alpha, beta).toarray()
    out = Bp @ np.concatenate([z.real, z.imag])
    assert np.allclose(out, np.concatenate([f.ravel().imag, f.ravel().real]), atol=1e-9)
    Bn = O.block_matrix(K, alpha, beta).toarray()
    assert np.allclose(Bp @ Bp, Bn @ Bn, atol=1e-8)


# ---------------------------------------------------------------- preconditioner

@pytest.mark.parametrize("shape,lengths", [((7, 7), None), ((3, 7, 5), [1.0, 2.0, 0.5])])
def test_pinv_matches_dense_eigendecomposition(shape, lengths):
    abar, alpha, beta = 1.3, -40.0, 7.0
    x = _crand(shape, 31)
    Pd = O.dense_Pinv(shape, abar, alpha, beta, lengths)
    ref = (Pd @ x.ravel().real) + 1j * (Pd @ x.ravel().imag)
    got = O.apply_Pinv(x, abar, alpha, beta, lengths)
    assert np.allclose(got.ravel(), ref, rtol=1e-11, atol=1e-14 * np.abs(ref).max())


def test_ideal_preconditioner_is_absolute_value():
    # Eq. (3): |A| = blkdiag(sqrt(S^2 + beta^2 I)) twice.
    n = 4
    K = O.build_K(_rand_coef((n, n), 41))
    alpha, beta = -20.0, 3.0
    B = O.block_matrix(K, alpha, beta).toarray()
    S = (K + alpha * sp.identity(n * n)).toarray()
    Q = O.sqrtm_spd(S @ S + beta ** 2 * np.eye(n * n))
    ref = sla.block_diag(Q, Q)
    assert np.allclose(O.absm(B), ref, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("alpha,beta", WL.paper_shifts_table1())
def test_theorem1_eigenvalues_pm1(alpha, beta):
    # Theorem 1: for constant a, |A|^{-1} A is Hermitian and unitary (eig +-1).
    n = 5
    K = O.build_K(np.ones((n, n)))
    B = O.block_matrix(K, alpha, beta).toarray()
    Ainv_abs = np.linalg.inv(O.absm(B))
    C = Ainv_abs @ B
    assert np.allclose(C, C.T, atol=1e-10)
    assert np.allclose(C @ C, np.eye(2 * n * n), atol=1e-10)
    ev = np.linalg.eigvalsh((C + C.T) / 2)
    assert np.allclose(np.abs(ev), 1.0, atol=1e-10)


# ---------------------------------------------------------------- MINRES

def test_minres_iterates_minimise_preconditioned_residual():
    # Brute force: x_k = argmin_{x in K_k(P^{-1}A, P^{-1}b)} ||b - A x||_{P^{-1}},
    # and |eta_k| equals that minimum.
    shape = (5, 4)
    a = _rand_coef(shape, 51)
    prob = O.Problem(a, alpha=-60.0, beta=9.0)
    f = _crand(shape, 52)
    _, info = prob.solve(f, fixed_iters=7, record=True)
    M = a.size
    B = O.block_matrix(prob.K, prob.alpha, prob.beta).toarray()
    Pi = O.dense_Pinv(shape, prob.abar, prob.alpha, prob.beta)
    Pinv_block = sla.block_diag(Pi, Pi)
    b = O.to_block(f)
    Rp = O.sqrtm_spd(Pinv_block)          # P^{-1/2}
    basis = [Pinv_block @ b]
    for k in range(1, 8):
        V = np.array(basis).T
        Qb, _ = np.linalg.qr(V)
        coef, *_ = np.linalg.lstsq(Rp @ B @ Qb, Rp @ b, rcond=None)
        xk = Qb @ coef
        got = O.to_block(info["history"][k - 1])
        assert np.allclose(got, xk, atol=1e-8 * np.abs(xk).max()), k
        r = b - B @ xk
        assert abs(info["eta"][k - 1]) == pytest.approx(math.sqrt(r @ Pinv_block @ r), rel=1e-8)
        basis.append(Pinv_block @ (B @ basis[-1]))
    assert M == 20


@pytest.mark.parametrize("n", [7, 15, 31])
def test_minres_converges_to_direct_solution(n):
    a = WL.coef_c1(n)
    prob = O.Problem(a, 1.0, 1.0)
    f = _crand((n, n), n)
    z, info = prob.solve(f, tol=1e-12)
    zd = prob.direct(f)
    assert info["status"] == O.STATUS_OK
    assert np.linalg.norm(z - zd) / np.linalg.norm(zd) < 1e-9
    assert info["relres_true"] <= 1e-12


def test_minres_paper_style_known_solution():
    # Section 3 draws the exact solution and forms f from it.
    n = 15
    prob = O.Problem(WL.coef_paper_ex2(n), -100.0, 100.0, abar_rule="geomean")
    zs = _crand((n, n), 99)
    f = (prob.K @ zs.ravel() + complex(-100.0, 100.0) * zs.ravel()).reshape(n, n)
    z, info = prob.solve(f, tol=1e-10)
    assert np.linalg.norm(z - zs) / np.linalg.norm(zs) < 1e-8


def test_table1a_two_iterations():
    gold = json.load(open(os.path.join(GOLD, "table1a_iterations.json")))
    for n in (7, 15, 31, 63):
        for alpha, beta in gold["shifts_alpha_beta"]:
            prob = O.Problem(np.ones((n, n)), alpha, beta)
            f = _crand((n, n), abs(n * 1000 + int(alpha) * 7 + int(beta)))
            z, info = prob.solve(f, tol=1e-8)
            assert info["iters"] == gold["iterations"], (n, alpha, beta, info["iters"])
            zd = prob.direct(f)
            assert np.linalg.norm(z - zd) / np.linalg.norm(zd) < 1e-11


@pytest.mark.parametrize("alpha,beta", [(100.0, 100.0), (1.0, -100.0), (30.0, 5.0)])
def test_theorem3_spectrum_bounds_alpha_nonneg(alpha, beta):
    for n in (7, 15):
        a = WL.coef_paper_ex2(n)
        prob = O.Problem(a, alpha, beta, abar_rule="geomean")
        B = O.block_matrix(prob.K, alpha, beta).toarray()
        P = np.linalg.inv(O.dense_Pinv(a.shape, prob.abar, alpha, beta))
        Pb = sla.block_diag(P, P)
        ev = np.abs(sla.eigh(B, Pb, eigvals_only=True))
        amin, amax = O.coefficient_bounds(a)
        lo, hi = O.theorem3_bounds(amin, amax, O.mode_eigenvalues(a.shape).min(), alpha, beta)
        assert ev.min() >= lo * (1 - 1e-9) and ev.max() <= hi * (1 + 1e-9)


def test_theorem3_alpha_negative_and_n_independence():
    alpha, beta = -100.0, 100.0
    spans = []
    for n in (7, 15, 31):
        a = WL.coef_c1(n)
        prob = O.Problem(a, alpha, beta, abar_rule="geomean")
        B = O.block_matrix(prob.K, alpha, beta).toarray()
        P = np.linalg.inv(O.dense_Pinv(a.shape, prob.abar, alpha, beta))
        ev = np.abs(sla.eigh(B, sla.block_diag(P, P), eigvals_only=True))
        amin, amax = O.coefficient_bounds(a)
        c0 = O.mode_eigenvalues(a.shape).min()
        assert amin * c0 + abs(beta) + alpha > 0          # Theorem 3 (ii) applies
        lo, hi = O.theorem3_bounds(amin, amax, c0, alpha, beta)
        assert ev.min() >= lo * (1 - 1e-9) and ev.max() <= hi * (1 + 1e-9)
        spans.append((ev.min(), ev.max()))
    # bounded independently of n: the extreme |eigenvalues| barely move
    mins = [s[0] for s in spans]
    maxs = [s[1] for s in spans]
    assert max(maxs) / min(maxs) < 1.2 and max(mins) / min(mins) < 1.2


def test_lemma1_bound_holds():
    # Lemma 1 with the symmetric interval [-a, -b] U [b, a] from the actual
    # spectrum; the residual measured in the norm MINRES minimises.
    n = 7
    a = WL.coef_c1(n)
    prob = O.Problem(a, 20.0, 40.0)
    B = O.block_matrix(prob.K, 20.0, 40.0).toarray()
    P = np.linalg.inv(O.dense_Pinv(a.shape, prob.abar, 20.0, 40.0))
    ev = np.abs(sla.eigh(B, sla.block_diag(P, P), eigvals_only=True))
    hi, lo = ev.max(), ev.min()
    f = _crand((n, n), 5)
    _, info = prob.solve(f, fixed_iters=20, record=True)
    eta0 = math.sqrt(O.rdot(f, prob.Pinv(f)))
    for k, eta in enumerate(info["eta"], start=1):
        assert abs(eta) / eta0 <= O.lemma1_bound(hi, lo, lo, hi, k) * (1 + 1e-8) + 1e-13


def test_theorem4_iterations_flat_in_n():
    # Theorem 4 / Table 2(a): the count does not grow with n, and at the
    # table's size n = 255 (unit square, the reading of the unstated domain)
    # it is the printed 14 for every shift and every right-hand side tried.
    # At n = 63 the count depends on the random right-hand side (the paper's
    # own is not reproducible): 14 for most draws, 12 for some (seed 3), so
    # there the pin is 14 for a majority of eight seeds and nothing outside
    # {12, 14}.
    gold = json.load(open(os.path.join(GOLD, "table2a_iterations.json")))
    for alpha, beta in gold["shifts_alpha_beta"]:
        its = {}
        for n in (15, 31, 63, 255):
            prob = O.Problem(WL.coef_paper_ex2(n), alpha, beta, abar_rule="geomean")
            seeds = range(8) if n == 63 else (range(2) if n == 255 else (7,))
            its[n] = []
            for seed in seeds:
                _, info = prob.solve(_crand((n, n), seed), tol=1e-8)
                assert info["status"] == O.STATUS_OK
                its[n].append(info["iters"])
        flat = [k for v in its.values() for k in v]
        assert max(flat) - min(flat) <= 2, its
        assert all(k == gold["iterations"] for k in its[255]), its
        assert set(its[63]) <= {gold["iterations"] - 2, gold["iterations"]}, its
        assert its[63].count(gold["iterations"]) > len(its[63]) // 2, its


def test_minres_status_paths():
    n = 7
    prob = O.Problem(WL.coef_c1(n), -50.0, 2.0)
    f = _crand((n, n), 3)
    _, info = prob.solve(f, maxit=2)
    assert info["status"] == O.STATUS_NOT_CONVERGED and info["iters"] == 2
    z, info = prob.solve(np.zeros((n, n), complex))
    assert info["status"] == O.STATUS_OK and info["iters"] == 0 and not z.any()
    bad = f.copy()
    bad[1, 1] = np.nan
    _, info = prob.solve(bad)
    assert info["status"] == O.STATUS_NONFINITE


# ---------------------------------------------------------------- adjoint

def _loss_grad_fd(a, alpha, beta, f, zt, which, idx, h=1e-6):
    def L(a_, al, be, f_):
        p = O.Problem(a_, al, be)
        z = p.direct(f_)
        return float(np.sum(np.abs(z - zt) ** 2))
    if which == "alpha":
        return (L(a, alpha + h, beta, f) - L(a, alpha - h, beta, f)) / (2 * h)
    if which == "beta":
        return (L(a, alpha, beta + h, f) - L(a, alpha, beta - h, f)) / (2 * h)
    if which in ("fre", "fim"):
        e = np.zeros_like(f)
        e[idx] = h if which == "fre" else 1j * h
        return (L(a, alpha, beta, f + e) - L(a, alpha, beta, f - e)) / (2 * h)
    if which == "a":
        e = np.zeros_like(a)
        e[idx] = h
        return (L(a + e, alpha, beta, f) - L(a - e, alpha, beta, f)) / (2 * h)
    raise ValueError(which)


def test_adjoint_against_finite_differences():
    n = 6
    a = _rand_coef((n, n), 61, 0.7, 1.6)
    alpha, beta = -35.0, 20.0
    f = _crand((n, n), 62)
    zt = _crand((n, n), 63)
    prob = O.Problem(a, alpha, beta)
    z = prob.direct(f)
    G = 2.0 * (z - zt)
    y, _ = O.adjoint_solve(prob, G, direct=True)
    g = O.adjoint_gradients(a, alpha, beta, z, y)
    # central differences with step 1e-6 carry rounding noise of about
    # eps * L / h, so the absolute tolerance is scaled by the loss value
    loss = float(np.sum(np.abs(z - zt) ** 2))
    noise = 100 * np.finfo(float).eps * loss / 1e-6
    fd = lambda which, idx: _loss_grad_fd(a, alpha, beta, f, zt, which, idx)
    assert g["alpha"] == pytest.approx(fd("alpha", None), rel=1e-6, abs=noise)
    assert g["beta"] == pytest.approx(fd("beta", None), rel=1e-6, abs=noise)
    for idx in [(0, 0), (2, 3), (5, 1)]:
        assert g["f"][idx].real == pytest.approx(fd("fre", idx), rel=1e-6, abs=noise)
        assert g["f"][idx].imag == pytest.approx(fd("fim", idx), rel=1e-6, abs=noise)
    for idx in [(0, 0), (0, 3), (3, 3), (5, 5), (2, 5)]:
        assert g["a"][idx] == pytest.approx(fd("a", idx), rel=1e-6, abs=noise)


def test_adjoint_against_torch_autograd_dense():
    torch = pytest.importorskip("torch")
    n = 4
    a_np = _rand_coef((n, n), 71, 0.6, 1.8)
    alpha, beta = 12.0, -7.0
    f_np = _crand((n, n), 72)
    zt_np = _crand((n, n), 73)
    # dense K assembled differentiably, from the stencil definition
    a = torch.tensor(a_np, dtype=torch.float64, requires_grad=True)
    al = torch.tensor(alpha, dtype=torch.float64, requires_grad=True)
    be = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    f = torch.tensor(f_np, dtype=torch.complex128, requires_grad=True)
    h = 1.0 / (n + 1)
    M = n * n
    rows = []
    for i in range(n):
        for j in range(n):
            row = [torch.zeros((), dtype=torch.float64) for _ in range(M)]
            for (di, dj) in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < n and 0 <= jj < n:
                    c = 2 * a[i, j] * a[ii, jj] / (a[i, j] + a[ii, jj])
                    row[ii * n + jj] = row[ii * n + jj] - c / h ** 2
                else:
                    c = a[i, j]
                row[i * n + j] = row[i * n + j] + c / h ** 2
            rows.append(torch.stack(row))
    K = torch.stack(rows)
    Kc = K.to(torch.complex128) + torch.complex(al, be) * torch.eye(M, dtype=torch.complex128)
    z = torch.linalg.solve(Kc, f.reshape(-1))
    loss = torch.sum(torch.abs(z - torch.tensor(zt_np.ravel())) ** 2)
    loss.backward()
    prob = O.Problem(a_np, alpha, beta)
    zz = prob.direct(f_np)
    y, _ = O.adjoint_solve(prob, 2.0 * (zz - zt_np), direct=True)
    g = O.adjoint_gradients(a_np, alpha, beta, zz, y)
    assert np.allclose(g["a"], a.grad.numpy(), rtol=1e-8, atol=1e-10)
    assert g["alpha"] == pytest.approx(al.grad.item(), rel=1e-9)
    assert g["beta"] == pytest.approx(be.grad.item(), rel=1e-9)
    assert np.allclose(g["f"], f.grad.numpy().reshape(n, n), rtol=1e-9, atol=1e-12)


def test_adjoint_minres_matches_direct():
    n = 15
    a = WL.coef_c1(n)
    prob = O.Problem(a, -20.0, 30.0)
    G = _crand((n, n), 81)
    y_it, info = O.adjoint_solve(prob, G, tol=1e-12)
    y_d, _ = O.adjoint_solve(prob, G, direct=True)
    assert np.linalg.norm(y_it - y_d) / np.linalg.norm(y_d) < 1e-10


# ---- the alpha-circulant all-at-once layer --------------------------------

@pytest.mark.parametrize("L,alpha_c", [(8, 0.1), (16, 1e-2), (8, 1.0)])
def test_alpha_circulant_shifts_are_its_eigenvalues(L, alpha_c):
    tau = 0.05
    C = O.alpha_circulant(L, tau, alpha_c)
    D = O.alpha_circulant_shifts(L, tau, alpha_c)
    ev = np.linalg.eigvals(C)
    scale = np.abs(D).max()
    # every closed-form shift is an eigenvalue, and they are L distinct ones
    assert max(np.abs(ev - d).min() for d in D) <= 1e-12 * scale
    assert min(abs(D[i] - D[j]) for i in range(L) for j in range(i)) > 1e-6 * scale


@pytest.mark.parametrize("alpha_c", [0.1, 1e-3])
def test_paradiag_transforms_diagonalise_the_alpha_circulant(alpha_c):
    # inverse(D * forward(X)) = C X fixes the order of the shifts, the sign of
    # the DFT and the direction of the alpha^(k/L) scaling
    L, tau = 16, 0.02
    C = O.alpha_circulant(L, tau, alpha_c)
    D = O.alpha_circulant_shifts(L, tau, alpha_c)
    X = _crand((L, 5), 11)
    Y = O.paradiag_inverse(D[:, None] * O.paradiag_forward(X, alpha_c), alpha_c)
    assert np.abs(Y - C @ X).max() <= 1e-10 * np.abs(C @ X).max()
    # forward and inverse are each other's inverse
    assert np.abs(O.paradiag_inverse(O.paradiag_forward(X, alpha_c), alpha_c) - X).max() <= 1e-12


@pytest.mark.parametrize("shape", [(7, 7), (7, 3, 7)])
def test_paradiag_solve_matches_all_at_once_direct_solve(shape):
    L, tau, alpha_c = 8, 0.1, 0.1
    a = np.random.default_rng(3).uniform(0.5, 2.0, shape)
    R = _crand((L,) + shape, 4)
    U, _ = O.paradiag_solve(a, L, tau, alpha_c, R)
    A = O.all_at_once_matrix(O.build_K(a), L, tau, alpha_c)
    Ud = spla.spsolve(A, R.ravel()).reshape(R.shape)
    assert np.linalg.norm(U - Ud) <= 1e-11 * np.linalg.norm(Ud)
    # with MINRES on each mode (tol 1e-10) the result stays within the
    # modes' tolerance times the conditioning of the alpha scaling
    Um, infos = O.paradiag_solve(a, L, tau, alpha_c, R, direct=False, tol=1e-10)
    assert all(i["status"] == O.STATUS_OK for i in infos)
    assert np.linalg.norm(Um - Ud) <= 1e-8 * np.linalg.norm(Ud)


def test_paradiag_small_alpha_approaches_implicit_euler():
    # alpha -> 0 turns the alpha-circulant factor into implicit Euler's
    # bidiagonal one: the all-at-once solution approaches the step-by-step
    # solution at O(alpha)
    L, tau, n = 8, 0.1, 7
    a = np.random.default_rng(3).uniform(0.5, 2.0, (n, n))
    R = _crand((L, n, n), 6)
    Ue = O.implicit_euler(a, L, tau, R)
    errs = []
    for alpha_c in (1e-3, 1e-5):
        U, _ = O.paradiag_solve(a, L, tau, alpha_c, R)
        errs.append(np.linalg.norm(U - Ue) / np.linalg.norm(Ue))
    assert errs[1] <= 1e-4 and errs[1] < errs[0] / 50, errs


# ---- Ritz values of the Lanczos tridiagonal --------------------------------

def test_ritz_values_constant_coefficient_are_pm1():
    # Theorem 1: with a constant, P^{-1} A has only the eigenvalues +-1; the
    # two-step Lanczos tridiagonal reproduces them
    n = 15
    prob = O.Problem(np.full((n, n), 1.7), 30.0, 40.0)
    _, info = prob.solve(_crand((n, n), 3), tol=1e-10)
    assert info["iters"] == 2
    th = O.ritz_values(info["delta"], info["gamma"])
    assert np.allclose(th, [-1.0, 1.0], atol=1e-10)


def test_ritz_values_interlace_and_converge_to_the_extremes():
    # Ritz values of T_k lie between the extreme eigenvalues of P^{-1} A
    # (from the dense generalised problem) and the outermost ones converge
    # to them
    n = 7
    a = WL.coef_c1(n) * 1.5
    alpha, beta = 20.0, 15.0
    prob = O.Problem(a, alpha, beta)
    B = O.block_matrix(prob.K, alpha, beta).toarray()
    P = np.linalg.inv(O.dense_Pinv(a.shape, prob.abar, alpha, beta))
    ev = sla.eigh(B, sla.block_diag(P, P), eigvals_only=True)
    _, info = prob.solve(_crand((n, n), 4), fixed_iters=40)
    th = O.ritz_values(info["delta"], info["gamma"])
    assert th.min() >= ev.min() * (1 + 1e-10) - 1e-12 and th.max() <= ev.max() * (1 + 1e-10) + 1e-12
    # the two largest |eigenvalues| nearly coincide (1.402769, 1.402816),
    # so the outermost Ritz values approach them slowly: 5e-6 after 40 steps
    assert abs(th.max() - ev.max()) <= 1e-4 * abs(ev.max())
    assert abs(th.min() - ev.min()) <= 1e-4 * abs(ev.min())
