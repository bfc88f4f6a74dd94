"""Plain FP64 CPU oracle for absolute-value preconditioned MINRES on
complex-shifted Laplacian systems (Lin, Li & Hon, arXiv:2408.00488).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or call this module.  The product
path (the HIP library and its Python binding) never does, and this module
imports nothing from the product package: both sides receive the same
seeded inputs from the caller.

Everything here is deliberately slow and literal: NumPy / SciPy in float64,
no blocking, no fusion.  Each function names the passage of the paper it
writes out.  Where the paper is silent or garbled, the reading used is stated
in the docstring (the same readings are listed in the design notes).

Storage convention.  A real block vector [x1; x2] of length 2M is held as
the complex array x1 + i*x2 of shape (n,)*d (last axis contiguous).  The real
inner product of two block vectors is then Re(p^H q).

Pins.  Every function is pinned by tests against something other than
itself (closed forms, dense linear algebra, the paper's theorems and tables,
brute force on tiny grids); see tests/test_oracle_pins.py.  The paper does
not state the domain of its Example 2; on the unit square the iteration
count of Table 2(a) (14 for every listed shift) is reproduced at n = 63 and
n = 255, and checked there together with its independence of n.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# --------------------------------------------------------------------------
# Grid, coefficient, finite-difference operator  (Section 1, Eq. (1))
# --------------------------------------------------------------------------


def mesh_widths(shape, lengths=None):
    """h_k = length_k / (n_k + 1) on a rectangular domain (unit by default)."""
    if lengths is None:
        lengths = [1.0] * len(shape)
    return [float(lengths[k]) / (shape[k] + 1) for k in range(len(shape))]


def face_coefficients(a):
    """Face coefficients of the variable-coefficient stencil.

    Reading (the paper gives no scheme for variable a, Section 1): the face
    between neighbouring interior nodes p, q carries the harmonic mean
    c = 2 a_p a_q / (a_p + a_q); a face between node p and the Dirichlet
    boundary carries c = a_p (ghost value equal to the adjacent interior one).

    Returns one array per axis k with n_k + 1 faces along that axis:
    face j lies between nodes j-1 and j (faces 0 and n_k are boundary faces).
    """
    a = np.asarray(a, dtype=np.float64)
    out = []
    for ax in range(a.ndim):
        n = a.shape[ax]
        lo = np.take(a, np.arange(0, n - 1), axis=ax)
        hi = np.take(a, np.arange(1, n), axis=ax)
        inner = 2.0 * lo * hi / (lo + hi)
        first = np.take(a, [0], axis=ax)
        last = np.take(a, [n - 1], axis=ax)
        out.append(np.concatenate([first, inner, last], axis=ax))
    return out


def build_K(a, lengths=None):
    """Sparse FD matrix K of -div(a grad) with homogeneous Dirichlet data.

    (K u)_p = sum over the 2d faces e of p of c_e (u_p - u_nbr(e)) / h_axis^2,
    with u = 0 outside the domain (Section 1, Eq. (1); 5-point in 2-D,
    7-point in 3-D).  Nodes are numbered in C order (last axis fastest).
    Assembled face by face, so it is symmetric by construction.
    """
    a = np.asarray(a, dtype=np.float64)
    shape = a.shape
    M = a.size
    hs = mesh_widths(shape, lengths)
    idx = np.arange(M).reshape(shape)
    rows, cols, vals = [], [], []
    diag = np.zeros(M)
    for ax, c in enumerate(face_coefficients(a)):
        n = shape[ax]
        w = c / hs[ax] ** 2
        # boundary faces: diagonal only
        w_first = np.take(w, [0], axis=ax).ravel()
        w_last = np.take(w, [n], axis=ax).ravel()
        diag[np.take(idx, [0], axis=ax).ravel()] += w_first
        diag[np.take(idx, [n - 1], axis=ax).ravel()] += w_last
        # interior faces between p = (.., j-1, ..) and q = (.., j, ..)
        if n > 1:
            wi = np.take(w, np.arange(1, n), axis=ax).ravel()
            p = np.take(idx, np.arange(0, n - 1), axis=ax).ravel()
            q = np.take(idx, np.arange(1, n), axis=ax).ravel()
            np.add.at(diag, p, wi)
            np.add.at(diag, q, wi)
            rows += [p, q]
            cols += [q, p]
            vals += [-wi, -wi]
    rows.append(np.arange(M))
    cols.append(np.arange(M))
    vals.append(diag)
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows),
                                              np.concatenate(cols))),
                      shape=(M, M)).tocsr()
    K.sum_duplicates()
    return K


def laplacian_1d(n, h):
    """Textbook tridiag(-1, 2, -1) / h^2 (Dirichlet), dense."""
    T = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return T / h ** 2


# --------------------------------------------------------------------------
# Real 2x2 block form  (Section 1, Eq. (2); orientation reading A1)
# --------------------------------------------------------------------------


def apply_A(K, alpha, beta, x):
    """Block operator  A = [[S, beta I], [beta I, -S]],  S = K + alpha I.

    Reading of Eq. (2): as printed, its right-hand side [a; b] does not
    match its first block row; we use the consistent form whose unknown is
    [Re z; -Im z] and whose right-hand side is [Re f; Im f].  In complex
    storage (x = x1 + i x2) the product is y = (K + lambda I) conj(x).
    """
    x = np.asarray(x)
    xc = np.conj(x).ravel()
    y = K @ xc + complex(alpha, beta) * xc
    return y.reshape(x.shape)


def block_matrix(K, alpha, beta):
    """Explicit real 2M x 2M matrix of apply_A acting on [x1; x2]."""
    M = K.shape[0]
    S = (K + alpha * sp.identity(M)).tocsr()
    B = beta * sp.identity(M)
    return sp.bmat([[S, B], [B, -S]]).tocsr()


def paper_block_matrix(K, alpha, beta):
    """Eq. (2) exactly as printed: [[beta I, S], [S, -beta I]] acting on
    [z1; z2].  Used only to test the orientation reading."""
    M = K.shape[0]
    S = (K + alpha * sp.identity(M)).tocsr()
    B = beta * sp.identity(M)
    return sp.bmat([[B, S], [S, -B]]).tocsr()


def to_block(x):
    x = np.asarray(x).ravel()
    return np.concatenate([x.real, x.imag])


def from_block(v, shape):
    M = len(v) // 2
    return (v[:M] + 1j * v[M:]).reshape(shape)


def absm(H):
    """|H| = Q^T diag(|lambda_i|) Q for a real symmetric H (Section 1)."""
    lam, Q = np.linalg.eigh(H)
    return (Q * np.abs(lam)) @ Q.T


def sqrtm_spd(H):
    """sqrt(H) = Q^T diag(sqrt(lambda_i)) Q for symmetric H >= 0 (Section 1)."""
    lam, Q = np.linalg.eigh(H)
    return (Q * np.sqrt(np.maximum(lam, 0.0))) @ Q.T


# --------------------------------------------------------------------------
# Sine transform and the averaged preconditioner  (Eq. (4), Section 2.3)
# --------------------------------------------------------------------------


def mu_1d(n, h):
    """Eigenvalues of tridiag(-1,2,-1)/h^2: (4/h^2) sin^2(k pi / (2(n+1))),
    k = 1..n (closed form; the paper only says they are positive)."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return (4.0 / h ** 2) * np.sin(k * np.pi / (2.0 * (n + 1))) ** 2


def sine_matrix(n):
    """Dense orthonormal DST-I matrix W_jk = sqrt(2/(n+1)) sin(pi j k/(n+1))
    (Section 2.3: real, symmetric, orthogonal)."""
    j = np.arange(1, n + 1, dtype=np.float64)
    return math.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(j, j) / (n + 1))


def dst1(x, axes=None):
    """Orthonormal DST-I along the given axes (all by default), applied to
    the real and imaginary parts separately (the transform is real)."""
    x = np.asarray(x)
    if axes is None:
        axes = tuple(range(x.ndim))
    re = sfft.dstn(np.real(x), type=1, norm="ortho", axes=axes)
    if np.iscomplexobj(x):
        im = sfft.dstn(np.imag(x), type=1, norm="ortho", axes=axes)
        return re + 1j * im
    return re


def abar_value(a, rule="mean", given=None):
    """The averaged coefficient of K_bar = abar * L.

    The paper's theory uses gamma = sqrt(a_min a_max) (Eq. (4)); its
    abstract speaks of averaging.  rule="mean": arithmetic mean of the nodal
    samples; rule="geomean": sqrt(min c_e * max c_e) over all face
    coefficients (the discrete a_min, a_max of Lemma 3); rule="given".
    """
    if rule == "mean":
        return float(np.mean(a))
    if rule == "geomean":
        cs = np.concatenate([c.ravel() for c in face_coefficients(a)])
        return math.sqrt(float(cs.min()) * float(cs.max()))
    if rule == "given":
        return float(given)
    raise ValueError(rule)


def coefficient_bounds(a):
    """(a_min, a_max) over the face coefficients (the discrete reading of
    the bounds in Eq. (1) used by Lemma 3)."""
    cs = np.concatenate([c.ravel() for c in face_coefficients(a)])
    return float(cs.min()), float(cs.max())


def mode_eigenvalues(shape, lengths=None):
    """Eigenvalues of L on the tensor grid, as an array of shape `shape`:
    sum over axes of the 1-D values (L is a Kronecker sum)."""
    hs = mesh_widths(shape, lengths)
    lam = np.zeros(shape)
    for ax, n in enumerate(shape):
        mu = mu_1d(n, hs[ax])
        sh = [1] * len(shape)
        sh[ax] = n
        lam = lam + mu.reshape(sh)
    return lam


def pinv_scale(shape, abar, alpha, beta, lengths=None):
    """Per-mode factor 1/sqrt((abar*lambda_k + alpha)^2 + beta^2)
    (Eq. (4) diagonalised by the sine transform, Section 2.3)."""
    lam = abar * mode_eigenvalues(shape, lengths)
    return 1.0 / np.sqrt((lam + alpha) ** 2 + beta ** 2)


def apply_Pinv(x, abar, alpha, beta, lengths=None):
    """P^{-1} x with P = blkdiag(sqrt((abar L + alpha I)^2 + beta^2 I)) twice.

    Both diagonal blocks are the same real matrix, so in complex storage the
    real and imaginary parts are transformed alike:
    P^{-1} x = W diag(s) W x, with W the d-D orthonormal DST-I (its own
    inverse) and s the per-mode factor (Eq. (4), Section 2.3).
    """
    x = np.asarray(x)
    s = pinv_scale(x.shape, abar, alpha, beta, lengths)
    return dst1(dst1(x) * s)


def dense_Pinv(shape, abar, alpha, beta, lengths=None):
    """Dense M x M inverse of sqrt((abar L + alpha I)^2 + beta^2 I) built
    from an eigendecomposition of the assembled L (no sine transform)."""
    L = build_K(np.ones(shape), lengths).toarray()
    S = abar * L + alpha * np.eye(L.shape[0])
    P = sqrtm_spd(S @ S + beta ** 2 * np.eye(L.shape[0]))
    return np.linalg.inv(P)


# --------------------------------------------------------------------------
# Preconditioned MINRES  (Section 3: Octave's minres, zero initial guess,
# tolerance 1e-8; theory in Lemma 1 after Elman-Silvester-Wathen)
# --------------------------------------------------------------------------

STATUS_OK = 0
STATUS_NOT_CONVERGED = 3
STATUS_BREAKDOWN = 4
STATUS_NONFINITE = 5


def rdot(p, q):
    """Real inner product of block vectors in complex storage."""
    return float(np.real(np.vdot(np.ravel(p), np.ravel(q))))


def minres(A, Pinv, b, tol=1e-8, maxit=1000, check_true=True,
           fixed_iters=None, record=False):
    """Preconditioned MINRES for a symmetric A and an SPD preconditioner P.

    A(x) and Pinv(x) are callables on block vectors; b is the right-hand
    side; the initial guess is 0.  Steps: a Lanczos process in the P-inner
    product builds the tridiagonal T_k (diagonal delta_j, off-diagonal
    gamma_j); Givens rotations turn T_k into upper-triangular form; the
    iterate is advanced along the search directions w_j.  |eta_k| is the
    P^{-1}-norm of the residual b - A x_k.

    Stopping rule (reading of Section 3, which stops on a relative residual
    reduction without naming the norm): stop after iteration k when |eta_k|/|eta_0| <= tol and, if
    check_true, also ||b - A x_k||_2 / ||b||_2 <= tol (checked only once the
    first test has passed).  One iteration = one product with A and one
    with P^{-1}; the initial P^{-1} b is not counted.

    fixed_iters: run exactly that many iterations (no stopping test).
    Returns (x, info); info has iters, status, relres_est, relres_true, the
    Lanczos coefficients delta_1..delta_k and gamma_2..gamma_{k+1} (lists
    "delta", "gamma") and, if record, the list of iterates x_k and of eta_k.
    """
    b = np.asarray(b)
    bnorm = math.sqrt(rdot(b, b))
    info = {"iters": 0, "status": STATUS_OK, "relres_est": 0.0,
            "relres_true": 0.0, "history": [], "eta": [], "delta": [], "gamma": []}
    x = np.zeros_like(b)
    if not np.isfinite(bnorm):
        info["status"] = STATUS_NONFINITE
        return x, info
    if bnorm == 0.0:
        return x, info
    # Lanczos start: v_1 = b, z_1 = P^{-1} v_1, gamma_1 = sqrt(<z_1, v_1>)
    v_old = np.zeros_like(b)
    v = b.copy()
    z = Pinv(v)
    g2 = rdot(z, v)
    if not np.isfinite(g2):
        info["status"] = STATUS_NONFINITE
        return x, info
    if g2 <= 0.0:
        info["status"] = STATUS_BREAKDOWN
        return x, info
    gamma = math.sqrt(g2)
    gamma_old = 1.0
    eta0 = gamma
    eta = gamma
    c_old, c = 1.0, 1.0
    s_old, s = 0.0, 0.0
    w_old = np.zeros_like(b)
    w = np.zeros_like(b)
    limit = fixed_iters if fixed_iters is not None else maxit
    for k in range(1, limit + 1):
        z = z / gamma                       # normalised Lanczos vector
        q = A(z)
        delta = rdot(z, q)                  # diagonal of T_k
        v_new = q - (delta / gamma) * v - (gamma / gamma_old) * v_old
        z_new = Pinv(v_new)
        g2 = rdot(z_new, v_new)
        if not np.isfinite(g2):
            info["status"] = STATUS_NONFINITE
            info["iters"] = k - 1
            break
        if g2 < 0.0:
            info["status"] = STATUS_BREAKDOWN
            info["iters"] = k - 1
            break
        gamma_new = math.sqrt(g2)           # off-diagonal of T_k
        # apply the two previous rotations to column k of T_k, then the new one
        e0 = c * delta - c_old * s * gamma
        e1 = math.hypot(e0, gamma_new)
        e2 = s * delta + c_old * c * gamma
        e3 = s_old * gamma
        c_new = e0 / e1
        s_new = gamma_new / e1
        w_new = (z - e3 * w_old - e2 * w) / e1
        x = x + (c_new * eta) * w_new
        eta = -s_new * eta
        info["iters"] = k
        info["delta"].append(delta)
        info["gamma"].append(gamma_new)
        est = abs(eta) / eta0
        info["relres_est"] = est
        if record:
            info["history"].append(x.copy())
            info["eta"].append(eta)
        # rotate the recurrences
        v_old, v = v, v_new
        z = z_new
        w_old, w = w, w_new
        gamma_old, gamma = gamma, gamma_new
        c_old, c = c, c_new
        s_old, s = s, s_new
        if fixed_iters is not None:
            continue
        if gamma_new == 0.0:                # invariant subspace: x is exact
            info["relres_true"] = _relres(A, b, x, bnorm)
            break
        if est <= tol:
            if not check_true:
                break
            rt = _relres(A, b, x, bnorm)
            info["relres_true"] = rt
            if rt <= tol:
                break
        if k == maxit:
            info["status"] = STATUS_NOT_CONVERGED
    info["relres_true"] = _relres(A, b, x, bnorm)
    return x, info


def _relres(A, b, x, bnorm):
    r = b - A(x)
    return math.sqrt(rdot(r, r)) / bnorm


# --------------------------------------------------------------------------
# The complete solve of (K + lambda I) z = f  (Eqs. (1), (2), (4))
# --------------------------------------------------------------------------


class Problem:
    """One complex-shifted system with the averaged preconditioner."""

    def __init__(self, a, alpha, beta, abar_rule="mean", abar=None,
                 lengths=None):
        self.a = np.asarray(a, dtype=np.float64)
        self.shape = self.a.shape
        self.lengths = lengths
        self.alpha = float(alpha)
        self.beta = float(beta)
        self.K = build_K(self.a, lengths)
        self.abar = abar_value(self.a, abar_rule, abar)
        self.scale = pinv_scale(self.shape, self.abar, self.alpha, self.beta,
                                lengths)

    def A(self, x):
        return apply_A(self.K, self.alpha, self.beta, x)

    def Pinv(self, x):
        return dst1(dst1(x) * self.scale)

    def solve(self, f, tol=1e-8, maxit=1000, check_true=True,
              fixed_iters=None, record=False):
        """MINRES on the block system; returns (z, info) with z the
        solution of (K + lambda I) z = f (z = conj of the block iterate)."""
        x, info = minres(self.A, self.Pinv, np.asarray(f, dtype=np.complex128),
                         tol=tol, maxit=maxit, check_true=check_true,
                         fixed_iters=fixed_iters, record=record)
        return np.conj(x), info

    def direct(self, f):
        """Exact solution by a sparse direct solve (reference only)."""
        M = self.K.shape[0]
        Kc = (self.K + complex(self.alpha, self.beta) * sp.identity(M)).tocsc()
        z = spla.spsolve(Kc.astype(np.complex128), np.ravel(f))
        return z.reshape(self.shape)


# --------------------------------------------------------------------------
# Adjoint of the solve  (derived from Eq. (1): z = (K + lambda I)^{-1} f)
# --------------------------------------------------------------------------


def adjoint_gradients(a, alpha, beta, z, y, lengths=None):
    """Gradients of a real loss L(z) given the adjoint y.

    With G = dL/dRe z + i dL/dIm z and y = (K + conj(lambda) I)^{-1} G:
      dL/df     = y
      dL/dalpha = -Re(y^H z)
      dL/dbeta  =  Im(y^H z)
      dL/dc_e   = -Re(y^H (dK/dc_e) z)     for every face e,
      dL/da_p   = sum over faces e of p of dL/dc_e * dc_e/da_p,
    with dc_e/da_p = 2 a_q^2 / (a_p + a_q)^2 for an interior face (p, q)
    and 1 for a boundary face (c_e = a_p).
    """
    a = np.asarray(a, dtype=np.float64)
    shape = a.shape
    hs = mesh_widths(shape, lengths)
    yz = np.vdot(np.ravel(y), np.ravel(z))
    g_alpha = -float(np.real(yz))
    g_beta = float(np.imag(yz))
    g_a = np.zeros(shape)
    for ax in range(a.ndim):
        n = shape[ax]
        inv_h2 = 1.0 / hs[ax] ** 2
        # boundary faces at index 0 and n-1 along ax
        for j in (0, n - 1):
            yp = np.take(y, [j], axis=ax)
            zp = np.take(z, [j], axis=ax)
            dLdc = -inv_h2 * np.real(np.conj(yp) * zp)
            sl = [slice(None)] * a.ndim
            sl[ax] = slice(j, j + 1)
            g_a[tuple(sl)] += dLdc
        if n > 1:
            ap = np.take(a, np.arange(0, n - 1), axis=ax)
            aq = np.take(a, np.arange(1, n), axis=ax)
            dy = np.take(y, np.arange(0, n - 1), axis=ax) - \
                np.take(y, np.arange(1, n), axis=ax)
            dz = np.take(z, np.arange(0, n - 1), axis=ax) - \
                np.take(z, np.arange(1, n), axis=ax)
            dLdc = -inv_h2 * np.real(np.conj(dy) * dz)
            s2 = (ap + aq) ** 2
            lo = [slice(None)] * a.ndim
            hi = [slice(None)] * a.ndim
            lo[ax] = slice(0, n - 1)
            hi[ax] = slice(1, n)
            g_a[tuple(lo)] += dLdc * 2.0 * aq ** 2 / s2
            g_a[tuple(hi)] += dLdc * 2.0 * ap ** 2 / s2
    return {"f": np.asarray(y), "alpha": g_alpha, "beta": g_beta, "a": g_a}


def adjoint_solve(prob: Problem, G, tol=1e-8, maxit=1000, check_true=True,
                  direct=False):
    """y = (K + conj(lambda) I)^{-1} G, by the same MINRES on the same
    symmetric block matrix with right-hand side conj(G) (y is then the block
    iterate itself), or by a direct solve."""
    if direct:
        M = prob.K.shape[0]
        Kc = (prob.K + complex(prob.alpha, -prob.beta) *
              sp.identity(M)).tocsc()
        return spla.spsolve(Kc.astype(np.complex128),
                            np.ravel(G)).reshape(prob.shape), {}
    x, info = minres(prob.A, prob.Pinv, np.conj(np.asarray(G, np.complex128)),
                     tol=tol, maxit=maxit, check_true=check_true)
    return x, info


# --------------------------------------------------------------------------
# Theory helpers used as test pins  (Lemma 1, Lemma 3, Theorem 3, Theorem 4)
# --------------------------------------------------------------------------


def lemma1_bound(a1, a2, a3, a4, k):
    """2 ((sqrt(a1 a4) - sqrt(a2 a3)) / (sqrt(a1 a4) + sqrt(a2 a3)))^floor(k/2)."""
    p = math.sqrt(a1 * a4)
    q = math.sqrt(a2 * a3)
    return 2.0 * ((p - q) / (p + q)) ** (k // 2)


def theorem3_bounds(a_min, a_max, c0, alpha, beta):
    """Interval [lo, hi] for |eig(P^{-1} A)| with abar = sqrt(a_min a_max)
    (Theorem 3).  Part (i) for alpha >= 0: [1/mu0, mu0], mu0 = sqrt(2 a_max /
    a_min).  Part (ii) for alpha < 0: [mu1~, mu0~]; because the printed
    conditions are inconsistent, the test interval widens to
    [min(1/mu0, mu1~), max(mu0, mu0~)]."""
    mu0 = math.sqrt(2.0 * a_max / a_min)
    if alpha >= 0:
        return 1.0 / mu0, mu0
    gam = math.sqrt(a_min * a_max)
    ab = abs(beta)
    mt0 = math.sqrt(2.0) * (c0 * a_max + ab - alpha) / (c0 * gam + ab + alpha)
    mt1 = math.sqrt(2.0) * (c0 * a_min + ab + alpha) / (2.0 * (c0 * gam + ab - alpha))
    return min(1.0 / mu0, mt1), max(mu0, mt0)


# --------------------------------------------------------------------------
# The alpha-circulant all-at-once layer  (Section 1: evolutionary problems
# whose time-stepping matrix is replaced by an alpha-circulant one become,
# after block diagonalisation, one complex-shifted system per eigenvalue)
#
# Reading (the paper describes the setting, not its matrices): implicit Euler
# with step tau for u' + K u = g over L steps gives the time factor
# B = (I - Z_0)/tau, Z_0 the down-shift; the alpha-circulant factor is
# C = (I - Z_alpha)/tau, where Z_alpha also carries alpha in its top-right
# corner.  The time-space matrix is kron(C, I) + kron(I, K); a right-hand
# side or solution is an array (L, *grid), step index first.
# --------------------------------------------------------------------------


def alpha_circulant(L, tau, alpha_c):
    """Dense C = (I - Z_alpha)/tau."""
    Z = np.zeros((L, L))
    Z[np.arange(1, L), np.arange(L - 1)] = 1.0
    Z[0, L - 1] = alpha_c
    return (np.eye(L) - Z) / tau


def alpha_circulant_shifts(L, tau, alpha_c):
    """Eigenvalues of C in the order of the forward transform below:
    D_j = (1 - alpha^(1/L) exp(-2 pi i j / L)) / tau, j = 0..L-1.  With
    Gamma = diag(alpha^(k/L)), Gamma Z_alpha Gamma^-1 = alpha^(1/L) times the
    cyclic shift, which the DFT F (exp(-2 pi i j k / L)) diagonalises."""
    j = np.arange(L)
    return (1.0 - alpha_c ** (1.0 / L) * np.exp(-2j * np.pi * j / L)) / tau


def all_at_once_matrix(K, L, tau, alpha_c):
    """kron(C, I_M) + kron(I_L, K), sparse complex (reference only)."""
    M = K.shape[0]
    C = sp.csr_matrix(alpha_circulant(L, tau, alpha_c))
    return (sp.kron(C, sp.identity(M)) + sp.kron(sp.identity(L), K)).tocsc().astype(np.complex128)


def paradiag_forward(R, alpha_c):
    """(F Gamma (x) I) R: step k scaled by alpha^(k/L), then the DFT over steps."""
    R = np.asarray(R, dtype=np.complex128)
    L = R.shape[0]
    g = alpha_c ** (np.arange(L) / L)
    return np.fft.fft(R * g.reshape((L,) + (1,) * (R.ndim - 1)), axis=0)


def paradiag_inverse(U, alpha_c):
    """(Gamma^-1 F^-1 (x) I) U: inverse DFT over steps, then alpha^(-k/L)."""
    U = np.asarray(U, dtype=np.complex128)
    L = U.shape[0]
    g = alpha_c ** (-np.arange(L) / L)
    return np.fft.ifft(U, axis=0) * g.reshape((L,) + (1,) * (U.ndim - 1))


def paradiag_solve(a, L, tau, alpha_c, R, direct=True, tol=1e-8, maxit=1000,
                   abar_rule="mean", lengths=None):
    """Solve (kron(C, I) + kron(I, K)) U = R through the diagonalisation:
    transform R, solve (K + D_j I) Ut_j = Rt_j for every step mode j (a direct
    solve, or MINRES with the averaged preconditioner), transform back.
    Returns (U, infos) with one info dict per mode (None for direct)."""
    D = alpha_circulant_shifts(L, tau, alpha_c)
    Rt = paradiag_forward(R, alpha_c)
    Ut = np.empty_like(Rt)
    infos = []
    for j in range(L):
        prob = Problem(a, D[j].real, D[j].imag, abar_rule=abar_rule, lengths=lengths)
        if direct:
            Ut[j] = prob.direct(Rt[j])
            infos.append(None)
        else:
            Ut[j], info = prob.solve(Rt[j], tol=tol, maxit=maxit)
            infos.append(info)
    return paradiag_inverse(Ut, alpha_c), infos


def implicit_euler(a, L, tau, R, lengths=None):
    """Step-by-step implicit Euler for u' + K u = g from u_0 = 0:
    (I/tau + K) u_k = u_{k-1}/tau + g_k, with R[k] = g_k; the system that
    the alpha-circulant factor approximates (reference only)."""
    K = build_K(np.asarray(a, dtype=np.float64), lengths)
    M = K.shape[0]
    Ak = (K + sp.identity(M) / tau).tocsc().astype(np.complex128)
    U = np.empty((L,) + np.shape(a), dtype=np.complex128)
    prev = np.zeros(M, dtype=np.complex128)
    for k in range(L):
        prev = spla.spsolve(Ak, prev / tau + np.ravel(R[k]))
        U[k] = prev.reshape(np.shape(a))
    return U


# --------------------------------------------------------------------------
# Ritz values of the preconditioned operator  (the Lanczos tridiagonal that
# MINRES builds, Section 3; its extreme eigenvalues approach those bounded
# by Theorem 3)
# --------------------------------------------------------------------------


def ritz_values(delta, gamma):
    """Eigenvalues of T_k = tridiag(gamma_2..gamma_k; delta_1..delta_k;
    gamma_2..gamma_k), ascending; delta and gamma as minres records them
    (gamma[j] = gamma_{j+2}, the last entry couples to step k + 1)."""
    import scipy.linalg as sla
    d = np.asarray(delta, dtype=np.float64)
    k = d.size
    if k == 0:
        return d
    e = np.asarray(gamma, dtype=np.float64)[:k - 1]
    return sla.eigvalsh_tridiagonal(d, e)
