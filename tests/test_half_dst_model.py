"""The half-length sine transform used by the FP64 plane phase, as a NumPy
model of its lane layout (CPU): a DST-I of n = N - 1 points through a complex
FFT of N points of the combined line y_j = sin(pi j/N)(x_j + x_{N-j}) +
(x_j - x_{N-j})/2, the even outputs from Y_m - Y_{N-m}, the odd ones a
running sum of Y_m + Y_{N-m} scanned over the line's N/4 lanes (each lane
holding m = 2t, 2t + 1 and leaving with outputs 4t .. 4t + 3).  Pinned to
SciPy's orthonormal DST-I (the transform the preconditioner of Section 2.3
applies along each axis) for complex lines of every length the plane admits,
and to its being its own inverse."""
import numpy as np
import pytest
from scipy.fft import dst


def half_dst(x):
    n = x.size
    N = n + 1
    Q = N // 4
    X = np.zeros(N, complex)
    X[1:] = x
    i = np.arange(N)
    s = np.sin(np.pi * i / N)
    y = s * (X + X[(N - i) % N]) + 0.5 * (X - X[(N - i) % N])
    y[0] = 0.0
    Y = np.fft.fft(y)
    cf = 1.0 / np.sqrt(2 * N)
    out = np.zeros(N, complex)
    B = np.zeros((Q, 2), complex)
    E = np.zeros((Q, 2), complex)
    for t in range(Q):
        ya, yb = Y[2 * t], Y[2 * t + 1]
        za, zb = Y[(N - 2 * t) % N], Y[N - 2 * t - 1]
        B[t, 0] = cf * ya if t == 0 else cf * (ya + za)
        B[t, 1] = cf * (yb + zb)
        E[t, 0] = 1j * cf * (ya - za)
        E[t, 1] = 1j * cf * (yb - zb)
    c = B[:, 0] + B[:, 1]
    incl = c.copy()
    d = 1
    while d < Q:   # shfl_up scan over the line's lanes
        prev = incl.copy()
        incl[d:] = prev[d:] + prev[:-d]
        d *= 2
    ex = incl - c
    for t in range(Q):
        if t >= 1:
            out[4 * t] = E[t, 0]
        out[4 * t + 1] = ex[t] + B[t, 0]
        out[4 * t + 2] = E[t, 1]
        out[4 * t + 3] = incl[t]
    return out[1:]


@pytest.mark.parametrize("n", [3, 7, 15, 31, 63, 127, 255, 511])
def test_half_length_dst_matches_dst1(n):
    g = np.random.default_rng(n)
    x = g.standard_normal(n) + 1j * g.standard_normal(n)
    ref = dst(x.real, type=1, norm="ortho") + 1j * dst(x.imag, type=1, norm="ortho")
    got = half_dst(x)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref)) * np.log2(n + 1)
    back = half_dst(got)
    assert np.max(np.abs(back - x)) <= 1e-14 * np.max(np.abs(x)) * np.log2(n + 1)


def test_half_length_dst_single_modes():
    # a single sine mode goes to a single output (up to the orthonormal scale)
    n = 63
    j = np.arange(1, n + 1)
    for k in (1, 2, 31, 32, 62, 63):
        x = np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * j * k / (n + 1)) + 0j
        got = half_dst(x)
        e = np.zeros(n)
        e[k - 1] = 1.0
        assert np.max(np.abs(got - e)) <= 1e-13
