"""Seeded synthetic inputs for the complex-shifted Laplacian solver.

This module only draws and tabulates inputs: grid sizes, nodal coefficient
samples, complex shifts and right-hand sides.  It contains none of the
solver's arithmetic (no stencil, no transform, no Krylov step), so both the
GPU path and the independent CPU checker can be fed from it without sharing
any of the method's code.  It imports nothing from the rest of the package.

Conventions
-----------
* A d-dimensional grid has ``n`` interior points per axis on the unit square
  or cube, mesh width ``h = 1/(n+1)``, interior node ``i`` (0-based) at
  coordinate ``(i+1)*h``.  Arrays are C-ordered with the LAST axis
  contiguous; array axis ``k`` carries coordinate ``x_{k+1}``
  (``numpy.meshgrid(..., indexing="ij")``).
* Complex vectors are complex128 arrays of shape ``(n,)*d``.
* Random numbers come from ``numpy.random.Generator(PCG64(seed))``, drawn in
  C order, real part first, then imaginary part.

The paper measures only synthetic inputs (a random exact solution, analytic
coefficients, chosen shifts; Section 3).  The workloads below are synthetic
stand-ins of the same family: 2-D or 3-D grids with n = 2^k - 1, random
complex data, zero initial guess, tolerance 1e-8.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload", "SystemSpec", "nodes", "coef_c1", "coef_c2", "coef_c3",
    "coef_paper_ex2", "rng", "complex_normal", "workload",
    "batched_shifts", "WORKLOAD_NAMES",
]


def rng(seed) -> np.random.Generator:
    """PCG64 generator; ``seed`` may be an int or a list of ints."""
    return np.random.Generator(np.random.PCG64(seed))


def complex_normal(g: np.random.Generator, shape) -> np.ndarray:
    """Re and Im i.i.d. N(0,1), real block drawn first (C order)."""
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return re + 1j * im


def nodes(n: int, d: int, length: float = 1.0):
    """Coordinates of the interior nodes, one array per axis (ij indexing)."""
    h = length / (n + 1)
    x = (np.arange(n, dtype=np.float64) + 1.0) * h
    return np.meshgrid(*([x] * d), indexing="ij")


def coef_c1(n: int) -> np.ndarray:
    """a(x,y) = 1 + 0.5 sin(2 pi x) sin(2 pi y), sampled at interior nodes."""
    x, y = nodes(n, 2)
    return 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)


def coef_c2(n: int) -> np.ndarray:
    """a(x,y) = 1 + 0.9 exp(-20((x-1/2)^2 + (y-1/2)^2)), in [1, 1.9]."""
    x, y = nodes(n, 2)
    return 1.0 + 0.9 * np.exp(-20.0 * ((x - 0.5) ** 2 + (y - 0.5) ** 2))


def coef_c3(n: int) -> np.ndarray:
    """a(x,y,z) = 2 + sin(pi x) cos(pi y) sin(pi z), in [1, 3]."""
    x, y, z = nodes(n, 3)
    return 2.0 + np.sin(np.pi * x) * np.cos(np.pi * y) * np.sin(np.pi * z)


def coef_paper_ex2(n: int) -> np.ndarray:
    """The paper's Example 2 coefficient a = (20 + x1^2)(20 + x2^2) on the
    unit square (the paper does not state its domain)."""
    x, y = nodes(n, 2)
    return (20.0 + x ** 2) * (20.0 + y ** 2)


def batched_shifts(count: int = 64, gamma_circ: float = 1e-2,
                   tau: float = 1.0 / 64) -> np.ndarray:
    """Shifts of an alpha-circulant all-at-once time discretisation:
    lambda_j = (1 - gamma^(1/count) e^{2 pi i j/count}) / tau, j = 0..count-1
    (the motivating setting of the paper's introduction)."""
    j = np.arange(count)
    return (1.0 - gamma_circ ** (1.0 / count) * np.exp(2j * np.pi * j / count)) / tau


def _box5(u: np.ndarray) -> np.ndarray:
    """5x5 mean filter over in-bounds cells (count-normalised)."""
    n0, n1 = u.shape
    pad = np.zeros((n0 + 4, n1 + 4))
    cnt = np.zeros((n0 + 4, n1 + 4))
    pad[2:-2, 2:-2] = u
    cnt[2:-2, 2:-2] = 1.0
    s = np.zeros_like(u)
    c = np.zeros_like(u)
    for di in range(5):
        for dj in range(5):
            s += pad[di:di + n0, dj:dj + n1]
            c += cnt[di:di + n0, dj:dj + n1]
    return s / c


@dataclass
class SystemSpec:
    """One shifted system (K + lambda I) z = f on one grid."""
    n: int
    d: int
    a: np.ndarray           # nodal coefficient, shape (n,)*d, float64
    lam: complex            # shift alpha + i beta
    f: np.ndarray           # right-hand side, complex128, shape (n,)*d
    z_target: np.ndarray | None = None   # only for the adjoint workload


@dataclass
class Workload:
    name: str
    description: str
    systems: list = field(default_factory=list)
    pinv_fp32: bool = False
    share_coefficient: bool = False


WORKLOAD_NAMES = ("c1", "c2", "c2_const", "c3", "c4", "c5")


def workload(name: str, n_override: int | None = None,
             count_override: int | None = None) -> Workload:
    """Build one of the named synthetic workloads.

    ``n_override`` shrinks the grid (same coefficient formula and draw order)
    for fast tests; ``count_override`` limits the number of systems of the
    batched workloads.
    """
    if name == "c1":
        n = n_override or 63
        g = rng(1)
        f = complex_normal(g, (n, n))
        return Workload("c1", f"2-D n={n}, a=1+0.5 sin(2pi x)sin(2pi y), "
                        "lambda=1+1i, FP64",
                        [SystemSpec(n, 2, coef_c1(n), 1 + 1j, f)])
    if name in ("c2", "c2_const"):
        n = n_override or 511
        g = rng(2)
        f = complex_normal(g, (n, n))
        a = coef_c2(n) if name == "c2" else np.ones((n, n))
        desc = "a=1+0.9exp(-20r^2)" if name == "c2" else "a=1"
        return Workload(name, f"2-D n={n}, {desc}, lambda=-200+50i, FP64",
                        [SystemSpec(n, 2, a, -200 + 50j, f)])
    if name == "c3":
        n = n_override or 127
        g = rng(3)
        f = complex_normal(g, (n, n, n))
        return Workload("c3", f"3-D n={n}, a=2+sin(pi x)cos(pi y)sin(pi z), "
                        "lambda=10+100i, FP32 preconditioner",
                        [SystemSpec(n, 3, coef_c3(n), 10 + 100j, f)],
                        pinv_fp32=True)
    if name == "c4":
        count = count_override or 64
        sizes = (63, 127, 255, 511)
        if n_override:
            sizes = tuple(min(s, n_override) for s in sizes)
        lams = batched_shifts(64)
        systems = []
        for j in range(count):
            n = sizes[j % 4]
            g = rng([4, j])
            f = complex_normal(g, (n, n))
            systems.append(SystemSpec(n, 2, coef_c1(n), complex(lams[j]), f))
        return Workload("c4", f"{count} shifted 2-D systems, "
                        "n in {63,127,255,511}, a=1+0.5 sin sin, "
                        "lambda_j alpha-circulant spectrum (tau=1/64, gamma=1e-2)",
                        systems, pinv_fp32=True)
    if name == "c5":
        n = n_override or 255
        count = count_override or 16
        g = rng(5)
        alpha = g.uniform(-50.0, 50.0, 16)
        beta = g.uniform(1.0, 100.0, 16)
        u = g.standard_normal((n, n)) * 0.3
        a = 1.0 + 0.5 * np.tanh(_box5(u))
        systems = []
        for j in range(16):
            f = complex_normal(g, (n, n))
            zt = complex_normal(g, (n, n))
            if j < count:
                systems.append(SystemSpec(n, 2, a, complex(alpha[j], beta[j]),
                                          f, zt))
        return Workload("c5", f"adjoint: 2-D n={n}, {count} shifts, "
                        "a=1+0.5 tanh(box5(u)), L=sum||z-z_t||^2",
                        systems, share_coefficient=True)
    raise ValueError(f"unknown workload {name!r}")


def paper_shifts_table1():
    """(alpha, beta) column headers of the paper's Table 1."""
    return [(100, 100), (-100, -100), (100, -100), (-100, 100), (-100, 1),
            (1, -100)]


def paper_shifts_table2():
    """(alpha, beta) column headers of the paper's Table 2."""
    return [(-600, 150), (-100, -25), (100, -100), (-100, 100), (-100, 1),
            (1, -100)]


def grid_h(n: int, length: float = 1.0) -> float:
    return length / (n + 1)


def describe(w: Workload) -> str:
    m = sum(s.a.size for s in w.systems)
    return f"{w.name}: {len(w.systems)} system(s), {m} points, {w.description}"


if __name__ == "__main__":  # pragma: no cover
    for nm in WORKLOAD_NAMES:
        w = workload(nm, n_override=15, count_override=4)
        print(describe(w), math.isfinite(float(w.systems[0].a.sum())))
