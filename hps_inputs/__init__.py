"""Seeded synthetic inputs for the composite spectral solver.

This module is the only code shared by the CPU oracle, the GPU tests and the
benchmark. It holds none of the solver's arithmetic: it only draws seeded random
numbers and evaluates closed-form coefficient and boundary functions at points
that the caller supplies (each side computes its own node coordinates).

Coefficients follow the operator of eq:defA (section 1.1),

    A u = -c11 u_11 - 2 c12 u_12 - c22 u_22 + c1 u_1 + c2 u_2 + c u,

so the six fields are returned in the order (c11, c12, c22, c1, c2, c).

Recipes (all on the unit square):

* ``fourier_field(rng)``: g(x) = (1/8) sum_{j=1..8} cos(2 pi k_j . x + phi_j)
  with k_j drawn uniformly from {-4..4}^2 minus the origin and phi_j ~ U[0, 2 pi),
  both from ``numpy.random.default_rng``; |g| <= 1.
* Laplace with u = log|x - (1.5, 1.5)| (harmonic, smooth on the closed square).
* Convection-diffusion: c11 = c22 = 1 + g/2, c1 = c2 = 10 h (g, h independent
  fields), c = 0; boundary data cos(2 x1)(1 - 2 x2) (the data used in the
  paper's section 9.2 examples).
* Variable Helmholtz: c11 = c22 = 1, c = -kappa^2 (1 - b), kappa = 40,
  b(x) = 0.5 exp(-|x - (0.5, 0.5)|^2 / (2 * 0.1^2)).
* Sweep fields: c11 = c22 = 1 + g/2, c = 1 + g' (g, g' independent).
* Paper section 9.2 problems (constant convection, variable Helmholtz,
  diffusion-convection) converted from the sign convention of eq:example,
  -Lap u - c1 u_1 - c2 u_2 - c u = 0, to the one of eq:defA by negating
  c1, c2 and c.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Sequence

import numpy as np

NCOEF = 6  # c11, c12, c22, c1, c2, c


@dataclasses.dataclass(frozen=True)
class FourierField:
    """g(x) = (1/8) sum_j cos(2 pi (k_j . x) + phi_j); eight modes."""

    k: np.ndarray    # [8, 2] integer wave vectors
    phi: np.ndarray  # [8] phases

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        out = np.zeros(np.broadcast(x, y).shape)
        for (kx, ky), ph in zip(self.k, self.phi):
            out += np.cos(2.0 * np.pi * (kx * x + ky * y) + ph)
        return out / len(self.phi)


def fourier_field(rng: np.random.Generator, nmodes: int = 8) -> FourierField:
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(-4, 5, size=2)
        if k[0] == 0 and k[1] == 0:
            continue
        ks.append(k)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    return FourierField(np.array(ks, dtype=np.int64), phi)


def field_from_seed(seed: int) -> FourierField:
    return fourier_field(np.random.default_rng(seed))


# ---------------------------------------------------------------------------
# Problem description: six coefficient callables plus a boundary function.
# ---------------------------------------------------------------------------

CoefFn = Callable[[np.ndarray, np.ndarray], np.ndarray]


@dataclasses.dataclass
class Problem:
    name: str
    coefs: Sequence[CoefFn]            # six callables (x, y) -> values
    box: tuple = (0.0, 1.0, 0.0, 1.0)  # x0, x1, y0, y1
    nleaf: tuple = (4, 4)              # nx, ny
    p: int = 16
    q: int = 14
    bc: List[CoefFn] = dataclasses.field(default_factory=list)  # RHS functions
    exact: CoefFn | None = None        # closed-form solution if known
    body: List[CoefFn] = dataclasses.field(default_factory=list)  # body loads g (A u = g)

    def coeffs_at(self, xy: np.ndarray) -> np.ndarray:
        """Evaluate the six fields at Chebyshev nodes.

        ``xy`` has shape [nleaf, p*p, 2]; the result has shape
        [nleaf, 6, p*p] (the layout the library takes, node a + p*b).
        """
        x = xy[..., 0]
        y = xy[..., 1]
        out = np.empty((xy.shape[0], NCOEF, xy.shape[1]), dtype=np.float64)
        for c, fn in enumerate(self.coefs):
            out[:, c, :] = np.broadcast_to(fn(x, y), x.shape)
        return out

    def body_at(self, xy: np.ndarray) -> np.ndarray:
        """Body loads [nrhs, nleaf, p*p] at every leaf's Chebyshev nodes xy [nleaf, p*p, 2]."""
        return np.stack([np.asarray(g(xy[..., 0], xy[..., 1]), dtype=np.float64)
                         * np.ones(xy.shape[:2]) for g in self.body])

    def bc_at(self, xy: np.ndarray) -> np.ndarray:
        """Boundary data [nrhs, n_bdry] at boundary points xy [n_bdry, 2]."""
        return np.stack([np.asarray(f(xy[:, 0], xy[:, 1]), dtype=np.float64)
                         * np.ones(xy.shape[0]) for f in self.bc])


def _const(v: float) -> CoefFn:
    return lambda x, y: np.full(np.broadcast(np.asarray(x), np.asarray(y)).shape, float(v))


ZERO = _const(0.0)
ONE = _const(1.0)


def log_solution(cx: float = 1.5, cy: float = 1.5) -> CoefFn:
    return lambda x, y: np.log(np.hypot(np.asarray(x) - cx, np.asarray(y) - cy))


def cos_bc(x, y):
    """f(x) = cos(2 x1)(1 - 2 x2), the boundary data of section 9.2."""
    return np.cos(2.0 * np.asarray(x)) * (1.0 - 2.0 * np.asarray(y))


def laplace_log(nleaf=(4, 4), p=16, q=14) -> Problem:
    u = log_solution()
    return Problem("laplace_log", [ONE, ZERO, ONE, ZERO, ZERO, ZERO],
                   nleaf=tuple(nleaf), p=p, q=q, bc=[u], exact=u)


def convdiff(seed_g=2001, seed_h=2002, nleaf=(64, 64), p=16, q=14, nrhs=1) -> Problem:
    g = field_from_seed(seed_g)
    h = field_from_seed(seed_h)
    a = lambda x, y: 1.0 + 0.5 * g(x, y)
    b = lambda x, y: 10.0 * h(x, y)
    bcs = [cos_bc] + [field_from_seed(900000 + seed_g * 10 + k) for k in range(1, nrhs)]
    return Problem("convdiff", [a, ZERO, a, b, b, ZERO], nleaf=tuple(nleaf), p=p, q=q, bc=bcs)


def bump(x, y):
    x = np.asarray(x)
    y = np.asarray(y)
    return 0.5 * np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2) / (2.0 * 0.1 ** 2))


def helmholtz_bump(kappa=40.0, nleaf=(128, 128), p=16, q=14, nrhs=64, seed0=3000) -> Problem:
    c = lambda x, y: -kappa ** 2 * (1.0 - bump(x, y))
    bcs = [field_from_seed(seed0 + k) for k in range(nrhs)]
    return Problem("helmholtz_bump", [ONE, ZERO, ONE, ZERO, ZERO, c],
                   nleaf=tuple(nleaf), p=p, q=q, bc=bcs)


def batched_problems(nprob=32, seed0=4000, nrhs=16) -> List[Problem]:
    """Heterogeneous batch: n ~ U{8..64}, p ~ U{12,16,20}, q = p - 2."""
    out = []
    for i in range(nprob):
        rng = np.random.default_rng(seed0 + i)
        n = int(rng.integers(8, 65))
        p = int(rng.choice([12, 16, 20]))
        g = fourier_field(rng)
        h = fourier_field(rng)
        a = (lambda g: (lambda x, y: 1.0 + 0.5 * g(x, y)))(g)
        b = (lambda h: (lambda x, y: 10.0 * h(x, y)))(h)
        bcs = [field_from_seed(400000 + 100 * i + k) for k in range(nrhs)]
        out.append(Problem(f"batch{i}", [a, ZERO, a, b, b, ZERO], nleaf=(n, n), p=p, q=p - 2, bc=bcs))
    return out


def sweep_field(seed: int, nleaf=(256, 256), p=12, q=10) -> Problem:
    rng = np.random.default_rng(seed)
    g = fourier_field(rng)
    g2 = fourier_field(rng)
    a = lambda x, y: 1.0 + 0.5 * g(x, y)
    c = lambda x, y: 1.0 + g2(x, y)
    return Problem(f"sweep{seed}", [a, ZERO, a, ZERO, ZERO, c], nleaf=tuple(nleaf), p=p, q=q,
                   bc=[cos_bc])


def paper_constant_convection(nleaf=(64, 64), p=21, q=20) -> Problem:
    """Section 9.2, constant convection: c2 = -1e5 in eq:example, i.e. +1e5 in eq:defA."""
    return Problem("const_conv", [ONE, ZERO, ONE, ZERO, _const(1.0e5), ZERO],
                   nleaf=tuple(nleaf), p=p, q=q, bc=[cos_bc])


def paper_diffusion_convection(nleaf=(64, 64), p=21, q=20) -> Problem:
    """Section 9.2: c1 = -1e4 cos(4 pi x2), c2 = -1e4 cos(4 pi x1) in eq:example."""
    c1 = lambda x, y: 1.0e4 * np.cos(4.0 * np.pi * np.asarray(y)) + 0.0 * np.asarray(x)
    c2 = lambda x, y: 1.0e4 * np.cos(4.0 * np.pi * np.asarray(x)) + 0.0 * np.asarray(y)
    return Problem("diff_conv", [ONE, ZERO, ONE, c1, c2, ZERO], nleaf=tuple(nleaf), p=p, q=q,
                   bc=[cos_bc])


def paper_variable_helmholtz(nleaf=(64, 64), p=21, q=20, kappa=640.0) -> Problem:
    """Section 9.2: c = kappa^2 (1 - (sin 4 pi x1 sin 4 pi x2)^2) in eq:example."""
    c = lambda x, y: -kappa ** 2 * (1.0 - (np.sin(4 * np.pi * np.asarray(x))
                                           * np.sin(4 * np.pi * np.asarray(y))) ** 2)
    return Problem("var_helm", [ONE, ZERO, ONE, ZERO, ZERO, c], nleaf=tuple(nleaf), p=p, q=q,
                   bc=[cos_bc])


def manufactured_variable(nleaf=(2, 2), p=12, q=10, seed=11) -> Problem:
    """Variable-coefficient problem with a known smooth solution.

    u = 2 + x^2 y - x y^2 + 0.5 x^3 (positive on the unit square); the
    coefficients c11, c12, c22, c1, c2 are seeded smooth fields and c is chosen
    so that A u = 0 pointwise: c = (c11 u_11 + 2 c12 u_12 + c22 u_22
    - c1 u_1 - c2 u_2) / u.  Since u is a cubic, the discrete solution is exact
    up to rounding once p, q >= 4.
    """
    rng = np.random.default_rng(seed)
    g = [fourier_field(rng) for _ in range(5)]
    c11 = lambda x, y: 1.0 + 0.3 * g[0](x, y)
    c12 = lambda x, y: 0.2 * g[1](x, y)
    c22 = lambda x, y: 1.0 + 0.3 * g[2](x, y)
    c1 = lambda x, y: 2.0 * g[3](x, y)
    c2 = lambda x, y: 2.0 * g[4](x, y)
    u = lambda x, y: 2.0 + x * x * y - x * y * y + 0.5 * x ** 3
    ux = lambda x, y: 2.0 * x * y - y * y + 1.5 * x * x
    uy = lambda x, y: x * x - 2.0 * x * y
    uxx = lambda x, y: 2.0 * y + 3.0 * x
    uxy = lambda x, y: 2.0 * x - 2.0 * y
    uyy = lambda x, y: -2.0 * x

    def c(x, y):
        x = np.asarray(x)
        y = np.asarray(y)
        return (c11(x, y) * uxx(x, y) + 2 * c12(x, y) * uxy(x, y) + c22(x, y) * uyy(x, y)
                - c1(x, y) * ux(x, y) - c2(x, y) * uy(x, y)) / u(x, y)

    return Problem("manufactured", [c11, c12, c22, c1, c2, c], nleaf=tuple(nleaf), p=p, q=q,
                   bc=[u], exact=u)


def manufactured_body(nleaf=(3, 2), p=12, q=10, seed=12) -> Problem:
    """Body load with a known solution: A u = g with all six coefficients
    seeded smooth fields (c too) and u = 1 + x^3 - 2 x y^2 + x^2 y - 3 y^3;
    g = A u in closed form.  u is a cubic, so the discrete solution is exact up
    to rounding once p, q >= 4."""
    rng = np.random.default_rng(seed)
    f = [fourier_field(rng) for _ in range(6)]
    c11 = lambda x, y: 1.0 + 0.3 * f[0](x, y)
    c12 = lambda x, y: 0.2 * f[1](x, y)
    c22 = lambda x, y: 1.0 + 0.3 * f[2](x, y)
    c1 = lambda x, y: 2.0 * f[3](x, y)
    c2 = lambda x, y: 2.0 * f[4](x, y)
    c = lambda x, y: 1.0 + 0.5 * f[5](x, y)
    u = lambda x, y: 1.0 + x ** 3 - 2.0 * x * y * y + x * x * y - 3.0 * y ** 3
    ux = lambda x, y: 3.0 * x * x - 2.0 * y * y + 2.0 * x * y
    uy = lambda x, y: -4.0 * x * y + x * x - 9.0 * y * y
    uxx = lambda x, y: 6.0 * x + 2.0 * y
    uxy = lambda x, y: -4.0 * y + 2.0 * x
    uyy = lambda x, y: -4.0 * x - 18.0 * y

    def g(x, y):
        x = np.asarray(x)
        y = np.asarray(y)
        return (-c11(x, y) * uxx(x, y) - 2.0 * c12(x, y) * uxy(x, y) - c22(x, y) * uyy(x, y)
                + c1(x, y) * ux(x, y) + c2(x, y) * uy(x, y) + c(x, y) * u(x, y))

    return Problem("manufactured_body", [c11, c12, c22, c1, c2, c], nleaf=tuple(nleaf), p=p, q=q,
                   bc=[u], exact=u, body=[g])


def rhs_fields(seeds: Sequence[int]) -> List[FourierField]:
    return [field_from_seed(int(s)) for s in seeds]


def hbs_factors(seed: int, L: int, m: int, k: int) -> dict:
    """Seeded random factors of an HBS matrix of m 2^L rows and rank k, in the blocks
    of the library's factor buffer: D [2^L, m, m], U [2^L, m, k], Vt [2^L, k, m],
    Up[l] [2^l, 2k, k] and Vtp[l] [2^l, k, 2k] for l = 1 .. L-1, B[l] [2^l, 2k, 2k]
    for l = 0 .. L-1 (diagonal k x k blocks zero).

    Recipe: D = m I + N(0, 1); basis entries N(0, 1/rows); each row basis is the
    column basis plus a quarter of an independent draw of the same scale, so the
    k x k products V* D^-1 U stay well away from singular; the children's
    interaction blocks N(0, 1)."""
    rng = np.random.default_rng(seed)
    nl = 1 << L
    D = m * np.eye(m)[None] + rng.standard_normal((nl, m, m))
    U = rng.standard_normal((nl, m, k)) / np.sqrt(m)
    Vt = np.ascontiguousarray(
        (U + 0.25 * rng.standard_normal((nl, m, k)) / np.sqrt(m)).transpose(0, 2, 1))
    Up, Vtp, B = {}, {}, {}
    for l in range(L - 1, 0, -1):
        Up[l] = rng.standard_normal((1 << l, 2 * k, k)) / np.sqrt(2 * k)
        Vtp[l] = np.ascontiguousarray(
            (Up[l] + 0.25 * rng.standard_normal((1 << l, 2 * k, k)) / np.sqrt(2 * k))
            .transpose(0, 2, 1))
    for l in range(L - 1, -1, -1):
        b = rng.standard_normal((1 << l, 2 * k, 2 * k))
        b[:, :k, :k] = 0.0
        b[:, k:, k:] = 0.0
        B[l] = b
    return dict(D=D, U=U, Vt=Vt, Up=Up, Vtp=Vtp, B=B)
