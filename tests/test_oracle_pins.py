"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these re-types an oracle formula: each compares with a closed form, a
library routine used as an independent reference, an invariant stated in the
paper, or an independent brute-force assembly.
"""
import numpy as np
import pytest

import hps_inputs as hi
from oracle import brute, hps


# ---------------------------------------------------------------------------
# Nodes, differentiation, interpolation (sections 2 and 3.1).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", [4, 8, 12, 16, 21])
def test_cheb_diff_differentiates_polynomials(p):
    x = hps.cheb_points(p)
    D = hps.cheb_diff(p)
    for k in range(1, p):
        exact = k * x ** (k - 1)
        assert np.max(np.abs(D @ x ** k - exact)) <= 1e-12 * max(1.0, k * k * p)
    assert np.max(np.abs(D @ np.ones(p))) < 1e-12


def test_cheb_points_are_lobatto_extrema():
    # Chebyshev-Lobatto points are the extrema of T_{p-1}: T'_{p-1} vanishes inside.
    p = 13
    x = hps.cheb_points(p)
    assert x[0] == -1.0 and abs(x[-1] - 1.0) < 1e-15 and np.all(np.diff(x) > 0)
    dT = np.polynomial.chebyshev.Chebyshev.basis(p - 1).deriv()
    assert np.max(np.abs(dT(x[1:-1]))) < 1e-9


@pytest.mark.parametrize("q", [5, 10, 14, 21])
def test_gauss_points_integrate_exactly(q):
    g = hps.gauss_points(q)
    # Recover weights by solving the moment system and check degree 2q-1 exactness.
    V = np.vstack([g ** k for k in range(q)])
    mom = np.array([(1 - (-1) ** (k + 1)) / (k + 1) for k in range(q)])
    w = np.linalg.solve(V, mom)
    for k in range(2 * q):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(w @ g ** k - exact) < 1e-12
    assert np.all(np.abs(g) < 1) and np.all(np.diff(g) > 0)


def test_lagrange_reproduces_polynomials():
    src = hps.gauss_points(10)
    dst = hps.cheb_points(12)
    L = hps.lagrange_matrix(src, dst)
    for k in range(10):
        assert np.max(np.abs(L @ src ** k - dst ** k)) < 1e-11
    # and fails (as it must) at degree q for the extrapolated end points
    assert np.max(np.abs(L @ src ** 10 - dst ** 10)) > 1e-6


# ---------------------------------------------------------------------------
# Leaf DtN (section 3).
# ---------------------------------------------------------------------------

def _leaf_flux_exact(grid, u_x, u_y):
    xy = grid.node_xy()
    Ie = grid.boundary(0, 1, 0, 1)
    P = xy[Ie]
    q = grid.q
    return np.concatenate([u_y(*P[:q].T), u_x(*P[q:2 * q].T), u_y(*P[2 * q:3 * q].T),
                           u_x(*P[3 * q:].T)]), P


@pytest.mark.parametrize("p,q", [(16, 14), (12, 10), (16, 16), (8, 8)])
def test_leaf_harmonic_polynomial_exact(p, q):
    """A harmonic polynomial of degree <= q-1 is reproduced exactly by T (Laplace)."""
    box = (0.3, 0.55, -0.2, 0.05)
    u = lambda x, y: x ** 3 - 3 * x * y ** 2 + 2 * x * y + 1
    ux = lambda x, y: 3 * x ** 2 - 3 * y ** 2 + 2 * y
    uy = lambda x, y: -6 * x * y + 2 * x
    g = hps.Grid(box, 1, 1, q)
    coef = np.zeros((6, p * p))
    coef[0] = coef[2] = 1.0
    lo = hps.leaf_dtn(coef, p, q, g.hx, g.hy)
    vex, P = _leaf_flux_exact(g, ux, uy)
    v = lo.T @ u(P[:, 0], P[:, 1])
    assert np.max(np.abs(v - vex)) < 1e-11 * np.max(np.abs(lo.T))


def test_leaf_manufactured_variable_coefficients():
    """All six coefficients active (incl. c12): exact cubic solution is reproduced."""
    pr = hi.manufactured_variable(nleaf=(1, 1), p=12, q=10)
    box = (0.0, 0.5, 0.25, 0.75)
    g = hps.Grid(box, 1, 1, pr.q)
    coef = pr.coeffs_at(g.cheb_xy(pr.p))[0]
    lo = hps.leaf_dtn(coef, pr.p, pr.q, g.hx, g.hy)
    ux = lambda x, y: 2.0 * x * y - y * y + 1.5 * x * x
    uy = lambda x, y: x * x - 2.0 * x * y
    vex, P = _leaf_flux_exact(g, ux, uy)
    v = lo.T @ pr.exact(P[:, 0], P[:, 1])
    assert np.max(np.abs(v - vex)) < 1e-10 * np.max(np.abs(vex))


def test_leaf_constants_have_zero_flux():
    p, q = 16, 14
    rng = np.random.default_rng(0)
    coef = np.zeros((6, p * p))
    coef[0] = 1 + 0.3 * rng.random(p * p)
    coef[2] = 1 + 0.3 * rng.random(p * p)
    coef[1] = 0.1 * rng.random(p * p)
    lo = hps.leaf_dtn(coef, p, q, 0.1, 0.1)
    assert np.max(np.abs(lo.T @ np.ones(4 * q))) < 1e-10 * np.max(np.abs(lo.T))


def test_leaf_laplace_scaling():
    """For Laplace, T on an h-box equals T on a unit box divided by h."""
    p, q = 16, 14
    coef = np.zeros((6, p * p))
    coef[0] = coef[2] = 1.0
    T1 = hps.leaf_dtn(coef, p, q, 1.0, 1.0).T
    Th = hps.leaf_dtn(coef, p, q, 1 / 64, 1 / 64).T
    assert np.max(np.abs(Th * (1 / 64) - T1)) < 1e-11 * np.max(np.abs(T1))


def test_leaf_flux_sign_convention():
    """u = x2: flux v = du/dx2 = 1 on S and N, du/dx1 = 0 on E and W (section 2)."""
    p, q = 10, 8
    coef = np.zeros((6, p * p))
    coef[0] = coef[2] = 1.0
    g = hps.Grid((0, 1, 0, 1), 1, 1, q)
    lo = hps.leaf_dtn(coef, p, q, 1.0, 1.0)
    P = g.node_xy()[g.boundary(0, 1, 0, 1)]
    v = lo.T @ P[:, 1]
    np.testing.assert_allclose(v[:q], 1.0, atol=1e-11)
    np.testing.assert_allclose(v[2 * q:3 * q], 1.0, atol=1e-11)
    np.testing.assert_allclose(v[q:2 * q], 0.0, atol=1e-11)
    np.testing.assert_allclose(v[3 * q:], 0.0, atol=1e-11)


# ---------------------------------------------------------------------------
# Merges, Algorithms 1 and 2 (sections 4, 5).
# ---------------------------------------------------------------------------

def _problem_ops(pr, nleaf, **kw):
    grid = hps.Grid(pr.box, nleaf[0], nleaf[1], pr.q)
    C = pr.coeffs_at(grid.cheb_xy(pr.p))
    op = hps.build(C, pr.box, nleaf, pr.p, pr.q, **kw)
    return op, C, grid


@pytest.mark.parametrize("nleaf", [(4, 4), (3, 2), (1, 3)])
def test_hierarchical_equals_brute_force_collocation(nleaf):
    """Remark 5.1: merges are exact, so the tree solve equals one global collocation solve."""
    pr = hi.manufactured_variable(p=10, q=8, seed=5)
    pr.bc = [hi.field_from_seed(77)]
    op, C, grid = _problem_ops(pr, nleaf)
    f = pr.bc_at(hps.gamma_xy(op))
    u = hps.solve(op, f)[0]
    ub = brute.collocation_solve(C, pr.box, nleaf, pr.p, pr.q, f[0])
    assert np.max(np.abs(u - ub)) < 1e-11 * np.max(np.abs(ub))


def test_config1_brute_force_and_exact():
    pr = hi.laplace_log()
    op, C, grid = _problem_ops(pr, (4, 4))
    f = pr.bc_at(hps.gamma_xy(op))
    u = hps.solve(op, f)[0]
    ub = brute.collocation_solve(C, pr.box, (4, 4), pr.p, pr.q, f[0])
    assert np.max(np.abs(u - ub)) < 1e-11
    ex = pr.exact(*grid.node_xy().T)
    assert np.max(np.abs(u - ex)) < 1e-11


def test_root_dtn_is_schur_complement_of_interface_system():
    pr = hi.convdiff(nleaf=(3, 3), p=10, q=8)
    op, C, grid = _problem_ops(pr, (3, 3))
    T1 = brute.interface_root_dtn(op)
    assert np.max(np.abs(T1 - op.rootT)) < 1e-11 * np.max(np.abs(T1))


def test_root_dtn_independent_of_tree_shape():
    """Algorithm 1 allows any bottom-up order; the root DtN must not depend on it."""
    pr = hi.convdiff(nleaf=(4, 4), p=10, q=8)
    a, _, _ = _problem_ops(pr, (4, 4), x_first=True)
    b, _, _ = _problem_ops(pr, (4, 4), x_first=False)
    assert np.max(np.abs(a.rootT - b.rootT)) < 1e-11 * np.max(np.abs(a.rootT))


def test_root_dtn_reproduces_harmonic_flux():
    """Root DtN applied to a harmonic polynomial gives its section-2 flux on Gamma."""
    pr = hi.laplace_log(nleaf=(2, 2), p=12, q=10)
    op, _, grid = _problem_ops(pr, (2, 2))
    u = lambda x, y: x ** 3 - 3 * x * y ** 2
    ux = lambda x, y: 3 * x ** 2 - 3 * y ** 2
    uy = lambda x, y: -6 * x * y
    P = hps.gamma_xy(op)
    q, nx, ny = 10, 2, 2
    v = op.rootT @ u(*P.T)
    vex = np.concatenate([uy(*P[:nx * q].T), ux(*P[nx * q:(nx + ny) * q].T),
                          uy(*P[(nx + ny) * q:(2 * nx + ny) * q].T), ux(*P[(2 * nx + ny) * q:].T)])
    assert np.max(np.abs(v - vex)) < 1e-10 * np.max(np.abs(vex))


def test_manufactured_solution_exact_everywhere():
    pr = hi.manufactured_variable(p=12, q=10)
    op, _, grid = _problem_ops(pr, (4, 2))
    f = pr.bc_at(hps.gamma_xy(op))
    u = hps.solve(op, f)[0]
    ex = pr.exact(*grid.node_xy().T)
    assert np.max(np.abs(u - ex)) < 1e-11


def test_spectral_convergence_in_p():
    """Config-1 problem: error against log|x - (1.5,1.5)| decays geometrically with p."""
    errs = []
    for p in (6, 8, 10, 12):
        pr = hi.laplace_log(nleaf=(2, 2), p=p, q=p - 2)
        op, _, grid = _problem_ops(pr, (2, 2))
        u = hps.solve(op, pr.bc_at(hps.gamma_xy(op)))[0]
        errs.append(np.max(np.abs(u - pr.exact(*grid.node_xy().T))))
    assert all(errs[i + 1] < 0.2 * errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-7


def test_helmholtz_plane_wave():
    """-Lap u - k^2 u = 0 with c = -k^2 (eq:defA): plane waves are exact solutions."""
    k = 12.0
    d = np.array([0.6, 0.8])
    u = lambda x, y: np.cos(k * (d[0] * np.asarray(x) + d[1] * np.asarray(y)))
    pr = hi.Problem("pw", [hi.ONE, hi.ZERO, hi.ONE, hi.ZERO, hi.ZERO, hi._const(-k * k)],
                    nleaf=(4, 4), p=14, q=12, bc=[u], exact=u)
    op, _, grid = _problem_ops(pr, (4, 4))
    sol = hps.solve(op, pr.bc_at(hps.gamma_xy(op)))[0]
    assert np.max(np.abs(sol - u(*grid.node_xy().T))) < 1e-9


# ---------------------------------------------------------------------------
# Interface residual, upward pass, refinement.
# ---------------------------------------------------------------------------

def test_residual_vanishes_on_hierarchical_solution():
    pr = hi.convdiff(nleaf=(4, 4), p=10, q=8)
    op, _, _ = _problem_ops(pr, (4, 4))
    u = hps.solve(op, pr.bc_at(hps.gamma_xy(op)))
    r = hps.interface_residual(op, u)
    assert np.max(np.abs(r)) < 1e-10 * np.max(np.abs(op.leafT[len(op.boxes) - 1]))


def test_upward_with_sources_solves_interface_system():
    """Random interface sources s: hierarchical (upward + downward) vs a dense solve."""
    pr = hi.convdiff(nleaf=(3, 4), p=10, q=8)
    op, _, grid = _problem_ops(pr, (3, 4))
    rng = np.random.default_rng(3)
    gamma = op.boxes[0].Ie
    s = rng.standard_normal(grid.N)
    s[gamma] = 0.0
    z = hps.upward(op, s[None, :])
    u = hps.solve(op, np.zeros((1, len(gamma))), z=z)[0]
    # dense: jump(u) = s at interior nodes, u = 0 on gamma
    r = hps.interface_residual(op, u[None, :])[0]
    assert np.max(np.abs(r - s)) < 1e-9 * np.max(np.abs(s)) * np.max(np.abs(op.leafT[len(op.boxes) - 1]))
    # zero source gives zero correction
    z0 = hps.upward(op, np.zeros((1, grid.N)))
    assert all(np.max(np.abs(v)) == 0.0 for v in z0.values())


def test_refinement_fixes_a_perturbed_solution():
    pr = hi.convdiff(nleaf=(4, 4), p=10, q=8)
    op, _, grid = _problem_ops(pr, (4, 4))
    f = pr.bc_at(hps.gamma_xy(op))
    u = hps.solve(op, f)
    rng = np.random.default_rng(9)
    bad = u.copy()
    inner = np.setdiff1d(np.arange(grid.N), op.boxes[0].Ie)
    bad[:, inner] += 1e-3 * rng.standard_normal(len(inner))
    fixed = bad + hps.refine_step(op, bad)
    assert np.max(np.abs(fixed - u)) < 1e-11


# ---- section 5.3: post-processing on the leaf Chebyshev grids ----------------

def test_postprocess_interior_equals_global_collocation():
    """Interior grid values recovered leaf by leaf equal the interior unknowns
    of the one global collocation system (brute force)."""
    pr = hi.manufactured_variable(p=10, q=8, seed=5)
    pr.bc = [hi.field_from_seed(78)]
    nleaf = (3, 2)
    op, C, grid = _problem_ops(pr, nleaf)
    f = pr.bc_at(hps.gamma_xy(op))
    u = hps.solve(op, f)[0]
    ub, wb = brute.collocation_solve(C, pr.box, nleaf, pr.p, pr.q, f[0], with_interior=True)
    ji = hps.leaf_matrices(pr.p, pr.q, grid.hx, grid.hy)["Ji"]
    for j in range(nleaf[1]):
        for i in range(nleaf[0]):
            w = hps.leaf_cheb_values(op, u, hps.find_leaf(op, i, j))[0]
            ref = wb[i + nleaf[0] * j]
            assert np.max(np.abs(w[ji] - ref)) < 1e-11 * np.max(np.abs(ref))


def test_postprocess_reproduces_manufactured_cubic():
    """All six coefficients active: every leaf's Chebyshev grid (boundary,
    corners and interior) carries the exact cubic solution."""
    pr = hi.manufactured_variable(p=12, q=10)
    nleaf = (4, 2)
    op, _, grid = _problem_ops(pr, nleaf)
    u = hps.solve(op, pr.bc_at(hps.gamma_xy(op)))[0]
    xy = grid.cheb_xy(pr.p)
    for j in range(nleaf[1]):
        for i in range(nleaf[0]):
            w = hps.leaf_cheb_values(op, u, hps.find_leaf(op, i, j))[0]
            ex = pr.exact(*xy[i + nleaf[0] * j].T)
            assert np.max(np.abs(w - ex)) < 1e-11 * np.max(np.abs(ex))


# ---- body loads, A u = g (extension; leaf particular solutions + upward pass) -

def test_body_load_reproduces_manufactured_cubic():
    """All six coefficients active and g = A u for a cubic u: the body-load
    solve is exact at the Gauss nodes and on every leaf's Chebyshev grid."""
    pr = hi.manufactured_body(p=12, q=10)
    nleaf = (3, 2)
    op, C, grid = _problem_ops(pr, nleaf)
    g = pr.body_at(grid.cheb_xy(pr.p))
    u, wpart = hps.body_solve(op, C, pr.bc_at(hps.gamma_xy(op)), g)
    ex = pr.exact(*grid.node_xy().T)
    assert np.max(np.abs(u[0] - ex)) < 1e-11 * np.max(np.abs(ex))
    xy = grid.cheb_xy(pr.p)
    for j in range(nleaf[1]):
        for i in range(nleaf[0]):
            w = hps.body_cheb_values(op, u, hps.find_leaf(op, i, j), wpart)[0]
            exc = pr.exact(*xy[i + nleaf[0] * j].T)
            assert np.max(np.abs(w - exc)) < 1e-11 * np.max(np.abs(exc))


def test_body_load_equals_global_collocation():
    """Random smooth load and boundary data (no closed form): the hierarchical
    body-load solve equals the one global collocation system with the load on
    its interior rows, at the Gauss nodes and at every interior node."""
    pr = hi.manufactured_variable(p=10, q=8, seed=5)
    pr.bc = [hi.field_from_seed(79)]
    pr.body = [hi.field_from_seed(80)]
    nleaf = (3, 3)
    op, C, grid = _problem_ops(pr, nleaf)
    f = pr.bc_at(hps.gamma_xy(op))
    g = pr.body_at(grid.cheb_xy(pr.p))
    u, wpart = hps.body_solve(op, C, f, g)
    ub, wb = brute.collocation_solve(C, pr.box, nleaf, pr.p, pr.q, f[0], with_interior=True,
                                     body=g[0])
    assert np.max(np.abs(u[0] - ub)) < 1e-11 * np.max(np.abs(ub))
    ji = hps.leaf_matrices(pr.p, pr.q, grid.hx, grid.hy)["Ji"]
    for j in range(nleaf[1]):
        for i in range(nleaf[0]):
            w = hps.body_cheb_values(op, u, hps.find_leaf(op, i, j), wpart)[0]
            ref = wb[i + nleaf[0] * j]
            assert np.max(np.abs(w[ji] - ref)) < 1e-11 * np.max(np.abs(wb))


def test_body_load_zero_is_the_plain_solve():
    pr = hi.convdiff(nleaf=(4, 3), p=10, q=8)
    op, C, grid = _problem_ops(pr, (4, 3))
    f = np.random.default_rng(1).standard_normal((2, op.n_bdry))
    u, _ = hps.body_solve(op, C, f, np.zeros((2, 12, pr.p * pr.p)))
    assert np.max(np.abs(u - hps.solve(op, f))) < 1e-13 * np.max(np.abs(u))


# ---------------------------------------------------------------------------
# Admissible (p, q): section 3.2 step 1 and the cross-point null modes.
# ---------------------------------------------------------------------------

def _cross_point_mode(grid, p):
    """At the centre of a 2x2-leaf grid: on each of the four edges meeting
    there, the Gauss values of the degree-(p-1) polynomial that is 1 at the
    edge's Chebyshev node at the centre and 0 at its other p-1 Chebyshev
    nodes; + on the two horizontal edges, - on the two vertical ones.  Every
    leaf sees one edge of each sign at its corner there, so the corner average
    of step 1 cancels and its boundary Chebyshev values all vanish."""
    q = grid.q
    xc = hps.cheb_points(p)
    xg = hps.gauss_points(q)
    ell_end = hps.lagrange_matrix(xc, xg)[:, -1]     # 1 at the node x = +1
    ell_start = hps.lagrange_matrix(xc, xg)[:, 0]    # 1 at the node x = -1
    v = np.zeros(grid.N)
    v[grid.hedge(0, 1)] = ell_end        # west of the centre: its east end
    v[grid.hedge(1, 1)] = ell_start      # east of the centre: its west end
    v[grid.vedge(1, 0)] = -ell_end       # south of the centre: its north end
    v[grid.vedge(1, 1)] = -ell_start     # north of the centre: its south end
    return v


def test_cross_point_mode_is_invisible_only_when_q_equals_p():
    """With q = p the cross-point mode lies in the null space of all four leaf
    DtNs and of the root merge system M = T33a - T33b; with q = p - 1 the same
    construction is seen by every leaf."""
    for p, q, singular in ((8, 8, True), (12, 12, True), (12, 11, False)):
        pr = hi.laplace_log(nleaf=(2, 2), p=p, q=q)
        grid = hps.Grid(pr.box, 2, 2, q)
        op = hps.build(pr.coeffs_at(grid.cheb_xy(p)), pr.box, (2, 2), p, q, allow_singular=True)
        v = _cross_point_mode(grid, p)
        flux = max(np.max(np.abs(T @ v[op.boxes[t].Ie])) / np.max(np.abs(T))
                   for t, T in op.leafT.items())
        root = op.merges[0]
        v3 = v[op.boxes[0].Ii]
        mv = np.max(np.abs(root.M @ v3)) / (np.max(np.abs(root.M)) * np.max(np.abs(v3)))
        cond = np.linalg.cond(root.M)
        if singular:
            assert flux < 1e-12 and mv < 1e-12 and cond > 1e12, (p, q, flux, mv, cond)
        else:
            assert flux > 1e-3 and mv > 1e-3 and cond < 1e3, (p, q, flux, mv, cond)


@pytest.mark.parametrize("p", [8, 12, 16])
def test_q_equal_p_ruins_the_gauss_solution(p):
    """4x4 Laplace leaves, u = log|x - (1.5, 1.5)|: at q = p - 1 the merges are
    well conditioned and the Gauss-node solution is accurate; at q = p the
    solution is off by O(1) (the singular merges amplify rounding along the
    cross-point modes).  The oracle refuses q >= p unless asked."""
    def run(q):
        pr = hi.laplace_log(nleaf=(4, 4), p=p, q=q)
        grid = hps.Grid(pr.box, 4, 4, q)
        op = hps.build(pr.coeffs_at(grid.cheb_xy(p)), pr.box, (4, 4), p, q, allow_singular=True)
        u = hps.solve(op, pr.bc_at(hps.gamma_xy(op)))[0]
        return np.max(np.abs(u - pr.exact(*grid.node_xy().T))), hps.level_conditions(op)
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        err_bad, cond_bad = run(p)
    err_ok, cond_ok = run(p - 1)
    assert err_ok < 1e-8 and err_bad > 1e-3, (err_ok, err_bad)
    assert np.max(cond_ok) < 1e2 and np.max(cond_bad) > 1e12, (cond_ok, cond_bad)
    with pytest.raises(ValueError):
        pr = hi.laplace_log(nleaf=(2, 2), p=p, q=p)
        hps.build(pr.coeffs_at(hps.Grid(pr.box, 2, 2, p).cheb_xy(p)), pr.box, (2, 2), p, p)


def test_level_condition_estimate_brackets_cond2():
    """max|M| / min |u_kk| (the per-depth estimate both sides report) stays
    below cond_2(M) and within a factor 50 of it on a variable-coefficient
    problem (p = 16, q = 14)."""
    import scipy.linalg as sla
    pr = hi.convdiff(nleaf=(4, 4), p=16, q=14)
    op, _, _ = _problem_ops(pr, (4, 4))
    est = hps.level_conditions(op)
    for t, mo in op.merges.items():
        lu, _ = sla.lu_factor(mo.M)
        e = np.max(np.abs(mo.M)) / np.min(np.abs(np.diag(lu)))
        c2 = np.linalg.cond(mo.M)
        assert c2 / 50 < e <= c2 * (1 + 1e-12), (t, e, c2)
        assert e <= est[op.boxes[t].level]
    assert est[-1] == 0.0
