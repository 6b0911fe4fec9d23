"""Post-processing (section 5.3) through the C ABI against the CPU oracle.

hps_postprocess turns the Gauss-node solution into values on every leaf's
p x p Chebyshev grid with the leaf solution operators the build kept.  Each
case compares every leaf with the oracle's leaf_cheb_values (1e-10, relative
max-norm per right-hand side).  Right-hand-side counts leave ragged rounds of
the kernel's right-hand-side blocks; p = 21 runs the unfused leaf path (its Z
is transposed out of the augmented systems), a batch keeps Z for leaves of
several operators in one leaf launch.
"""
import numpy as np
import pytest

import hps_inputs as hi
from oracle import hps

from .helpers import library_inputs, oracle_problem, rel_err, say

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def H(gpu):
    import paper_1307_2665_amd as H
    return H


def _t(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def _oracle_grid_values(op_o, u_o, nx, ny):
    """Oracle Chebyshev-grid values, [nrhs, nx*ny, p*p] in the library's leaf order."""
    out = np.zeros((u_o.shape[0], nx * ny, op_o.p * op_o.p))
    for j in range(ny):
        for i in range(nx):
            out[:, i + nx * j] = hps.leaf_cheb_values(op_o, u_o, hps.find_leaf(op_o, i, j))
    return out


def _check(uc, ref):
    e = max(rel_err(uc[k], ref[k]) for k in range(ref.shape[0]))
    say(f"  vs oracle {e:.2e}")
    assert e < TOL


@pytest.mark.parametrize("maker,nleaf,p,q,nrhs", [
    (hi.convdiff, (6, 5), 10, 8, 1),
    (hi.convdiff, (4, 4), 16, 14, 20),
    (hi.helmholtz_bump, (3, 5), 12, 10, 5),
    (hi.manufactured_variable, (3, 2), 21, 19, 3),
])
def test_postprocess_matches_oracle(H, gpu, maker, nleaf, p, q, nrhs):
    say(f"postprocess {maker.__name__} {nleaf} p{p} q{q} nrhs {nrhs}")
    pr = maker(nleaf=nleaf, p=p, q=q)
    op_o, C_o, f_o, grid = oracle_problem(pr)
    C, _ = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, p, q, keep_leaf_solution=True)
    f = np.random.default_rng(nrhs).standard_normal((nrhs, op.n_bdry))
    u = op.solve(_t(f, gpu))
    uc = op.postprocess(u).cpu().numpy()
    assert uc.shape == (nrhs, nleaf[0] * nleaf[1], p * p)
    _check(uc, _oracle_grid_values(op_o, hps.solve(op_o, f), *nleaf))


def test_postprocess_host_pointers_and_exact_cubic(H, gpu):
    """Host arrays in and out; the manufactured cubic is reproduced on every grid."""
    say("postprocess host pointers, manufactured cubic 4x3 p12 q10")
    pr = hi.manufactured_variable(nleaf=(4, 3), p=12, q=10)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(C, pr.box, pr.nleaf, pr.p, pr.q, keep_leaf_solution=True)
    u = op.solve(f)
    uc = op.postprocess(np.asarray(u))
    assert isinstance(uc, np.ndarray)
    xy = H.cheb_nodes(pr.box, pr.nleaf, pr.p)
    ex = pr.exact(xy[..., 0], xy[..., 1])
    e = rel_err(uc[0], ex)
    say(f"  vs exact {e:.2e}")
    assert e < TOL


def test_postprocess_batch(H, gpu):
    say("postprocess batch: 3 uneven problems")
    probs = [hi.convdiff(nleaf=(4, 3), p=10, q=8), hi.convdiff(nleaf=(5, 5), p=10, q=8),
             hi.helmholtz_bump(nleaf=(3, 4), p=12, q=10)]
    ins = [library_inputs(pr) for pr in probs]
    ops = H.build_batch([dict(coeffs=_t(C, gpu), box=pr.box, nleaf=pr.nleaf, p=pr.p, q=pr.q)
                         for pr, (C, f) in zip(probs, ins)], keep_leaf_solution=True)
    rng = np.random.default_rng(5)
    for pr, op, k in zip(probs, ops, (2, 17, 1)):
        op_o, *_ = oracle_problem(pr)
        f = rng.standard_normal((k, op.n_bdry))
        uc = op.postprocess(op.solve(_t(f, gpu))).cpu().numpy()
        _check(uc, _oracle_grid_values(op_o, hps.solve(op_o, f), *pr.nleaf))


def test_postprocess_needs_kept_operators(H, gpu):
    pr = hi.convdiff(nleaf=(2, 2), p=10, q=8)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    u = op.solve(_t(f, gpu))
    with pytest.raises(H.HpsError) as e:
        op.postprocess(u)
    assert e.value.status == H.HPS_EINVAL


def test_config2_full_size_postprocess_sampled(H, gpu):
    """64x64, p=16, q=14: on sampled leaves the grid values equal the oracle's
    leaf map (L1 on the grid boundary, -A_ii^-1 A_ie L1 inside) applied to the
    same leaf's Gauss values."""
    say("config2 full size postprocess")
    pr = hi.convdiff()
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q,
                                   keep_leaf_solution=True)
    ud = op.solve(_t(f, gpu))
    uc = op.postprocess(ud).cpu().numpy()[0]
    u = ud.cpu().numpy()[0]
    grid = hps.Grid(pr.box, 64, 64, pr.q)
    Co = pr.coeffs_at(grid.cheb_xy(pr.p))
    mats = hps.leaf_matrices(pr.p, pr.q, grid.hx, grid.hy)
    rng = np.random.default_rng(3)
    worst = 0.0
    for k in rng.choice(64 * 64, size=24, replace=False):
        i, j = int(k % 64), int(k // 64)
        lo = hps.leaf_dtn(Co[k], pr.p, pr.q, grid.hx, grid.hy, mats)
        we = lo.L1 @ u[grid.boundary(i, i + 1, j, j + 1)]
        ref = np.zeros(pr.p * pr.p)
        ref[lo.Je] = we
        ref[lo.Ji] = lo.X @ we
        worst = max(worst, rel_err(uc[k], ref))
    say(f"  sampled leaves vs oracle leaf map {worst:.2e}")
    assert worst < TOL


def test_postprocess_rows_per_lane_variants(H, gpu):
    """1, 2 and 4 grid rows per lane (ragged row chunks and right-hand-side
    rounds at p = 12, 13 right-hand sides) give identical bits and match the
    oracle."""
    say("postprocess rows-per-lane variants, convdiff 5x4 p12 q10, 13 rhs")
    pr = hi.convdiff(nleaf=(5, 4), p=12, q=10)
    op_o, *_ = oracle_problem(pr)
    C, _ = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q,
                                   keep_leaf_solution=True)
    f = np.random.default_rng(13).standard_normal((13, op.n_bdry))
    u = op.solve(_t(f, gpu))
    out = {}
    try:
        for rows in (1, 2, 4):
            H.tune_set("post_rows", rows)
            out[rows] = op.postprocess(u).cpu().numpy()
    finally:
        H.tune_set("post_rows", -1)
    assert np.array_equal(out[1], out[2]) and np.array_equal(out[1], out[4])
    _check(out[1], _oracle_grid_values(op_o, hps.solve(op_o, f), *pr.nleaf))
