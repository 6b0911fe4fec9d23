"""Conditioning reports and the relative pivot test of the build (GPU).

Reading of the paper: section 4's interface systems (T33a - T33b) u3 = ...
are assumed solvable; the build reports, per tree depth, max|M| / min |pivot|
of every merge system M (an estimate of cond(M)), and with pivot_tol > 0 it
refuses leaf systems A_ii and merge systems whose pivots fall below
pivot_tol times their largest entry.  The oracle computes the same estimate
from LAPACK's LU (oracle.hps.level_conditions).
"""
import numpy as np
import pytest

import hps_inputs as hi
from oracle import hps

from .helpers import library_inputs, oracle_problem, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H(gpu):
    import paper_1307_2665_amd as H
    return H


def _t(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def _resonant_strip(p, q):
    """-Lap u - (5/4) pi^2 u = 0 on [0,2] x [0,1] with 2 x 1 leaves: the merged box
    has the Dirichlet eigenvalue (5/4) pi^2 (mode sin(pi x/2) sin(pi y)), the unit
    leaves do not (their lowest is 2 pi^2), so only the root merge is singular
    (up to the discretization error)."""
    kap2 = 1.25 * np.pi ** 2
    return hi.Problem("resonant_strip", [hi.ONE, hi.ZERO, hi.ONE, hi.ZERO, hi.ZERO,
                                         lambda x, y: -kap2 + 0.0 * np.asarray(x)],
                      box=(0.0, 2.0, 0.0, 1.0), nleaf=(2, 1), p=p, q=q, bc=[hi.cos_bc])


@pytest.mark.parametrize("maker,nleaf", [(hi.convdiff, (8, 8)), (hi.helmholtz_bump, (8, 8)),
                                         (hi.laplace_log, (4, 4))])
def test_level_conditions_match_oracle(H, gpu, maker, nleaf):
    pr = maker(nleaf=nleaf)
    say(f"level conditions {pr.name} {nleaf}")
    op_o, _, _, _ = oracle_problem(pr)
    C, _ = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    got = op.level_conditions()
    ref = hps.level_conditions(op_o)
    assert got.shape == ref.shape and got[-1] == 0.0
    # The pivots may differ on near ties (the GPU compares rounded magnitudes),
    # which moves the smallest pivot slightly: 5% relative.
    np.testing.assert_allclose(got, ref, rtol=5e-2)


@pytest.mark.parametrize("p,q", [(12, 10), (16, 14)])
def test_singular_merge_is_reported(H, gpu, p, q):
    pr = _resonant_strip(p, q)
    say(f"resonant strip p={p} q={q}")
    op_o, _, _, _ = oracle_problem(pr)
    C, _ = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, p, q)
    est = op.level_conditions()
    assert est[0] > 1e7 and est[0] > 1e3 * est[1:].max(), est
    ref = hps.level_conditions(op_o)
    assert ref[0] / 10 < est[0] < ref[0] * 10, (est, ref)
    with pytest.raises(H.HpsError) as e:
        H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, p, q, pivot_tol=1e-6)
    assert e.value.status == H.HPS_ESINGULAR
    assert "merge of box 0" in str(e.value) and "depth 0" in str(e.value)


def test_well_conditioned_build_passes_pivot_test(H, gpu):
    pr = hi.convdiff(nleaf=(8, 8))
    C, f = library_inputs(pr)
    op_o, _, f_o, _ = oracle_problem(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q, pivot_tol=1e-6)
    u = op.solve(_t(f, gpu)).cpu().numpy()
    u_o = hps.solve(op_o, f_o)
    assert np.max(np.abs(u - u_o)) / np.max(np.abs(u_o)) < 1e-10


@pytest.mark.parametrize("p,q", [(16, 14), (21, 19), (10, 8), (12, 10)])
def test_singular_leaf_is_reported(H, gpu, p, q):
    """c = -lambda_1 of the leaf's interior collocation operator makes every A_ii
    singular to rounding; p = 21 runs the unfused leaf path, p = 10 and 12 the
    MFMA leaf kernel."""
    h = 0.25
    m = hps.leaf_matrices(p, q, h, h)
    Ji = m["Ji"]
    lam = np.min(np.linalg.eigvals(-(m["D11"] + m["D22"])[np.ix_(Ji, Ji)]).real)
    pr = hi.Problem("resonant_leaf", [hi.ONE, hi.ZERO, hi.ONE, hi.ZERO, hi.ZERO,
                                      lambda x, y: -lam + 0.0 * np.asarray(x)],
                    nleaf=(4, 4), p=p, q=q, bc=[hi.cos_bc])
    say(f"resonant leaf p={p} q={q}")
    C, _ = library_inputs(pr)
    with pytest.raises(H.HpsError) as e:
        H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, p, q, pivot_tol=1e-8)
    assert e.value.status == H.HPS_ESINGULAR and "leaf" in str(e.value)
    # Shifted away from the eigenvalue the same build passes the test.
    pr.coefs[5] = lambda x, y: -0.5 * lam + 0.0 * np.asarray(x)
    C, _ = library_inputs(pr)
    H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, p, q, pivot_tol=1e-8)
