"""Mixed-precision Schur products + iterative refinement against the FP64 oracle.

The mixed operators' merges form their Schur products on FP32 MFMA from hi/lo
splits (HPS_MIXED_SPLIT32) or on BF16 MFMA from three-slice splits
(HPS_MIXED_BF16X6); LU and the block-row solves stay FP64.  Solves are
refined with the interface residual of the FP64 leaf DtNs (the discrete
system the FP64 path solves exactly) until the update is below 1e-12
relative; the result must match the FP64 oracle to 1e-10.
"""
import numpy as np
import pytest

import hps_inputs as hi
from oracle import hps

from .helpers import library_inputs, oracle_problem, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H(gpu):
    import paper_1307_2665_amd as H
    return H


_MODES = {"split32": lambda H: H.HPS_MIXED_SPLIT32, "bf16x6": lambda H: H.HPS_MIXED_BF16X6}


def _build(H, gpu, pr, C, mode):
    """Mixed operator; the BF16 mode runs its slice products on every merge level
    (by default levels with short interfaces stay FP64)."""
    try:
        if mode == "bf16x6":
            H.tune_set("bf16x6_min_k", 0)
        return H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q,
                                         mode=_MODES[mode](H))
    finally:
        H.tune_set("bf16x6_min_k", -1)


def _t(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


@pytest.mark.parametrize("mode", ["split32", "bf16x6"])
@pytest.mark.parametrize("maker,nleaf", [(hi.convdiff, (16, 16)), (hi.helmholtz_bump, (16, 16)),
                                         (hi.laplace_log, (4, 4))])
def test_mixed_refined_matches_fp64_oracle(H, gpu, maker, nleaf, mode):
    kw = dict(nleaf=nleaf)
    if maker is hi.helmholtz_bump:
        kw["nrhs"] = 3
    pr = maker(**kw)
    say(f"mixed ({mode}) {pr.name} {nleaf}")
    op_o, C_o, f_o, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    op = _build(H, gpu, pr, C, mode)
    u0 = op.solve(_t(f, gpu)).cpu().numpy()
    info = {}
    u = op.solve(_t(f, gpu), refine=True, tol=1e-12, max_iter=20, info=info).cpu().numpy()
    u_o = hps.solve(op_o, f_o)
    e0 = max(rel_err(u0[k], u_o[k]) for k in range(u.shape[0]))
    e = max(rel_err(u[k], u_o[k]) for k in range(u.shape[0]))
    say(f"  unrefined err {e0:.2e}, refined err {e:.2e} after {info['iters']} sweeps")
    assert e < 1e-10
    assert info["iters"] >= 1 and info["last_update_rel"] <= 1e-12
    # the root DtN of the mixed operator is only approximate, but close
    assert rel_err(op.export_root_dtn(), op_o.rootT) < 1e-4


@pytest.mark.parametrize("mode", ["split32", "bf16x6"])
def test_refinement_reports_nonconvergence(H, gpu, mode):
    say(f"mixed ({mode}) nonconvergence")
    pr = hi.convdiff(nleaf=(8, 8))
    C, f = library_inputs(pr)
    op = _build(H, gpu, pr, C, mode)
    with pytest.raises(H.HpsError) as e:
        op.solve(_t(f, gpu), refine=True, tol=1e-30, max_iter=2)
    assert e.value.status == H.HPS_ENOTCONV


def test_fp64_refinement_is_a_no_op(H, gpu):
    """On the FP64 operator the first correction is at rounding level."""
    say("fp64 refine")
    pr = hi.convdiff(nleaf=(8, 8))
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q, keep_factors=True)
    info = {}
    op.solve(_t(f, gpu), refine=True, tol=1e-12, max_iter=3, info=info)
    assert info["first_update_rel"] < 1e-12
