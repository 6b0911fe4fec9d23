"""hps_interface_residual_noalloc (the entry point that allocates nothing)
against hps_interface_residual, through the C ABI: two calls in a row, the
second with a smaller input, plus the size limit."""
import numpy as np
import pytest

import hps_inputs as hi

from .helpers import library_inputs, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H(gpu):
    import paper_1307_2665_amd as H
    return H


def _op(H, gpu, pr):
    import torch
    C, _ = library_inputs(pr)
    Cd = torch.as_tensor(C, dtype=torch.float64, device=gpu)
    return H.build_solution_operator(Cd, pr.box, pr.nleaf, pr.p, pr.q)


def test_noalloc_residual_matches_allocating_entry_point(H, gpu):
    import torch
    rng = np.random.default_rng(77)
    cases = [(hi.convdiff(nleaf=(8, 6), p=12, q=10), 5),     # larger first
             (hi.laplace_log(nleaf=(3, 2), p=10, q=8), 2)]     # then a smaller input
    for pr, nrhs in cases:
        op = _op(H, gpu, pr)
        u = torch.as_tensor(rng.standard_normal((nrhs, op.N)), dtype=torch.float64, device=gpu)
        ref = op.interface_residual(u)
        r = torch.full_like(u, np.nan)
        op.interface_residual_noalloc(u, r)
        torch.cuda.synchronize()
        diff = float((r - ref).abs().max())
        scale = float(ref.abs().max())
        say(f"{pr.name} {pr.nleaf} nrhs {nrhs}: max |noalloc - alloc| {diff:.3e} (scale {scale:.3e})")
        assert torch.isfinite(r).all()
        assert diff <= 1e-10 * scale
        assert torch.equal(r, ref)      # same kernels, same order: identical bits


def test_noalloc_residual_rejects_oversized_input(H, gpu):
    import torch
    pr = hi.laplace_log(nleaf=(64, 64), p=6, q=4)
    op = _op(H, gpu, pr)
    cap = 64 << 20                     # HPS_NOALLOC_SCRATCH_BYTES
    per_rhs = 64 * 64 * 4 * pr.q * 8   # one right-hand side's leaf fluxes
    nrhs = cap // per_rhs + 1
    u = torch.zeros((nrhs, op.N), dtype=torch.float64, device=gpu)
    r = torch.zeros_like(u)
    with pytest.raises(H.HpsError) as e:
        op.interface_residual_noalloc(u, r)
    say(f"oversized call rejected: {e.value}")
    assert "scratch" in str(e.value)
