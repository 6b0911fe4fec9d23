"""Heterogeneous batches: one build and one solve launch sequence for many problems.

Small batches are compared element by element with the oracle (1e-10); the
full 32-problem workload (n in [8, 64], p in {12, 16, 20}, q = p - 2, 16 seeded
right-hand sides each) is checked on sampled leaves: the leaf DtNs against the
oracle and the oracle's flux-matching equations evaluated on the GPU solution.
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


def _t(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


# queue: the merges' products as one persistent launch over a largest-first tile
# queue; small: levels of interfaces up to 20 nodes as whole merges per workgroup.
@pytest.mark.parametrize("queue,small", [(1, 1), (0, 0), (1, 0)])
def test_small_heterogeneous_batch_matches_oracle(H, gpu, queue, small):
    probs = [hi.convdiff(seed_g=11, seed_h=12, nleaf=(3, 5), p=8, q=6, nrhs=2),
             hi.convdiff(seed_g=13, seed_h=14, nleaf=(4, 4), p=10, q=8, nrhs=1),
             hi.laplace_log(nleaf=(2, 1), p=12, q=10),
             hi.helmholtz_bump(nleaf=(6, 6), p=10, q=8, nrhs=3),
             hi.manufactured_variable(nleaf=(5, 3), p=8, q=6),
             hi.convdiff(seed_g=15, seed_h=16, nleaf=(12, 9), p=12, q=10, nrhs=1)]
    say(f"small batch (queue {queue}, small merges {small}): " +
        ", ".join(f"{p.name}{p.nleaf}p{p.p}" for p in probs))
    inputs = [library_inputs(p) for p in probs]
    H.tune_set("gemm_queue", queue)
    H.tune_set("merge_small", small)
    try:
        ops = H.build_batch([dict(coeffs=_t(C, gpu), box=p.box, nleaf=p.nleaf, p=p.p, q=p.q)
                             for p, (C, f) in zip(probs, inputs)])
    finally:
        H.tune_set("gemm_queue", -1)
        H.tune_set("merge_small", -1)
    us = H.solve_batch(ops, [_t(f, gpu) for (C, f) in inputs])
    for p, op, u in zip(probs, ops, us):
        op_o, C_o, f_o, grid = oracle_problem(p)
        u_o = hps.solve(op_o, f_o)
        e = max(rel_err(u.cpu().numpy()[k], u_o[k]) for k in range(u_o.shape[0]))
        eT = rel_err(op.export_root_dtn(), op_o.rootT)
        say(f"  {p.name}: u {e:.2e}, root T {eT:.2e}")
        assert e < 1e-10 and eT < 1e-10


def test_config4_batch_sampled(H, gpu):
    import torch
    probs = hi.batched_problems()
    say("config4: " + " ".join(f"{p.nleaf[0]}/{p.p}" for p in probs))
    inputs = [library_inputs(p) for p in probs]
    ops = H.build_batch([dict(coeffs=_t(C, gpu), box=p.box, nleaf=p.nleaf, p=p.p, q=p.q)
                         for p, (C, f) in zip(probs, inputs)])
    us = H.solve_batch(ops, [_t(f, gpu) for (C, f) in inputs])
    torch.cuda.synchronize()
    say("config4 built and solved; sampling")
    rng = np.random.default_rng(4)
    for i in rng.choice(len(probs), size=4, replace=False):
        pr, op = probs[i], ops[i]
        n, q = pr.nleaf[0], pr.q
        u = us[i].cpu().numpy()
        assert u.shape == (16, op.N)
        grid = hps.Grid(pr.box, n, n, q)
        Co = pr.coeffs_at(grid.cheb_xy(pr.p))
        mats = hps.leaf_matrices(pr.p, q, grid.hx, grid.hy)
        for k in rng.choice(n * n, size=3, replace=False):
            a, b = int(k % n), int(k // n)
            T = hps.leaf_dtn(Co[k], pr.p, q, grid.hx, grid.hy, mats).T
            assert rel_err(op.export_leaf_dtn(int(k)), T) < 1e-10
            if a + 1 < n:
                Te = hps.leaf_dtn(Co[k + 1], pr.p, q, grid.hx, grid.hy, mats).T
                v1 = (T @ u[:, grid.boundary(a, a + 1, b, b + 1)].T).T
                v2 = (Te @ u[:, grid.boundary(a + 1, a + 2, b, b + 1)].T).T
                jump = np.max(np.abs(v1[:, q:2 * q] - v2[:, 3 * q:]))
                scale = np.max(np.abs(T)) * np.max(np.abs(u))
                assert jump < 1e-10 * scale, (i, k, jump / scale)
        say(f"  problem {i} (n={n}, p={pr.p}) ok")
    # a batched build equals the single-problem build of the same problem
    j = int(np.argmin([p.nleaf[0] for p in probs]))
    single = H.build_solution_operator(_t(inputs[j][0], gpu), probs[j].box, probs[j].nleaf,
                                       probs[j].p, probs[j].q)
    assert rel_err(single.export_root_dtn(), ops[j].export_root_dtn()) < 1e-12
