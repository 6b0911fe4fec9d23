"""Pins of the HBS oracle (sections 6-8) against facts the paper and linear algebra fix.

* A matrix whose off-diagonal blocks have known rank (a sum of lower and upper
  rank-r semiseparable parts plus a diagonal, built here without the oracle):
  every node's rank is at most 2r (r on the first and last leaves, which have
  neighbours on one side only), the telescoping factorization (eq:tele1 -
  eq:tele3) rebuilds the matrix, and the telescoping product equals H x.
* Algorithms 3 and 4 against LAPACK's dense solve of the same matrix, for one
  level (where they reduce to eq:woodbury) and for several.
* The root DtN of a 16 x 16-leaf problem at tolerance 1e-10: section 8 states
  ranks between 10 and 80 for non-oscillatory problems at that tolerance.
* ``low_rank`` on an exactly rank-5 matrix.
"""
import numpy as np
import pytest

import hps_inputs as hi
from oracle import hbs

from .helpers import oracle_problem


def semiseparable(M, r, seed):
    rng = np.random.default_rng(seed)
    u, v, p, q = (rng.standard_normal((M, r)) for _ in range(4))
    return np.tril(u @ v.T, -1) + np.triu(p @ q.T, 1) + np.diag(10.0 + M * rng.random(M))


@pytest.mark.parametrize("M,L,r", [(64, 1, 2), (256, 4, 3), (240, 3, 5)])
def test_semiseparable_ranks_and_reconstruction(M, L, r):
    H = semiseparable(M, r, seed=M + r)
    F = hbs.compress(H, L, tol=1e-13)
    rk = hbs.ranks(F)
    assert max(rk.values()) <= 2 * r
    # The first leaf's block row only reaches to its right: rank r.
    assert rk[(L, 0)] == r
    scale = np.abs(H).max()
    assert np.abs(hbs.to_dense(F) - H).max() <= 1e-13 * scale
    x = np.random.default_rng(1).standard_normal(M)
    assert np.abs(hbs.apply(F, x) - H @ x).max() <= 1e-13 * np.abs(H @ x).max()


@pytest.mark.parametrize("L", [1, 2, 4])
def test_inverse_matches_dense_solve(L):
    H = semiseparable(256, 3, seed=7)
    F = hbs.compress(H, L, tol=1e-14)
    x = np.random.default_rng(2).standard_normal(256)
    ref = np.linalg.solve(H, x)
    y = hbs.solve(hbs.invert(F), x)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_inverse_of_random_factors():
    """Factors that are not a compression: Algorithm 4 inverts the matrix that the
    telescoping factorization defines."""
    L, m, k = 3, 20, 6
    from .helpers import hbs_oracle_factors
    F = hbs_oracle_factors(hi.hbs_factors(5, L, m, k), L, m, k)
    H = hbs.to_dense(F)
    x = np.random.default_rng(3).standard_normal(m << L)
    ref = np.linalg.solve(H, x)
    assert np.abs(hbs.solve(hbs.invert(F), x) - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(hbs.apply(F, x) - H @ x).max() <= 1e-13 * np.abs(H @ x).max()


def test_root_dtn_ranks_in_the_stated_range():
    pr = hi.laplace_log(nleaf=(16, 16), p=12, q=10)
    op, C, f, grid = oracle_problem(pr, keep=False)
    T = op.rootT
    F = hbs.compress(T, 4, tol=1e-10)
    rk = list(hbs.ranks(F).values())
    assert 10 <= min(rk) and max(rk) <= 80
    x = np.random.default_rng(4).standard_normal(T.shape[0])
    assert np.abs(hbs.apply(F, x) - T @ x).max() <= 1e-9 * np.abs(T @ x).max()


def test_low_rank_exact():
    rng = np.random.default_rng(6)
    A = rng.standard_normal((120, 5)) @ rng.standard_normal((5, 300))
    X, Y = hbs.low_rank(A, 1e-12)
    assert X.shape[1] == 5
    assert np.abs(X @ Y - A).max() <= 1e-12 * np.abs(A).max()
