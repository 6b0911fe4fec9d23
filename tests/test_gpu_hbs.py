"""HBS matrices on the device (sections 6-7) through the C ABI against the oracle.

Seeded random factors (hps_inputs.hbs_factors) go to both sides; the library
runs the telescoping product, Algorithm 3 and Algorithm 4 on its own kernels and
the oracle (oracle.hbs) in NumPy.  Every entry of y = H x, of the inverse
factors E, F*, G of every level and of y = H^-1 x is compared (relative
max-norm, 1e-12 for the product, 1e-10 for the inversion, which multiplies
rounding by the conditioning of the blocks it inverts).  Sizes cover one level,
ragged blocks (m and k off the 16- and 64-wide tiles) and several right-hand
sides; a singular leaf block must give HPS_ESINGULAR.
"""
import numpy as np
import pytest

import hps_inputs as hi
from oracle import hbs

from .helpers import hbs_oracle_factors, rel_err, say

pytestmark = pytest.mark.gpu

# (L, m, k, nrhs); 11 right-hand sides take two column chunks of the pass, and at
# k = 30 with 70 right-hand sides a parent's hat blocks (2k x nrhs) exceed the pass's
# LDS staging and are read from memory row by row.
CASES = [(1, 16, 4, 1), (3, 40, 12, 3), (4, 100, 30, 5), (5, 64, 24, 2), (6, 160, 48, 1),
         (3, 48, 16, 11), (3, 64, 30, 70)]


@pytest.fixture(scope="module")
def H(gpu):
    import paper_1307_2665_amd as H
    return H


def _setup(H, gpu, L, m, k, seed):
    import torch
    fac = hi.hbs_factors(seed, L, m, k)
    buf = H.hbs_pack(fac["D"], fac["U"], fac["Vt"], fac["Up"], fac["Vtp"], fac["B"])
    assert buf.size == H.hbs_sizes(L, m, k)[0]
    return fac, torch.from_numpy(buf).to(gpu), hbs_oracle_factors(fac, L, m, k)


@pytest.mark.parametrize("L,m,k,nrhs", CASES)
def test_apply_matches_oracle(H, gpu, L, m, k, nrhs):
    import torch
    say(f"hbs apply L={L} m={m} k={k} nrhs={nrhs}")
    fac, d_fac, F = _setup(H, gpu, L, m, k, seed=100 + L)
    x = np.random.default_rng(L).standard_normal((m << L, nrhs))
    y = H.hbs_apply(d_fac, torch.from_numpy(x).to(gpu), L, m, k).cpu().numpy()
    ref = np.stack([hbs.apply(F, x[:, c]) for c in range(nrhs)], axis=1)
    assert rel_err(y, ref) <= 1e-12


@pytest.mark.parametrize("L,m,k,nrhs", CASES)
def test_invert_and_solve_match_oracle(H, gpu, L, m, k, nrhs):
    import torch
    say(f"hbs invert/solve L={L} m={m} k={k} nrhs={nrhs}")
    fac, d_fac, F = _setup(H, gpu, L, m, k, seed=200 + L)
    inv = H.hbs_invert(d_fac, L, m, k)
    Fi = hbs.invert(F)
    E, Fs, G = H.hbs_unpack_inverse(inv.cpu().numpy(), L, m, k)
    worst = 0.0
    for l in range(1, L + 1):
        for j in range(1 << l):
            worst = max(worst, rel_err(E[l][j], Fi["E"][(l, j)]), rel_err(Fs[l][j], Fi["Fs"][(l, j)]),
                        rel_err(G[l][j], Fi["G"][(l, j)]))
    worst = max(worst, rel_err(G[0], Fi["G"][(0, 0)]))
    assert worst <= 1e-10
    x = np.random.default_rng(L + 50).standard_normal((m << L, nrhs))
    dx = torch.from_numpy(x).to(gpu)
    y = H.hbs_solve(inv, dx, L, m, k)
    ref = np.stack([hbs.solve(Fi, x[:, c]) for c in range(nrhs)], axis=1)
    assert rel_err(y.cpu().numpy(), ref) <= 1e-10
    # H (H^-1 x) = x on the device.
    back = H.hbs_apply(d_fac, y, L, m, k).cpu().numpy()
    assert rel_err(back, x) <= 1e-10


def test_singular_leaf_block_is_reported(H, gpu):
    import torch
    L, m, k = 2, 32, 8
    fac = hi.hbs_factors(7, L, m, k)
    fac["D"][1] = 0.0
    buf = H.hbs_pack(fac["D"], fac["U"], fac["Vt"], fac["Up"], fac["Vtp"], fac["B"])
    with pytest.raises(H.HpsError) as e:
        H.hbs_invert(torch.from_numpy(buf).to(gpu), L, m, k)
    assert e.value.status == H.HPS_ESINGULAR


def _samples(gpu, M, k, seed):
    import torch
    rng = np.random.default_rng(seed)
    om = torch.from_numpy(rng.standard_normal((M, k))).to(gpu)
    pt = torch.from_numpy(rng.standard_normal((k, M))).to(gpu)
    return om, pt


def _semiseparable(M, r, seed):
    rng = np.random.default_rng(seed)
    u, v, p, q = (rng.standard_normal((M, r)) for _ in range(4))
    return np.tril(u @ v.T, -1) + np.triu(p @ q.T, 1) + np.diag(10.0 + M * rng.random(M))


@pytest.mark.parametrize("M,L,r,k", [(512, 3, 3, 8), (480, 4, 2, 10), (128, 1, 4, 12)])
def test_compress_recovers_a_low_rank_structure(H, gpu, M, L, r, k):
    """Off-diagonal block rows and columns of rank <= 2r <= k: the randomized
    bases span them exactly, so the compressed matrix equals H to rounding;
    bases are orthonormal, D is copied, and Algorithms 3 and 4 on the compressed
    factors solve H y = x (LAPACK reference)."""
    import torch
    say(f"hbs compress M={M} L={L} r={r} k={k}")
    Hm = _semiseparable(M, r, seed=M + k)
    m = M >> L
    om, pt = _samples(gpu, M, k, seed=k)
    fac = H.hbs_compress(torch.from_numpy(Hm).to(gpu), L, k, om, pt)
    x = np.random.default_rng(9).standard_normal((M, 2))
    y = H.hbs_apply(fac, torch.from_numpy(x).to(gpu), L, m, k).cpu().numpy()
    assert rel_err(y, Hm @ x) <= 1e-12
    f = fac.cpu().numpy()
    nl = 1 << L
    D = f[:nl * m * m].reshape(nl, m, m)
    U = f[nl * m * m:nl * m * (m + k)].reshape(nl, m, k)
    Vt = f[nl * m * (m + k):nl * m * (m + 2 * k)].reshape(nl, k, m)
    for j in range(nl):
        assert np.array_equal(D[j], Hm[j * m:(j + 1) * m, j * m:(j + 1) * m])
        assert np.abs(U[j].T @ U[j] - np.eye(k)).max() <= 1e-13
        assert np.abs(Vt[j] @ Vt[j].T - np.eye(k)).max() <= 1e-13
    inv = H.hbs_invert(fac, L, m, k)
    ys = H.hbs_solve(inv, torch.from_numpy(x).to(gpu), L, m, k).cpu().numpy()
    assert rel_err(ys, np.linalg.solve(Hm, x)) <= 1e-10


def test_compress_root_dtn(H, gpu):
    """The root DtN of a built operator in HBS form (Remark 8.2 at the root):
    the compressed T_apply matches the dense root DtN to within a small multiple
    of the error of the best bases of the same rank (oracle: truncated SVDs)."""
    import torch
    pr = hi.laplace_log(nleaf=(16, 16), p=12, q=10)
    from .helpers import library_inputs
    C, f = library_inputs(pr)
    op = H.build_solution_operator(torch.from_numpy(C).to(gpu), pr.box, pr.nleaf, pr.p, pr.q)
    T = op.export_root_dtn()
    M, L, k = T.shape[0], 3, 60
    m = M >> L
    say(f"hbs root DtN M={M} L={L} k={k}")
    om, pt = _samples(gpu, M, k, seed=5)
    fac = H.hbs_compress(op, L, k, om, pt)
    x = np.random.default_rng(10).standard_normal((M, 3))
    y = H.hbs_apply(fac, torch.from_numpy(x).to(gpu), L, m, k).cpu().numpy()
    err = rel_err(y, T @ x)
    best = hbs.compress(T, L, rank=k)
    err_svd = rel_err(np.stack([hbs.apply(best, x[:, c]) for c in range(3)], axis=1), T @ x)
    say(f"  randomized {err:.2e}, truncated SVD {err_svd:.2e}")
    assert err <= max(100 * err_svd, 1e-12) and err <= 1e-8


def test_replayed_passes_match_each_time(H, gpu):
    """The apply and solve passes are recorded into a graph on the first call and
    replayed afterwards: every replay, with new right-hand sides written into the
    same buffers and other device work in between, matches the oracle."""
    import torch
    L, m, k, nrhs = 4, 48, 12, 2
    fac, d_fac, F = _setup(H, gpu, L, m, k, seed=300)
    Fi = hbs.invert(F)
    inv = H.hbs_invert(d_fac, L, m, k)
    dx = torch.empty((m << L, nrhs), dtype=torch.float64, device=gpu)
    y = torch.empty_like(dx)
    z = torch.empty_like(dx)
    for rep in range(4):
        x = np.random.default_rng(400 + rep).standard_normal((m << L, nrhs))
        dx.copy_(torch.from_numpy(x))
        H.hbs_apply(d_fac, dx, L, m, k, y)
        torch.cuda.synchronize()
        ref = np.stack([hbs.apply(F, x[:, c]) for c in range(nrhs)], axis=1)
        assert rel_err(y.cpu().numpy(), ref) <= 1e-12, rep
        H.hbs_solve(inv, dx, L, m, k, z)
        ref = np.stack([hbs.solve(Fi, x[:, c]) for c in range(nrhs)], axis=1)
        assert rel_err(z.cpu().numpy(), ref) <= 1e-10, rep
        # Unrelated device work between replays.
        (torch.ones(4096, device=gpu, dtype=torch.float64) * rep).sum().item()
        H.hbs_invert(d_fac, L, m, k, inv)
