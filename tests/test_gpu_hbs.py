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

CASES = [(1, 16, 4, 1), (3, 40, 12, 3), (4, 100, 30, 5), (5, 64, 24, 2), (6, 160, 48, 1)]


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
