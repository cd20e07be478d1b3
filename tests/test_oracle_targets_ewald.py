"""Pin of the oracle's structure-factor Ewald sum (a few targets from many sources), which states
the exact triply periodic sum at sampled targets of the full-size workloads: it must reproduce
the pairwise Ewald sums of oracle/periodic.py (themselves pinned by xi-independence, periodicity,
zero face flux and the rock-salt Madelung constant)."""
import numpy as np
import pytest

from oracle import _native, kernels as K, periodic


@pytest.mark.parametrize("kernel", [K.LAPLACE, K.STOKES])
def test_structure_factor_ewald_matches_pairwise_ewald(kernel):
    rng = np.random.default_rng(3)
    src = rng.random((300, 3))
    trg = np.concatenate([src[:20], rng.random((20, 3)) + [1.0, -2.0, 0.0]])   # coincident and shifted
    k = K.kdim(kernel)
    d = rng.standard_normal((2, 300, k))
    d -= d.mean(axis=1, keepdims=True)
    got = _native.tp_ewald_targets(kernel, trg, src, d)
    assert got.shape == (2, 40, k)
    for r in range(2):
        ex = periodic.exact_potential(kernel, 7, trg, src, d[r])
        assert np.max(np.abs(got[r] - ex)) < 1e-12 * np.max(np.abs(ex))
    one = _native.tp_ewald_targets(kernel, trg, src, d[1])      # one right-hand side alone
    assert np.max(np.abs(one - got[1])) < 1e-14 * np.max(np.abs(got[1]))
    # another splitting parameter gives the same sum
    other = _native.tp_ewald_targets(kernel, trg, src, d, xi=12.0)
    assert np.max(np.abs(other - got)) < 1e-12 * np.max(np.abs(got))
