"""The seeded input generators that the oracle's tests, the GPU parity tests and the benchmark
share: determinism, points inside the unit box, shapes, and the zero net density that singly and
doubly periodic sums need (the neutrality condition of Section 2.2)."""
import numpy as np
import pytest

import workloads as W


def _small():
    probs = [W.laplace_sp_uniform(n=3000, seed=1),
             W.laplace_sp_uniform(n=3000, seed=1, mask=W.DP_XY),
             W.stokes_tp_uniform(n=3000, seed=2, n_rhs=2),
             W.stokes_dp_slab(n=3000, seed=3),
             W.stokes_tp_clustered(n=3000, seed=5)]
    probs += W.laplace_sp_batch(n_problems=3, n_rhs=2, lo=2.0, hi=3.0)
    return probs


def test_generators_are_deterministic_by_seed():
    a, b = W.stokes_tp_uniform(n=1000, seed=11), W.stokes_tp_uniform(n=1000, seed=11)
    c = W.stokes_tp_uniform(n=1000, seed=12)
    assert np.array_equal(a.points, b.points) and np.array_equal(a.density, b.density)
    assert not np.array_equal(a.points, c.points)
    d, e = W.laplace_sp_batch(n_problems=2, lo=2.0, hi=3.0), W.laplace_sp_batch(n_problems=2, lo=2.0, hi=3.0)
    assert all(np.array_equal(x.points, y.points) for x, y in zip(d, e))


@pytest.mark.parametrize("i", range(8))
def test_points_shapes_and_net_density(i):
    pb = _small()[i]
    n = pb.points.shape[0]
    assert pb.points.shape == (n, 3) and pb.points.dtype == np.float64
    assert pb.density.shape[1:] == (n, pb.k) and pb.density.dtype == np.float64
    assert np.all(pb.points >= 0.0) and np.all(pb.points <= 1.0)
    periodic = [ax for ax in range(3) if pb.periodic_mask >> ax & 1]
    assert np.all(pb.points[:, periodic] < 1.0)
    naxes = len(periodic)
    if naxes in (1, 2):          # a singly or doubly periodic sum exists only for zero net density
        net = np.abs(pb.density.sum(axis=1))
        assert np.all(net <= 1e-12 * np.abs(pb.density).sum(axis=1))


def test_batch_sizes_are_log_uniform_within_bounds():
    sizes = np.array([pb.points.shape[0] for pb in W.laplace_sp_batch(n_problems=64, n_rhs=1)])
    assert sizes.min() >= 10 ** 4 and sizes.max() <= 10 ** 6
    logs = np.log10(sizes)
    assert 4.7 < logs.mean() < 5.3 and logs.std() > 0.4        # uniform on [4, 6]: mean 5, std 0.58


def test_clenshaw_curtis_nodes():
    c = W.clenshaw_curtis_nodes(97)
    assert c.shape == (97,) and c[0] == 0.0 and c[-1] == 1.0
    assert np.all(np.diff(c) > 0)
    assert np.allclose(c + c[::-1], 1.0, atol=1e-15)
    assert c[48] == pytest.approx(0.5, abs=1e-15)
    # extreme points of the Chebyshev polynomial T_96 mapped to [0, 1]: |T_96(2c - 1)| = 1
    t = np.cos(96 * np.arccos(np.clip(2 * c - 1, -1, 1)))
    assert np.allclose(np.abs(t), 1.0, atol=1e-9)


@pytest.mark.parametrize("mask", [W.TP, W.DP_XY, W.SP_X])
def test_paper_timing_points(mask):
    cheb = W.stokes_paper_points("chebyshev", mask=mask)
    logn = W.stokes_paper_points("lognormal", mask=mask)
    for pb in (cheb, logn):
        assert pb.points.shape == (97 ** 3, 3) == (912673, 3) and pb.s == 1000
        assert np.all(pb.points >= 0.0) and np.all(pb.points <= 1.0)
        assert np.all(np.abs(pb.density) <= 1.0)
        if mask != W.TP:
            assert np.abs(pb.density.sum(axis=1)).max() < 1e-9
    # the tensor grid: every node on every axis, each 97^2 times
    c = W.clenshaw_curtis_nodes(97)
    for ax in range(3):
        vals, counts = np.unique(cheb.points[:, ax], return_counts=True)
        assert np.array_equal(vals, c) and np.all(counts == 97 ** 2)
    # lognormal coordinates folded into [0, 1): still visibly non-uniform
    assert np.all(logn.points < 1.0)
    hist = np.histogram(logn.points[:, 0], bins=10, range=(0, 1))[0] / logn.points.shape[0]
    assert hist.max() - hist.min() > 0.02
