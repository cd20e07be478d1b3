"""GPU parity with separate targets (Section 2's problem: T targets apart from S sources), through
the C-ABI, against the oracle's union-tree evaluation."""
import numpy as np
import pytest

import workloads as W
from oracle import kifmm as okifmm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pk():
    import paper_1705_02043_amd as pk
    return pk


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(name):
    """Sources uniform, targets graded toward a corner (a union tree whose leaves hold sources
    only, targets only, or both)."""
    rng = np.random.default_rng(80)
    if name == "stokes_tp":
        pb = W.stokes_tp_uniform(n=20000, seed=81, p=6, s=300, n_rhs=2)
        trg = rng.random((7000, 3)) ** 2
    elif name == "laplace_sp":
        pb = W.laplace_sp_uniform(n=5000, seed=82, p=8, s=50, n_rhs=1)
        trg = rng.random((3000, 3)) ** 3
    else:
        pb = W.stokes_dp_slab(n=20000, seed=83, p=6, s=300)
        trg = np.column_stack([rng.random((4000, 2)), np.clip(rng.normal(0.5, 0.2, 4000), 0, 1)])
    return pb, trg


_ref = {}


def _oracle(name):
    if name not in _ref:
        pb, trg = _case(name)
        f = okifmm.KIFMM(pb.kernel, pb.periodic_mask, pb.p, pb.s, pb.points, targets=trg)
        _ref[name] = (pb, trg, f, np.stack([f.evaluate(d) for d in pb.density]))
    return _ref[name]


def _partitioned_perm(f):
    """The oracle's (key, index) order with every leaf's sources moved before its targets."""
    t = f.tree
    perm = t.perm.copy()
    for b in t.leaves():
        seg = perm[t.begin[b]:t.end[b]]
        perm[t.begin[b]:t.end[b]] = np.concatenate([seg[seg < f.n_src], seg[seg >= f.n_src]])
    return perm


@pytest.mark.parametrize("name", ["stokes_tp", "laplace_sp", "stokes_dp"])
def test_separate_targets_tree_and_parity(name):
    """Tree over the union bit-exact (boxes; each leaf's sources then targets), potentials at the
    targets against the oracle: float64 within 1e-10, mixed within 1e-6, per leaf too."""
    pk = _pk()
    pb, trg, f, ref = _oracle(name)
    t = f.tree
    for precision, tol in ((0, 1e-10), (1, 1e-6)):
        plan = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=precision)
        plan.set_points(_dev(pb.points), targets=_dev(trg))
        perm, boxes = plan.tree()
        assert boxes.shape[0] == t.nbox
        assert np.array_equal(boxes[:, 4], t.begin) and np.array_equal(boxes[:, 5], t.end)
        assert np.array_equal(perm, _partitioned_perm(f))
        out = plan.evaluate(_dev(pb.density)).cpu().numpy()
        assert out.shape == ref.shape
        err = _rel(out, ref)
        worst = 0.0
        for b in t.leaves():
            idx = t.perm[t.begin[b]:t.end[b]]
            idx = idx[idx >= f.n_src] - f.n_src
            if len(idx):
                worst = max(worst, _rel(out[:, idx], ref[:, idx]))
        print(f"{name} targets precision={precision}: rel L2 {err:.3e}, worst leaf {worst:.3e}", flush=True)
        assert err < tol and worst < 10 * tol


def test_separate_targets_edge_cases():
    """No targets: an empty result.  Targets that repeat the sources: the sources' own potentials to
    the KIFMM accuracy of the two trees.  A separate target set in a captured graph and in the
    allocation-free entry point: bitwise the eager result."""
    pk = _pk()
    pb = W.stokes_tp_uniform(n=8000, seed=84, p=6, s=200)
    plan = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=1)
    plan.set_points(_dev(pb.points), targets=_dev(np.zeros((0, 3))))
    out = plan.evaluate(_dev(pb.density))
    assert tuple(out.shape) == (1, 0, 3)
    plan.set_points(_dev(pb.points))
    same = plan.evaluate(_dev(pb.density)).cpu().numpy()
    plan.set_points(_dev(pb.points), targets=_dev(pb.points))
    rep = plan.evaluate(_dev(pb.density)).cpu().numpy()
    assert _rel(rep, same) < 1e-4
    rng = np.random.default_rng(85)
    trg = rng.random((3000, 3))
    plan.set_points(_dev(pb.points), targets=_dev(trg))
    eager = plan.evaluate(_dev(pb.density)).cpu().numpy()
    out = torch.empty((1, 3000, 3), dtype=torch.float64, device="cuda")
    plan.evaluate(_dev(pb.density), out=out, noalloc=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), eager)
    g = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=1, flags=pk.GRAPH)
    g.set_points(_dev(pb.points), targets=_dev(trg))
    dens = _dev(pb.density)
    for _ in range(2):
        out.zero_()
        g.evaluate(dens, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager)
