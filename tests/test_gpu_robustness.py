"""GPU robustness: multi-launch near field, stream ordering, close points, neutrality scale.

Each case goes through the C-ABI (the ctypes binding) and is compared with the oracle or with
another evaluation of the library whose agreement the method fixes."""
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


_many = {}


def _many_items():
    """Laplace TP, N = 30000, s = 12, p = 4: about 5000 near-field items, far more than the
    workgroups the near-field kernel keeps resident (4 per compute unit), so its work counter
    is in use; 3 right-hand sides take two near-field launches (blocks of 2 and 1)."""
    if not _many:
        pb = W.laplace_sp_uniform(n=30000, seed=41, p=4, s=12, n_rhs=3, mask=7)
        f = okifmm.KIFMM(pb.kernel, pb.periodic_mask, pb.p, pb.s, pb.points)
        _many["pb"] = pb
        _many["f"] = f
        _many["ref"] = np.stack([f.evaluate(d) for d in pb.density])
    return _many["pb"], _many["ref"]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
def test_every_rhs_block_takes_the_whole_item_list(precision, tol):
    """Several right-hand-side blocks, each its own near-field launch over a work counter:
    every right-hand side against the oracle, and per target."""
    pk = _pk()
    pb, ref = _many_items()
    plan = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=precision)
    plan.set_points(_dev(pb.points))
    out = plan.evaluate(_dev(pb.density)).cpu().numpy()
    for r in range(3):
        err = _rel(out[r], ref[r])
        print(f"precision={precision} rhs {r}: rel L2 {err:.3e}", flush=True)
        assert err < tol, r
        assert np.max(np.abs(out[r] - ref[r])) < 100 * tol * np.max(np.abs(ref[r])), r


@pytest.mark.timeout(300)
def test_rhs_change_back_to_back_without_sync():
    """n_rhs = 1 then n_rhs = 3 enqueued back to back with no synchronisation between them
    (the second call rebuilds work lists while the first may still run), then n_rhs = 1 again on
    another stream: each result against the oracle."""
    pk = _pk()
    pb, ref = _many_items()
    for precision, tol in ((0, 1e-10), (1, 1e-6)):
        plan = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=precision)
        plan.set_points(_dev(pb.points))
        d1, d3 = _dev(pb.density[:1]), _dev(pb.density)
        o1 = plan.evaluate(d1)
        o3 = plan.evaluate(d3)
        side = torch.cuda.Stream()
        o1b = plan.evaluate(d1, stream=side)
        side.synchronize()
        torch.cuda.synchronize()
        assert _rel(o1.cpu().numpy()[0], ref[0]) < tol
        assert _rel(o1b.cpu().numpy()[0], ref[0]) < tol
        for r in range(3):
            assert _rel(o3.cpu().numpy()[r], ref[r]) < tol, (precision, r)


def test_set_points_on_a_side_stream_after_producing_them():
    """Points produced by a kernel on torch's current stream and handed to set_points on a side
    stream: the library sees the finished points (tree bit-exact against the oracle's)."""
    pk = _pk()
    pb = W.stokes_tp_uniform(n=20000, seed=42, p=6, s=300)
    f = okifmm.KIFMM(pb.kernel, pb.periodic_mask, pb.p, pb.s, pb.points)
    plan = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=1)
    base = _dev(pb.points)
    x = torch.randn(2048, 2048, device="cuda", dtype=torch.float64)
    for _ in range(4):
        x = x @ x / 2048.0                           # keep the current stream busy
    xyz = base + 0.0 * x[0, 0]                        # produced after that work, on the current stream
    side = torch.cuda.Stream()
    plan.set_points(xyz, stream=side)
    perm, _ = plan.tree()
    assert np.array_equal(perm, f.tree.perm)


def test_close_points_across_a_periodic_face():
    """Two points 2^-41 apart through the periodic face x = 0 / x = 1 (different leaves; dyadic, so
    every separation below is exact in float64): the mixed form's integer positions of the pair
    coincide.  Set-up detects it and every near-field pair is guarded: the output is finite, the
    pair meets as coincident points (contributing nothing to each other), and every other target
    matches the oracle."""
    pk = _pk()
    pb = W.stokes_tp_uniform(n=20000, seed=43, p=6, s=300)
    pts = pb.points.copy()
    pts[0] = [2.0 ** -42, 0.3125, 0.46875]
    pts[1] = [1.0 - 2.0 ** -42, 0.3125, 0.46875]
    d = pb.density[0].copy()
    plan = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=1)
    plan.set_points(_dev(pts))
    assert plan.stats()["close_points"] == 1
    out = plan.evaluate(_dev(d)).cpu().numpy()
    assert np.all(np.isfinite(out))
    f = okifmm.KIFMM(pb.kernel, pb.periodic_mask, pb.p, pb.s, pts)
    ref = f.evaluate(d)
    rest = np.arange(2, pb.n)
    assert _rel(out[rest], ref[rest]) < 1e-6
    # the two points: the oracle's value less the pair's own term, K(+-2^-41 e_x) d_j (the other
    # images of the partner are far and stay in)
    r = 2.0 ** -41
    K = (np.eye(3) / r + np.diag([1.0 / r, 0.0, 0.0])) / (8 * np.pi)
    for i, j in ((0, 1), (1, 0)):
        want = ref[i] - K @ d[j]
        assert np.linalg.norm(out[i] - want) < 1e-4 * np.linalg.norm(want), (i, out[i], want)
    # an ordinary input needs no guard
    plan.set_points(_dev(pb.points))
    assert plan.stats()["close_points"] == 0


@pytest.mark.parametrize("scale", [1e-20, 1.0, 1e20])
def test_neutrality_check_is_scale_invariant(scale):
    """The SP/DP zero-net-density check is relative to the density's magnitude: a neutral input is
    accepted and a non-neutral one rejected at any scale (float64 form)."""
    pk = _pk()
    pb = W.laplace_sp_uniform(n=3000, seed=44, p=6, s=60)
    plan = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=0)
    plan.set_points(_dev(pb.points))
    q = pb.density * scale
    out = plan.evaluate(_dev(q)).cpu().numpy()
    ref = okifmm.KIFMM(pb.kernel, pb.periodic_mask, pb.p, pb.s, pb.points).evaluate(q[0])
    assert _rel(out[0], ref) < 1e-10
    bad = q.copy()
    bad[0, 0, 0] += 1e-6 * scale
    with pytest.raises(pk.PkifmmError) as e:
        plan.evaluate(_dev(bad))
    assert e.value.status == pk.ERR_INCOMPATIBLE


@pytest.mark.timeout(300)
def test_list_thread_on_new_points_and_destroy():
    """For one problem set_points leaves its U/V/W/X list build running on a host thread.
    Points set twice in a row (the first build still running), list sizes and lists read right
    after set_points, and plans destroyed right after set_points: the lists equal the oracle's
    and the evaluation on the second points matches the oracle."""
    pk = _pk()
    pb, ref = _many_items()
    f = _many["f"]
    other = W.laplace_sp_uniform(n=30000, seed=44, p=4, s=12, n_rhs=1, mask=7)
    for _ in range(3):   # destroyed while its lists may still be under construction
        tmp = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=1)
        tmp.set_points(_dev(other.points))
        tmp.close()
    plan = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=1)
    plan.set_points(_dev(other.points))
    plan.set_points(_dev(pb.points))
    st = plan.stats()
    assert st["n_u"] == sum(len(v) for v in f.lists.U.values())
    assert st["n_v"] == sum(len(v) for v in f.lists.V.values())
    for which in "UX":
        off, ent = plan.lists(which)
        lref = getattr(f.lists, which)
        for b in range(f.tree.nbox):
            got = [(int(e[0]), (int(e[1]), int(e[2]), int(e[3]))) for e in ent[off[b]:off[b + 1]]]
            assert got == list(lref.get(b, [])), (which, b)
    plan.set_points(_dev(other.points))
    plan.set_points(_dev(pb.points))   # straight into the evaluation this time
    out = plan.evaluate(_dev(pb.density)).cpu().numpy()
    for r in range(3):
        assert _rel(out[r], ref[r]) < 1e-6, r
