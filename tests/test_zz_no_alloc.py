"""pkifmm_evaluate_noalloc (the entry point that allocates nothing) against pkifmm_evaluate.

Its workspace is one static device array shared by every call on the GPU; the same kernels run
in the same order as in pkifmm_evaluate, so the results must be the same bits."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pk():
    import paper_1705_02043_amd as pk
    return pk


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("precision,n_rhs", [(1, 1), (0, 1), (1, 2), (0, 3)])
def test_noalloc_two_calls_in_a_row_second_smaller(precision, n_rhs):
    """Two problems, the second smaller: pkifmm_evaluate once each (it builds the work lists), then
    the allocation-free calls back to back on one stream, sharing the static array; each output
    bitwise equal to pkifmm_evaluate's.  Then both again in the opposite order."""
    pk = _pk()
    probs = [W.stokes_tp_uniform(n=12000, seed=51, p=6, s=300, n_rhs=n_rhs),
             W.stokes_tp_uniform(n=4000, seed=52, p=6, s=300, n_rhs=n_rhs)]
    plans, dens, refs = [], [], []
    for pb in probs:
        plan = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=precision)
        plan.set_points(_dev(pb.points))
        d = _dev(pb.density)
        with pytest.raises(pk.PkifmmError) as e:     # no work lists for these points yet
            plan.evaluate(d, out=torch.empty_like(d), noalloc=True)
        assert e.value.status == pk.ERR_INVALID_ARG
        refs.append(plan.evaluate(d).cpu().numpy())
        plans.append(plan)
        dens.append(d)
    for order in ((0, 1), (1, 0)):
        outs = {i: torch.full_like(dens[i], float("nan")) for i in order}
        for i in order:
            plans[i].evaluate(dens[i], out=outs[i], noalloc=True)
        torch.cuda.synchronize()
        for i in order:
            assert np.array_equal(outs[i].cpu().numpy(), refs[i]), (order, i)


def test_noalloc_refuses_a_workspace_beyond_its_array():
    """A problem whose workspace exceeds the static array is refused with CAPACITY (before anything
    is enqueued); pkifmm_evaluate still runs it."""
    pk = _pk()
    pb = W.stokes_tp_uniform(n=300000, seed=53, p=6, s=1000)
    plan = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=1)
    plan.set_points(_dev(pb.points))
    d = _dev(pb.density)
    ref = plan.evaluate(d).cpu().numpy()
    out = torch.zeros_like(d)
    with pytest.raises(pk.PkifmmError) as e:
        plan.evaluate(d, out=out, noalloc=True)
    assert e.value.status == pk.ERR_CAPACITY
    torch.cuda.synchronize()
    assert not torch.any(out).item()
    assert np.array_equal(plan.evaluate(d).cpu().numpy(), ref)
