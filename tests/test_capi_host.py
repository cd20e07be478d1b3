"""CPU checks of the C-ABI library: symbols, and the host topology code against the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1705_02043_amd as pk
from oracle import tree as otree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "pkifmm.h")).read()
    declared = set(re.findall(r"\b(pkifmm_\w+)\s*\(", hdr))
    assert declared == set(pk.EXPORTED), declared ^ set(pk.EXPORTED)
    L = pk.lib()
    for name in declared:
        assert getattr(L, name) is not None


def test_status_strings_and_bad_config():
    L = pk.lib()
    assert L.pkifmm_status_string(0) == b"ok"
    assert L.pkifmm_status_string(pk.ERR_OUT_OF_BOX).startswith(b"coordinate")
    cfg = pk.pkifmm_config()
    assert L.pkifmm_config_default(ctypes.byref(cfg)) == 0
    assert cfg.p == 8 and cfg.box_length == 1.0
    cfg.p = 2        # invalid order is rejected before any device call
    h = ctypes.c_void_p()
    assert L.pkifmm_plan_create(ctypes.byref(cfg), ctypes.byref(h)) == pk.ERR_INVALID_ARG
    cfg.p = 8
    cfg.kernel = 3                 # no such kernel
    assert L.pkifmm_plan_create(ctypes.byref(cfg), ctypes.byref(h)) == pk.ERR_INVALID_ARG
    cfg.kernel, cfg.periodic_mask = pk.STOKES, 8   # no such axis
    assert L.pkifmm_plan_create(ctypes.byref(cfg), ctypes.byref(h)) == pk.ERR_INVALID_ARG
    cfg.periodic_mask, cfg.flags = 7, 16           # no such flag
    assert L.pkifmm_plan_create(ctypes.byref(cfg), ctypes.byref(h)) == pk.ERR_INVALID_ARG
    cfg.flags = 0
    cfg.alloc = pk.ALLOC_FN(lambda ctx, n, s: None)   # an allocator without its free
    assert L.pkifmm_plan_create(ctypes.byref(cfg), ctypes.byref(h)) == pk.ERR_INVALID_ARG
    assert L.pkifmm_status_string(pk.ERR_CACHE_CORRUPT).startswith(b"operator cache")
    assert L.pkifmm_plan_destroy(None) == 0


def _oracle_rows(t):
    rows = []
    for b in range(t.nbox):
        fc = next((c for c in t.children[b] if c >= 0), -1)
        rows.append([t.level[b], *t.coord[b], t.begin[b], t.end[b], t.parent[b], fc])
    return np.array(rows, dtype=np.int32)


@pytest.mark.parametrize("mask,n,s,seed", [(0, 2000, 30, 1), (1, 2000, 50, 2), (7, 3000, 40, 3),
                                           (4, 1500, 20, 4), (7, 5, 1, 5), (7, 1, 4, 6), (1, 0, 4, 7)])
def test_host_topology_matches_oracle(mask, n, s, seed):
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3)) ** 3            # strongly graded -> adaptive, W/X lists present
    u = otree.wrap(pts, mask)
    t = otree.build_tree(u, s)
    lists = otree.build_lists(t, mask)
    for which in "UVWX":
        boxes, off, ent = pk.host_topology(t.keys, s, mask, which)
        assert np.array_equal(boxes, _oracle_rows(t))
        ref = getattr(lists, which)
        for b in range(t.nbox):
            got = [(int(e[0]), (int(e[1]), int(e[2]), int(e[3]))) for e in ent[off[b]:off[b + 1]]]
            assert got == list(ref.get(b, [])), (which, b)


class _DeviceLike:
    """Stands in for a float64 GPU tensor of n rows in the binding's host-side checks."""

    def __init__(self, n):
        import torch
        self.is_cuda, self.dtype, self.shape = True, torch.float64, (n, 3)

    def dim(self):
        return 2


def test_binding_refuses_point_arguments_before_any_library_call():
    """The library reads sum(counts) rows of xyz and cannot see the tensor's length: the binding
    refuses a mismatch (and host tensors, and negative counts) before it calls the library."""
    import torch
    plan = pk.Plan.__new__(pk.Plan)          # no library handle: a call that got through would fail
    plan._h = None
    with pytest.raises(ValueError):
        plan.set_points(torch.zeros(4, 3, dtype=torch.float64))
    with pytest.raises(ValueError):
        plan.set_points_batch([3, 4], _DeviceLike(10))
    with pytest.raises(ValueError):
        plan.set_points_batch([-1, 11], _DeviceLike(10))
    with pytest.raises(ValueError):
        plan.set_points_batch([5, 5], torch.zeros(10, 3, dtype=torch.float32))


def test_binding_refuses_density_arguments_before_any_library_call():
    """evaluate refuses a density that is not a float64 GPU tensor of shape [R, n, k] (or [n, k])
    before it calls the library: the library reads R * n * k values and cannot see the tensor."""
    import torch
    plan = pk.Plan.__new__(pk.Plan)
    plan._h, plan.n, plan.k = None, 10, 3
    for bad in (torch.zeros(1, 10, 3, dtype=torch.float64),              # host memory
                torch.zeros(10, dtype=torch.float64),                    # wrong rank
                torch.zeros(2, 1, 10, 3, dtype=torch.float64)):          # wrong rank
        with pytest.raises(ValueError):
            plan.evaluate(bad)


def _fnv1a(data: bytes) -> int:
    h = 1469598103934665603
    for b in data:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def _cache_file(path, kn=6, r_up=5, r_dn=4, seed=0):
    """An operator cache file in the library's layout (header, five arrays, FNV-1a checksum)."""
    import struct
    rng = np.random.default_rng(seed)
    head = b"PKIFMMOP" + struct.pack("<IiIiiiiiddd", 1, 2, 7, 4, kn, r_up, r_dn, 0, 1e-11, 3.0, 2.0)
    assert len(head) == 64
    body = b"".join(rng.random(n).tobytes() for n in (r_up * kn, kn * r_up, r_dn * kn, kn * r_dn, kn * kn))
    data = head + body
    with open(path, "wb") as f:
        f.write(data + _fnv1a(data).to_bytes(8, "little"))
    return data


def test_operator_cache_check_on_the_host(tmp_path):
    """The cache file checks run on the CPU: a well-formed file passes; a flipped bit, a truncated
    file, a wrong magic or a missing file are refused."""
    L = pk.lib()
    good = str(tmp_path / "ops.bin")
    data = _cache_file(good)
    assert L.pkifmm_operator_cache_check(good.encode()) == pk.OK
    for name, mutate in (("flip", lambda d: d[:100] + bytes([d[100] ^ 4]) + d[101:]),
                         ("short", lambda d: d[:-9]),
                         ("magic", lambda d: b"PKIFMMOX" + d[8:])):
        full = open(good, "rb").read()
        bad = str(tmp_path / f"{name}.bin")
        with open(bad, "wb") as f:
            f.write(mutate(full))
        assert L.pkifmm_operator_cache_check(bad.encode()) == pk.ERR_CACHE_CORRUPT, name
    assert L.pkifmm_operator_cache_check(str(tmp_path / "none.bin").encode()) == pk.ERR_INVALID_ARG
    assert len(data) == 64 + 8 * (2 * 5 * 6 + 2 * 4 * 6 + 36)
