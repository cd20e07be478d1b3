"""Periodic kernel-independent FMM evaluation pass on MI355X (gfx950).

Thin ctypes binding of the C interface in ``include/pkifmm.h``: every
``pkifmm_*`` function is exposed under the same name, and :class:`Plan` wraps
them for torch tensors (device memory and the current stream come from
PyTorch; all arithmetic runs in the library's HIP kernels).  Importing this
module does not touch the GPU; using it without the built library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpkifmm.so")
# launch choices measured by pkifmm_autotune on this project's target device (committed records)
TUNING_FILE = os.path.join(HERE, "tuning", "launch_choices.txt")

LAPLACE, STOKES = 1, 2
PERIODIC_X, PERIODIC_Y, PERIODIC_Z = 1, 2, 4
FP64, MIXED = 0, 1
SKIP_CHECKS = 1
PHASE_TIMING = 2
GRAPH = 4
FAR_STEP_D = 8

OK = 0
ERR_INVALID_ARG, ERR_OUT_OF_BOX, ERR_INCOMPATIBLE, ERR_UNSUPPORTED = -1, -2, -3, -4
ERR_OOM, ERR_HIP, ERR_NO_POINTS, ERR_NUMERICS, ERR_CAPACITY, ERR_CACHE_CORRUPT = -5, -6, -7, -8, -9, -10

EXPORTED = ["pkifmm_config_default", "pkifmm_plan_create", "pkifmm_set_points", "pkifmm_set_points_batch",
            "pkifmm_evaluate", "pkifmm_evaluate_noalloc",
            "pkifmm_get_stats", "pkifmm_get_tree", "pkifmm_get_list", "pkifmm_plan_destroy",
            "pkifmm_status_string", "pkifmm_last_error", "pkifmm_host_topology", "pkifmm_get_solve_factors", "pkifmm_operator_cache_check", "pkifmm_autotune"]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class pkifmm_config(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("periodic_mask", ctypes.c_uint), ("p", ctypes.c_int),
                ("max_pts_per_leaf", ctypes.c_int), ("precision", ctypes.c_int),
                ("box_length", ctypes.c_double), ("svd_rel_threshold", ctypes.c_double),
                ("flags", ctypes.c_uint), ("operator_cache_dir", ctypes.c_char_p),
                ("alloc_ctx", ctypes.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("tuning_file", ctypes.c_char_p), ("near_layers", ctypes.c_int)]


class pkifmm_stats(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_problems", ctypes.c_int),
                ("n_boxes", ctypes.c_int), ("n_leaves", ctypes.c_int),
                ("depth", ctypes.c_int), ("n_u", ctypes.c_int64), ("n_v", ctypes.c_int64),
                ("n_w", ctypes.c_int64), ("n_x", ctypes.c_int64), ("u_pairs", ctypes.c_int64),
                ("near_pairs", ctypes.c_int64),
                ("svd_rank_up", ctypes.c_int), ("svd_rank_down", ctypes.c_int),
                ("ms_set_points", ctypes.c_double), ("ms_evaluate", ctypes.c_double),
                ("n_timed", ctypes.c_int), ("ms_phase", ctypes.c_double * 5),
                ("close_points", ctypes.c_int), ("tune_near_wpc", ctypes.c_int), ("tune_rb_near", ctypes.c_int),
                ("tune_rb_s2m", ctypes.c_int), ("tune_ms", ctypes.c_double), ("tune_m2l_rows", ctypes.c_int)]

PHASES = ["near", "up", "m2l", "down", "leaf"]


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1705_02043_amd/build.py (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        sig = {
            "pkifmm_config_default": (i32, [ctypes.POINTER(pkifmm_config)]),
            "pkifmm_plan_create": (i32, [ctypes.POINTER(pkifmm_config), ctypes.POINTER(vp)]),
            "pkifmm_set_points": (i32, [vp, i64, vp, i64, vp, vp]),
            "pkifmm_set_points_batch": (i32, [vp, i32, vp, vp, vp]),
            "pkifmm_evaluate": (i32, [vp, i32, vp, vp, vp]),
            "pkifmm_evaluate_noalloc": (i32, [vp, i32, vp, vp, vp]),
            "pkifmm_get_stats": (i32, [vp, ctypes.POINTER(pkifmm_stats)]),
            "pkifmm_get_tree": (i32, [vp, vp, vp]),
            "pkifmm_get_list": (i32, [vp, ctypes.c_char, vp, vp]),
            "pkifmm_plan_destroy": (i32, [vp]),
            "pkifmm_status_string": (ctypes.c_char_p, [i32]),
            "pkifmm_last_error": (ctypes.c_char_p, [vp]),
            "pkifmm_host_topology": (i32, [vp, i64, i32, ctypes.c_uint, ctypes.c_char, vp, vp, vp, vp]),
            "pkifmm_get_solve_factors": (i32, [vp, i32, ctypes.POINTER(i32), vp, vp]),
            "pkifmm_operator_cache_check": (i32, [ctypes.c_char_p]),
            "pkifmm_autotune": (i32, [vp, i32, vp, vp, vp, ctypes.c_char_p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def __getattr__(name):
    if name in EXPORTED:
        return getattr(lib(), name)
    raise AttributeError(name)


class PkifmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _check(status: int, plan=None):
    if status != OK:
        L = lib()
        msg = L.pkifmm_status_string(status).decode()
        if plan is not None:
            extra = L.pkifmm_last_error(plan).decode()
            if extra:
                msg += ": " + extra
        raise PkifmmError(status, msg)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_points(torch, xyz):
    if not (xyz.is_cuda and xyz.dtype == torch.float64 and xyz.dim() == 2 and xyz.shape[1] == 3):
        raise ValueError("xyz must be a float64 GPU tensor of shape [n, 3]")


class Plan:
    """One (kernel, periodicity, p, s, precision) set of operators, a point set and its tree."""

    def __init__(self, kernel: int, periodic_mask: int, p: int, max_pts_per_leaf: int,
                 precision: int = FP64, box_length: float = 1.0,
                 svd_rel_threshold: float = 0.0, flags: int = 0,
                 operator_cache_dir: Optional[str] = None, torch_allocator: bool = False,
                 tuning_file: Optional[str] = TUNING_FILE, near_layers: int = 1):
        """torch_allocator: the plan's device buffers come from PyTorch's caching allocator
        (through the C-ABI's alloc/free callbacks) instead of hipMalloc.  tuning_file: the
        autotuner's records read at plan creation (None: the library's default choices)."""
        L = lib()
        cfg = pkifmm_config()
        _check(L.pkifmm_config_default(ctypes.byref(cfg)))
        cfg.kernel, cfg.periodic_mask, cfg.p = kernel, periodic_mask, p
        cfg.max_pts_per_leaf, cfg.precision = max_pts_per_leaf, precision
        cfg.box_length, cfg.svd_rel_threshold, cfg.flags = box_length, svd_rel_threshold, flags
        cfg.near_layers = near_layers
        if operator_cache_dir:
            cfg.operator_cache_dir = os.fsencode(operator_cache_dir)
        if tuning_file and os.path.exists(tuning_file):
            cfg.tuning_file = os.fsencode(tuning_file)
        self._callbacks = None
        if torch_allocator:
            import torch
            dev = torch.cuda.current_device()

            def _alloc(ctx, nbytes, stream):
                try:
                    return torch.cuda.caching_allocator_alloc(nbytes, dev, stream or 0)
                except Exception:
                    return None                  # the library reports out of memory

            def _free(ctx, ptr, stream):
                torch.cuda.caching_allocator_delete(ptr)
            self._callbacks = (ALLOC_FN(_alloc), FREE_FN(_free))   # kept alive with the plan
            cfg.alloc, cfg.free = self._callbacks
        h = ctypes.c_void_p()
        _check(L.pkifmm_plan_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.k = 1 if kernel == LAPLACE else 3
        self.n_surf = 6 * (p - 1) ** 2 + 2
        self.n = self.n_out = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().pkifmm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_points(self, xyz, targets=None, stream=None):
        """xyz: torch float64 CUDA tensor [n_src, 3], the sources (input order); targets: None (the
        targets are the sources) or a float64 CUDA tensor [n_trg, 3] of separate targets."""
        import torch
        _check_points(torch, xyz)
        xyz = xyz.contiguous()
        trg_ptr, n_trg = None, 0
        if targets is not None:
            _check_points(torch, targets)
            targets = targets.contiguous()
            trg_ptr, n_trg = ctypes.c_void_p(targets.data_ptr()), targets.shape[0]
            if n_trg == 0:   # an empty separate target set still needs a non-NULL pointer
                trg_ptr = ctypes.c_void_p(xyz.data_ptr() or 1)
        if stream is not None:   # the points (or their contiguous copies) come from torch's current stream
            stream.wait_stream(torch.cuda.current_stream())
        _check(lib().pkifmm_set_points(self._h, xyz.shape[0], ctypes.c_void_p(xyz.data_ptr()), n_trg, trg_ptr,
                                       _stream_ptr(stream)), self._h)
        self.n = xyz.shape[0]
        self.n_out = n_trg if targets is not None else self.n

    def set_points_batch(self, counts, xyz, stream=None):
        """counts: point count of each problem; xyz: float64 CUDA [sum(counts), 3], problems packed."""
        import numpy as np
        import torch
        _check_points(torch, xyz)
        c = np.ascontiguousarray(counts, dtype=np.int64).reshape(-1)
        # the library reads sum(counts) rows of xyz: a mismatch would read past the tensor
        if np.any(c < 0) or int(c.sum()) != xyz.shape[0]:
            raise ValueError(f"counts must be non-negative and sum to the {xyz.shape[0]} rows of xyz")
        xyz = xyz.contiguous()
        if stream is not None:   # the library synchronises `stream` before it returns
            stream.wait_stream(torch.cuda.current_stream())
        _check(lib().pkifmm_set_points_batch(self._h, len(c), c.ctypes.data, ctypes.c_void_p(xyz.data_ptr()),
                                             _stream_ptr(stream)), self._h)
        self.n = self.n_out = xyz.shape[0]

    def evaluate(self, density, out=None, stream=None, noalloc=False):
        """density: float64 CUDA [R, n_src, k] (or [n_src, k]); returns the potentials at the targets,
        [R, n_trg, k] (or [n_trg, k]; n_trg = n_src when the targets are the sources).

        out, if given, is a contiguous float64 CUDA tensor of that shape; when the targets are the
        sources it may be the density tensor itself (the pass reads every density before it writes
        a potential).  noalloc=True calls pkifmm_evaluate_noalloc (the library allocates nothing;
        its workspace is a static device array): give a contiguous density and an `out` so that
        this binding allocates nothing either."""
        import torch
        if density.dim() not in (2, 3):
            raise ValueError("density must be [n, k] or [R, n, k]")
        squeeze = density.dim() == 2
        d = density[None] if squeeze else density
        if not (d.is_cuda and d.dtype == torch.float64 and d.shape[1] == self.n and d.shape[2] == self.k):
            raise ValueError(f"density must be float64 on the GPU with shape [R, {self.n}, {self.k}]")
        d = d.contiguous()
        shape = (d.shape[0], self.n_out, self.k)
        if out is None:
            res = torch.empty(shape, dtype=torch.float64, device=d.device)
        else:
            want = shape[1:] if squeeze else shape
            if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and tuple(out.shape) == want):
                raise ValueError(f"out must be a contiguous float64 GPU tensor of shape {want}")
            res = out[None] if squeeze else out
        if stream is not None:
            # the pass runs on `stream`: it starts after the work queued so far on torch's current
            # stream (a contiguous copy made above included), and torch must not recycle that copy
            # or an output allocated here until `stream` has used them
            stream.wait_stream(torch.cuda.current_stream())
            d.record_stream(stream)
            res.record_stream(stream)
        fn = lib().pkifmm_evaluate_noalloc if noalloc else lib().pkifmm_evaluate
        _check(fn(self._h, d.shape[0], ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(res.data_ptr()),
                  _stream_ptr(stream)), self._h)
        return res[0] if squeeze else res

    def autotune(self, density, tuning_file: Optional[str] = None, stream=None):
        """Time the evaluation of `density` ([R, n_src, k]) under the bit-neutral launch choices and
        keep the fastest for this n_rhs (pkifmm_autotune); with tuning_file, record it there."""
        import torch
        d = density[None] if density.dim() == 2 else density
        d = d.contiguous()
        res = torch.empty((d.shape[0], self.n_out, self.k), dtype=torch.float64, device=d.device)
        path = os.fsencode(tuning_file) if tuning_file else None
        _check(lib().pkifmm_autotune(self._h, d.shape[0], ctypes.c_void_p(d.data_ptr()),
                                     ctypes.c_void_p(res.data_ptr()), _stream_ptr(stream), path), self._h)
        st = self.stats()
        return {"near_wpc": st["tune_near_wpc"], "rb_near": st["tune_rb_near"], "rb_s2m": st["tune_rb_s2m"],
                "m2l_rows": st["tune_m2l_rows"], "ms": st["tune_ms"]}

    def stats(self) -> dict:
        st = pkifmm_stats()
        _check(lib().pkifmm_get_stats(self._h, ctypes.byref(st)), self._h)
        out = {f: getattr(st, f) for f, _ in pkifmm_stats._fields_ if f != "ms_phase"}
        out["ms_phase"] = {PHASES[i]: st.ms_phase[i] for i in range(len(PHASES))}
        return out

    def solve_factors(self, which: int):
        """(U^T [r, kn], V S^+ [kn, r]) of the upward (0) or downward (1) check-to-equivalent solve."""
        import numpy as np
        r = ctypes.c_int()
        L = lib()
        _check(L.pkifmm_get_solve_factors(self._h, which, ctypes.byref(r), None, None), self._h)
        kn = self.k * self.n_surf
        ut = np.zeros((kn, r.value))          # column-major r x kn  = row-major kn x r
        vs = np.zeros((r.value, kn))          # column-major kn x r  = row-major r x kn
        _check(L.pkifmm_get_solve_factors(self._h, which, ctypes.byref(r), ut.ctypes.data, vs.ctypes.data), self._h)
        return ut.T.copy(), vs.T.copy()

    def tree(self):
        """(perm [n] int64, boxes [nbox, 8] int32) as numpy arrays; n counts every point the tree
        holds (with separate targets: sources and targets)."""
        import numpy as np
        st = self.stats()
        n = st["n_points"]
        perm = np.zeros(max(n, 1), dtype=np.int64)
        boxes = np.zeros((st["n_boxes"], 8), dtype=np.int32)
        _check(lib().pkifmm_get_tree(self._h, perm.ctypes.data, boxes.ctypes.data), self._h)
        return perm[:n], boxes

    def lists(self, which: str):
        """(offsets [nbox+1] int64, entries [m, 4] int32) of the U, V, W or X list."""
        import numpy as np
        st = self.stats()
        off = np.zeros(st["n_boxes"] + 1, dtype=np.int64)
        _check(lib().pkifmm_get_list(self._h, which.encode(), off.ctypes.data, None), self._h)
        ent = np.zeros((max(int(off[-1]), 1), 4), dtype=np.int32)
        _check(lib().pkifmm_get_list(self._h, which.encode(), off.ctypes.data, ent.ctypes.data), self._h)
        return off, ent[:int(off[-1])]


def host_topology(sorted_keys, max_pts_per_leaf: int, periodic_mask: int, which: str):
    """Host-only tree + one list from sorted Morton keys: (boxes [nbox, 8], offsets, entries [m, 4])."""
    import numpy as np
    keys = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    L = lib()
    nb = ctypes.c_int64()
    args = (keys.ctypes.data, keys.shape[0], max_pts_per_leaf, periodic_mask, which.encode())
    _check(L.pkifmm_host_topology(*args, ctypes.byref(nb), None, None, None))
    boxes = np.zeros((nb.value, 8), dtype=np.int32)
    off = np.zeros(nb.value + 1, dtype=np.int64)
    _check(L.pkifmm_host_topology(*args, ctypes.byref(nb), boxes.ctypes.data, off.ctypes.data, None))
    ent = np.zeros((max(int(off[-1]), 1), 4), dtype=np.int32)
    _check(L.pkifmm_host_topology(*args, ctypes.byref(nb), boxes.ctypes.data, off.ctypes.data, ent.ctypes.data))
    return boxes, off, ent[:int(off[-1])]
