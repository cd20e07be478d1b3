"""Throughput of the periodic KIFMM evaluation pass on one MI355X.

Workload: Stokes velocity kernel, triply periodic unit cube, N = 1,000,000
uniform random points, i.i.d. N(0,1) forces made force-free, p = 8, at most
2000 points per leaf (seeded, synthetic).  One step = one pass of the whole
path over the batch: wrap/validate, Morton sort, octree and lists
(pkifmm_set_points) and the evaluation (pkifmm_evaluate), inputs and outputs
resident in HBM.  The mixed-precision form is the headline value; the plain
float64 form is timed beside it.

Prints ONE JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "targets evaluated/sec, Stokes TP N=1M at 1e-6 rel. L2: mixed-prec vs plain FP64"
PEAK_FP32_VECTOR_TFLOPS = 157.3
FLOPS_PER_STOKES_PAIR = 28       # 3 sub, r^2 5, r^-3 2, f.r 5, scale 1, 6 FMA (rsqrt not counted)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


NEAR_SOURCE = os.path.join(ROOT, "paper_1705_02043_amd", "csrc", "kernels_p2p.hip")
NEAR_COUNTERS = os.path.join(ROOT, "profiles", "counters_near_stokes_tp_n1m_p8.txt")


def near_code_digest(text):
    """sha1 of a source with its // comments and all whitespace removed (comment edits do not
    change the kernel the counters were taken on)."""
    import hashlib
    import re
    code = re.sub(r"\s+", "", re.sub(r"//[^\n]*", "", text))
    return hashlib.sha1(code.encode()).hexdigest()


def near_traffic():
    """HBM bytes per launch of the near phase (near kernel + gather) from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE passes, each scaled by what the counter reads for a copy
    of known size; None when the kernel source has changed since the counters were taken."""
    try:
        with open(NEAR_SOURCE) as f:
            digest = near_code_digest(f.read())
        vals = {}
        with open(NEAR_COUNTERS) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip()
    except OSError:
        return None, "no counter summary"
    if vals.get("kernels_p2p.hip code sha1") != digest:
        return None, "kernel changed since the counters were taken"
    return float(vals["near phase HBM bytes per launch"]), vals.get("source", "")


def time_form(pk, torch, pb, precision, steps, warmup, tuning_file=None):
    t_plan = time.perf_counter()
    plan = pk.Plan(pb.kernel, pb.periodic_mask, pb.p, pb.s, precision=precision, flags=pk.PHASE_TIMING,
                   tuning_file=tuning_file or pk.TUNING_FILE)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t_plan
    xyz = torch.as_tensor(pb.points, device="cuda")
    dens = torch.as_tensor(pb.density, device="cuda")
    out = torch.empty_like(dens)
    for _ in range(warmup):
        plan.set_points(xyz)
        plan.evaluate(dens, out=out)
    torch.cuda.synchronize()
    plan.stats()                                  # drop the warm-up phase events
    t_sp = t_ev = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        plan.set_points(xyz)                      # synchronises (tree topology on the host)
        b = time.perf_counter()
        plan.evaluate(dens, out=out)
        torch.cuda.synchronize()
        c = time.perf_counter()
        t_sp += b - a
        t_ev += c - b
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    st = plan.stats()
    res = out.cpu().numpy()
    plan.close()
    return {"s_total": total, "s_set_points": t_sp / steps, "s_evaluate": t_ev / steps, "stats": st,
            "s_plan": t_plan}, res


def other_configs(pk, torch, W, steps=3, warmup=1):
    """Throughput of the other configurations (mixed form): SP Laplace N=2000; DP Stokes slab
    N=4M p=10; 64 SP Laplace problems x 16 RHS in one batched forest; clustered TP Stokes
    N=16M p=12 x 4 RHS.  One step = set_points (or set_points_batch) + evaluate."""
    res = {}

    def run(name, kernel, mask, p, s, set_pts, dens, n_total):
        t0 = time.perf_counter()
        plan = pk.Plan(kernel, mask, p, s, precision=pk.MIXED, flags=pk.PHASE_TIMING)
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        out = torch.empty_like(dens)
        for _ in range(warmup):
            set_pts(plan)
            plan.evaluate(dens, out=out)
        torch.cuda.synchronize()
        plan.stats()
        t0 = time.perf_counter()
        for _ in range(steps):
            set_pts(plan)
            plan.evaluate(dens, out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        st = plan.stats()
        R = dens.shape[0]
        res[name] = {"ms_per_step": ms, "targets_per_s": n_total / (ms * 1e-3),
                     "target_rhs_per_s": n_total * R / (ms * 1e-3), "n": n_total, "n_rhs": R, "p": p, "s": s,
                     "plan_create_s": t_plan, "ms_phase": st["ms_phase"], "boxes": st["n_boxes"],
                     "depth": st["depth"], "near_pairs": st["near_pairs"]}
        log(f"{name}: {ms:.2f} ms/step, {n_total / (ms * 1e-3):.3e} targets/s")
        plan.close()
        del out

    pb = W.laplace_sp_uniform()
    xyz = torch.as_tensor(pb.points, device="cuda")
    run("laplace_sp_n2000_p8_s50", pb.kernel, pb.periodic_mask, pb.p, pb.s, lambda pl: pl.set_points(xyz),
        torch.as_tensor(pb.density, device="cuda"), pb.n)
    pb = W.stokes_dp_slab()
    xyz = torch.as_tensor(pb.points, device="cuda")
    run("stokes_dp_slab_n4000000_p10_s2000", pb.kernel, pb.periodic_mask, pb.p, pb.s,
        lambda pl: pl.set_points(xyz), torch.as_tensor(pb.density, device="cuda"), pb.n)
    del pb, xyz
    probs = W.laplace_sp_batch()
    counts = [q.n for q in probs]
    xyz = torch.as_tensor(np.concatenate([q.points for q in probs]), device="cuda")
    dens = torch.as_tensor(np.concatenate([q.density for q in probs], axis=1), device="cuda")
    run("laplace_sp_batch64_rhs16_p8_s2000", probs[0].kernel, probs[0].periodic_mask, probs[0].p, probs[0].s,
        lambda pl: pl.set_points_batch(counts, xyz), dens, int(sum(counts)))
    # the same forest as one captured HIP graph: the points set once, then replays alone timed
    plan = pk.Plan(probs[0].kernel, probs[0].periodic_mask, probs[0].p, probs[0].s, precision=pk.MIXED,
                   flags=pk.GRAPH)
    plan.set_points_batch(counts, xyz)
    out = torch.empty_like(dens)
    for _ in range(warmup + 1):                       # capture, then replays
        plan.evaluate(dens, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.evaluate(dens, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    n_total = int(sum(counts))
    res["laplace_sp_batch64_rhs16_p8_s2000"]["graph_replay"] = {
        "ms_per_replay": ms, "targets_per_s": n_total / (ms * 1e-3),
        "target_rhs_per_s": n_total * dens.shape[0] / (ms * 1e-3),
        "note": "one hipGraph replay of the whole evaluation of 64 problems x 16 RHS (points set once)"}
    log(f"batched forest, graph replay: {ms:.2f} ms, {n_total / (ms * 1e-3):.3e} targets/s")
    plan.close()
    del out
    del probs, xyz, dens
    pb = W.stokes_tp_clustered()
    xyz = torch.as_tensor(pb.points, device="cuda")
    run("stokes_tp_clustered_n16000000_p12_s2000_rhs4", pb.kernel, pb.periodic_mask, pb.p, pb.s,
        lambda pl: pl.set_points(xyz), torch.as_tensor(pb.density, device="cuda"), pb.n)
    return res


def paper_configs(pk, torch, W, ps, steps=2, warmup=1):
    """The paper's timing workloads (Section 3.5): 97^3 Chebyshev and lognormal
    points, Stokes, free space / SP / DP / TP, s = 1000, mixed form.  Per (periodicity, p) one
    plan serves both point sets.  set_points (octree, lists) stands beside the paper's tau_tree;
    the evaluation covers its tau_N and tau_F together (the far field is folded into the tree)."""
    res = []
    names = {0: "free", 1: "SP", 3: "DP", 7: "TP"}
    for mask in (0, 1, 3, 7):
        for p in ps:
            t0 = time.perf_counter()
            plan = pk.Plan(pk.STOKES, mask, p, 1000, precision=pk.MIXED, flags=pk.PHASE_TIMING)
            torch.cuda.synchronize()
            t_plan = time.perf_counter() - t0
            for kind in ("chebyshev", "lognormal"):
                pb = W.stokes_paper_points(kind, mask, p)
                xyz = torch.as_tensor(pb.points, device="cuda")
                dens = torch.as_tensor(pb.density, device="cuda")
                out = torch.empty_like(dens)
                for _ in range(warmup):
                    plan.set_points(xyz)
                    plan.evaluate(dens, out=out)
                torch.cuda.synchronize()
                plan.stats()
                t_sp = t_ev = 0.0
                for _ in range(steps):
                    a = time.perf_counter()
                    plan.set_points(xyz)
                    torch.cuda.synchronize()
                    b = time.perf_counter()
                    plan.evaluate(dens, out=out)
                    torch.cuda.synchronize()
                    t_sp += b - a
                    t_ev += time.perf_counter() - b
                st = plan.stats()
                rec = {"points": kind, "periodic": names[mask], "p": p, "s": 1000, "n": pb.n,
                       "ms_set_points": t_sp / steps * 1e3, "ms_evaluate": t_ev / steps * 1e3,
                       "targets_per_s": pb.n / ((t_sp + t_ev) / steps), "ms_phase": st["ms_phase"],
                       "plan_create_s": t_plan, "boxes": st["n_boxes"], "depth": st["depth"],
                       "near_pairs": st["near_pairs"]}
                res.append(rec)
                log(f"paper {kind} {names[mask]} p={p}: set_points {rec['ms_set_points']:.1f} ms, "
                    f"evaluate {rec['ms_evaluate']:.1f} ms")
                del xyz, dens, out
            plan.close()
    return res


def layer_configs(pk, torch, W, ps, steps=3, warmup=1):
    """Section 3.6, Table 4 (context): the 97^3 Chebyshev points, Stokes, triply periodic,
    s = 1000, with the near-field layer l = 1, 2, 3 (the root's image ring by M2L, the far-field
    operator over |p|_inf > l), both forms; set_points + evaluate per step and the device phase
    times.  The paper's tau_N and tau_F stay almost constant in l; so should these."""
    res = []
    pb = None
    for p in ps:
        pb = W.stokes_paper_points("chebyshev", 7, p)
        xyz = torch.as_tensor(pb.points, device="cuda")
        dens = torch.as_tensor(pb.density, device="cuda")
        for prec in (pk.MIXED, pk.FP64):
            for layers in (1, 2, 3):
                plan = pk.Plan(pk.STOKES, 7, p, 1000, precision=prec, flags=pk.PHASE_TIMING, near_layers=layers)
                out = torch.empty_like(dens)
                for _ in range(warmup):
                    plan.set_points(xyz)
                    plan.evaluate(dens, out=out)
                torch.cuda.synchronize()
                plan.stats()
                t0 = time.perf_counter()
                for _ in range(steps):
                    plan.set_points(xyz)
                    plan.evaluate(dens, out=out)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) / steps * 1e3
                st = plan.stats()
                rec = {"p": p, "near_layers": layers, "precision": "mixed" if prec == pk.MIXED else "fp64",
                       "ms_per_step": ms, "ms_phase": st["ms_phase"], "n_v": st["n_v"]}
                res.append(rec)
                log(f"layers p={p} l={layers} {rec['precision']}: {ms:.1f} ms/step, near {st['ms_phase']['near']:.1f} ms")
                plan.close()
        del xyz, dens
    return res


def precompute_configs(pk, torch, ps):
    """Section 3.7, Tables 5 and 6 (context): operator precompute (plan creation: kernel
    matrices, the two check-to-equivalent SVDs, M2M/L2L/M2L operators, the periodic far-field
    operator by lattice and Ewald sums, and for the mixed form the int8 slices) for Laplace DP and
    Stokes TP at l = 1, 2, 3 (Laplace DP: l = 1 only), float64 form; and the same plan loaded
    from the operator cache."""
    import tempfile
    res = []
    with tempfile.TemporaryDirectory() as d:
        for kern, mask, name, layers in ((pk.LAPLACE, 3, "laplace_dp", (1,)), (pk.STOKES, 7, "stokes_tp", (1, 2, 3))):
            for p in ps:
                for l in layers:
                    t0 = time.perf_counter()
                    plan = pk.Plan(kern, mask, p, 1000, precision=pk.FP64, near_layers=l, operator_cache_dir=d)
                    torch.cuda.synchronize()
                    t_build = time.perf_counter() - t0
                    plan.close()
                    t0 = time.perf_counter()
                    plan = pk.Plan(kern, mask, p, 1000, precision=pk.FP64, near_layers=l, operator_cache_dir=d)
                    torch.cuda.synchronize()
                    t_cache = time.perf_counter() - t0
                    plan.close()
                    rec = {"kernel": name, "p": p, "near_layers": l, "s_build": t_build, "s_from_cache": t_cache}
                    res.append(rec)
                    log(f"precompute {name} p={p} l={l}: built {t_build:.2f} s, from the cache {t_cache:.2f} s")
    return res


def cpu_baseline_runs(pb, repeats=3, one_core_leaves=3):
    """The oracle on the whole workload, `repeats` times on every host core (the median is the
    reported value), and once on one core over a bounded sample (tree, lists and the whole upward
    pass, then `one_core_leaves` random leaves, scaled to N)."""
    from threadpoolctl import threadpool_limits
    runs = []
    first = None
    for i in range(repeats):
        cb, fs = cpu_baseline(pb)
        runs.append(cb)
        if first is None:
            first = fs
        log(f"cpu baseline run {i + 1}: {cb['value']:.4g} targets/s")
    med = sorted(runs, key=lambda r: r["value"])[len(runs) // 2]
    rec = dict(med)
    rec["runs_targets_per_s"] = [r["value"] for r in runs]
    rec["sample"] = f"median of {repeats} runs of " + med["sample"]
    with threadpool_limits(limits=1):
        one, _ = cpu_baseline(pb, n_leaves_sample=one_core_leaves)
    rec["one_core"] = {"value": one["value"], "unit": "targets/s", "cores": 1, "sample": one["sample"]}
    log(f"cpu baseline, one core: {one['value']:.4g} targets/s")
    return rec, first


def cpu_baseline(pb, n_leaves_sample=None):
    """The oracle (plain FP64 CPU KIFMM) on the same workload: every leaf by default (the whole job),
    else a bounded sample of n_leaves_sample random leaves scaled to N."""
    from oracle import kifmm
    t0 = time.perf_counter()
    f = kifmm.KIFMM(pb.kernel, pb.periodic_mask, pb.p, pb.s, pb.points)     # operators + tree + lists
    t1 = time.perf_counter()
    f_ops = t1 - t0
    # second construction: operators cached, so this is the tree and lists alone
    t1 = time.perf_counter()
    f = kifmm.KIFMM(pb.kernel, pb.periodic_mask, pb.p, pb.s, pb.points)
    t_tree = time.perf_counter() - t1
    leaves = f.tree.leaves()
    whole = n_leaves_sample is None or n_leaves_sample >= len(leaves)
    if whole:
        pick = list(leaves)
    else:
        rng = np.random.default_rng(1)
        pick = [leaves[i] for i in sorted(rng.choice(len(leaves), n_leaves_sample, replace=False))]
    dens = pb.density[0]
    t2 = time.perf_counter()
    f.upward(np.ascontiguousarray(dens.reshape(-1, 3)[f.tree.perm]))
    t_up = time.perf_counter() - t2
    t3 = time.perf_counter()
    sub = f.evaluate(dens, target_leaves=pick)       # repeats the upward pass, then the picked leaves
    t_sample = time.perf_counter() - t3 - t_up
    n_sample = sum(f.tree.end[b] - f.tree.begin[b] for b in pick)
    # whole-job time: tree + upward once, downward/leaf work (scaled by points for a sample)
    t_full = t_tree + t_up + max(t_sample, 0.0) * (pb.n / n_sample)
    from threadpoolctl import threadpool_info
    cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or
                [int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))])
    if whole:
        sample = (f"the whole workload: tree+lists and upward pass ({t_tree + t_up:.1f} s), downward pass and "
                  f"leaf sums for all {n_sample} targets ({t_sample:.1f} s); operator precompute "
                  f"({f_ops:.1f} s) excluded")
    else:
        sample = (f"tree+lists and the full upward pass timed once ({t_tree + t_up:.1f} s); downward pass "
                  f"and leaf sums timed on {n_sample} targets in {len(pick)} random leaves "
                  f"({t_sample:.1f} s) and scaled to N; operator precompute ({f_ops:.1f} s) excluded")
    return {"value": pb.n / t_full, "unit": "targets/s", "cores": cores, "kind": "oracle",
            "sample": sample, "seconds_estimated_full": t_full}, (f, sub)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--configs", action="store_true",
                    help="also time the other configurations (DP slab, batched forest, clustered p=12) and add "
                         "them to the line under 'other_configs' (takes several minutes)")
    ap.add_argument("--paper", default="",
                    help="comma-separated p values (6..16): also time the paper's 97^3 Chebyshev and "
                         "lognormal Stokes workloads (free, SP, DP, TP; s = 1000) and add them under "
                         "'paper_configs'")
    ap.add_argument("--layers", default="",
                    help="comma-separated p values: also time the 97^3 Chebyshev TP Stokes workload at near-field "
                         "layers l = 1, 2, 3 (both forms) and add them under 'layer_configs'")
    ap.add_argument("--precompute", default="",
                    help="comma-separated p values: also time operator precompute (plan creation) for Laplace DP "
                         "and Stokes TP (l = 1, 2, 3) and from the operator cache; under 'precompute'")
    ap.add_argument("--tuning-file", default="",
                    help="launch choices for the N = 1M line (default: the package's tuning file)")
    ap.add_argument("--forms", default="fp64,mixed",
                    help="forms to time: 'fp64,mixed' (default) or 'mixed' alone (for counter passes)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (a plain copy kernel of known size, "
                         "to calibrate rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(a problem is evaluated on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1705_02043_amd as pk
    import workloads as W
    if args.copy_calibration_mib:
        src = torch.ones(args.copy_calibration_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    pb = W.stokes_tp_uniform()
    log(f"workload {pb.name}: N={pb.n} p={pb.p} s={pb.s}")
    forms = args.forms.split(",")
    r64 = out64 = None
    if "fp64" in forms:
        r64, out64 = time_form(pk, torch, pb, pk.FP64, args.steps, args.warmup, args.tuning_file)
        log(f"fp64: {r64['s_total'] / args.steps * 1e3:.2f} ms/step")
    rmx, outmx = time_form(pk, torch, pb, pk.MIXED, args.steps, args.warmup, args.tuning_file)
    log(f"mixed: {rmx['s_total'] / args.steps * 1e3:.2f} ms/step")
    ms_step = rmx["s_total"] / args.steps * 1e3
    st = rmx["stats"]
    # dominant kernel: the float32 near-field direct sums (phase "near": k_p2p plus the gather of
    # the reverse-direction sums), timed with HIP events on the stream they run on
    t_near = st["ms_phase"]["near"] * 1e-3
    achieved = FLOPS_PER_STOKES_PAIR * st["near_pairs"] / t_near / 1e12
    traffic, traffic_src = near_traffic()
    roofline = {"bound": "alu",
                "kernel": "k_p2p<3,true,1> + k_mutual_gather (near field: U lists + direct W/X, float32)",
                "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic, "traffic_source": traffic_src,
                "algorithmic": f"{FLOPS_PER_STOKES_PAIR} flop/pair x {st['near_pairs']} ordered (target, source) "
                               f"pairs per launch (a pair of different leaves is evaluated once, both ways)",
                "ms_per_launch": t_near * 1e3}
    rec = {
        "metric": METRIC,
        "value": pb.n / (ms_step * 1e-3),
        "unit": "targets/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "stokes_tp_uniform_n1000000_p8_s2000", "kernel": "stokes", "periodic": "xyz",
                   "n": pb.n, "p": pb.p, "s": pb.s, "n_rhs": 1, "seed": 2, "precision": "mixed"},
        "step": "set_points + evaluate",
        "mixed": {"ms_set_points": rmx["s_set_points"] * 1e3, "ms_evaluate": rmx["s_evaluate"] * 1e3,
                  "eval_only_targets_per_s": pb.n / rmx["s_evaluate"], "ms_phase": st["ms_phase"]},
        "plan_create_s": {"mixed": rmx["s_plan"]},
        "tree": {k: st[k] for k in ("n_boxes", "n_leaves", "depth", "n_u", "n_v", "n_w", "n_x", "u_pairs",
                                    "near_pairs")},
        "accuracy": {},
        "roofline": roofline,
        "launch_choices": {"near_workgroups_per_cu": st["tune_near_wpc"], "rhs_per_near_pass": st["tune_rb_near"],
                           "rhs_per_s2m_pass": st["tune_rb_s2m"],
                           "m2l_int8_tile": f'{st["tune_m2l_rows"]}x64',
                           "near_tile": "2 targets per thread x 256 threads, 256-source LDS tiles",
                           "source": (args.tuning_file if args.tuning_file else
                                      "autotuner record in " + os.path.relpath(pk.TUNING_FILE, ROOT)
                                      if os.path.exists(pk.TUNING_FILE) else "library defaults")},
    }
    if r64 is not None:
        rec["fp64"] = {"value": pb.n / (r64["s_total"] / args.steps), "ms_per_step": r64["s_total"] / args.steps * 1e3,
                       "ms_set_points": r64["s_set_points"] * 1e3, "ms_evaluate": r64["s_evaluate"] * 1e3,
                       "eval_only_targets_per_s": pb.n / r64["s_evaluate"], "ms_phase": r64["stats"]["ms_phase"]}
        rec["speedup_mixed_vs_fp64"] = r64["s_total"] / rmx["s_total"]
        rec["plan_create_s"]["fp64"] = r64["s_plan"]
        rec["accuracy"]["rel_l2_mixed_vs_fp64_gpu"] = float(np.linalg.norm(outmx - out64) / np.linalg.norm(out64))
    if args.configs:
        rec["other_configs"] = other_configs(pk, torch, W)
    if args.paper:
        rec["paper_configs"] = paper_configs(pk, torch, W, [int(x) for x in args.paper.split(",")])
    if args.layers:
        rec["layer_configs"] = layer_configs(pk, torch, W, [int(x) for x in args.layers.split(",")])
    if args.precompute:
        rec["precompute"] = precompute_configs(pk, torch, [int(x) for x in args.precompute.split(",")])
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb, (f, sub) = cpu_baseline_runs(pb)
        rec["cpu_baseline"] = cb
        num64 = nummx = den = 0.0
        for b, ref in sub.items():
            idx = f.tree.perm[f.tree.begin[b]:f.tree.end[b]]
            if out64 is not None:
                num64 += np.sum((out64[0][idx] - ref) ** 2)
            nummx += np.sum((outmx[0][idx] - ref) ** 2)
            den += np.sum(ref ** 2)
        rec["accuracy"]["rel_l2_vs_oracle"] = {"fp64": float(np.sqrt(num64 / den)) if out64 is not None else None,
                                                       "mixed": float(np.sqrt(nummx / den)),
                                                       "targets": int(sum(len(v) for v in sub.values()))}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
