"""Record the autotuner's launch choices for the standard workloads on this device.

python -m paper_1705_02043_amd.tune [--out FILE]

Runs pkifmm_autotune (bit-neutral launch choices: near-field workgroups per compute unit and the
right-hand sides per geometry pass) on the Stokes triply periodic workload (N = 1M, p = 8,
s = 2000; both forms), the 64-problem singly periodic Laplace forest (16 right-hand sides,
p = 8, s = 2000; mixed form), the doubly periodic Stokes slab (N = 4M, p = 10, s = 2000; mixed
form) and the clustered triply periodic Stokes points (N = 16M, p = 12, 4 right-hand sides;
mixed form), and writes their records to FILE (default: the package's tuning file, which Plan
reads).
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.dirname(here))
    import torch
    import paper_1705_02043_amd as pk
    import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=pk.TUNING_FILE)
    ap.add_argument("--skip-large", action="store_true", help="skip the 4M-point slab and the 16M clustered points")
    args = ap.parse_args()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)

    def tune(name, kernel, mask, p, s, precision, set_pts, dens):
        plan = pk.Plan(kernel, mask, p, s, precision=precision, tuning_file=None)
        set_pts(plan)
        choice = plan.autotune(dens, tuning_file=args.out)
        print(f"{name} precision={precision}: {choice}", flush=True)
        plan.close()

    pb = W.stokes_tp_uniform()
    xyz, dens = torch.as_tensor(pb.points, device="cuda"), torch.as_tensor(pb.density, device="cuda")
    for prec in (pk.MIXED, pk.FP64):
        tune("stokes_tp_n1m_p8", pb.kernel, pb.periodic_mask, pb.p, pb.s, prec, lambda pl: pl.set_points(xyz), dens)
    del xyz, dens
    probs = W.laplace_sp_batch()
    counts = [q.n for q in probs]
    xyz = torch.as_tensor(np.concatenate([q.points for q in probs]), device="cuda")
    dens = torch.as_tensor(np.concatenate([q.density for q in probs], axis=1), device="cuda")
    tune("laplace_sp_batch64_rhs16", probs[0].kernel, probs[0].periodic_mask, probs[0].p, probs[0].s, pk.MIXED,
         lambda pl: pl.set_points_batch(counts, xyz), dens)
    del xyz, dens, probs
    if not args.skip_large:
        pb = W.stokes_dp_slab()
        xyz, dens = torch.as_tensor(pb.points, device="cuda"), torch.as_tensor(pb.density, device="cuda")
        tune("stokes_dp_slab_n4m_p10", pb.kernel, pb.periodic_mask, pb.p, pb.s, pk.MIXED,
             lambda pl: pl.set_points(xyz), dens)
        del xyz, dens
        pb = W.stokes_tp_clustered()
        xyz, dens = torch.as_tensor(pb.points, device="cuda"), torch.as_tensor(pb.density, device="cuda")
        tune("stokes_tp_clustered_n16m_p12_rhs4", pb.kernel, pb.periodic_mask, pb.p, pb.s, pk.MIXED,
             lambda pl: pl.set_points(xyz), dens)
    print(open(args.out).read(), flush=True)


if __name__ == "__main__":
    main()
