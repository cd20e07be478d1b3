"""Write the exact triply periodic Stokes sums at sampled targets of the triply periodic
workloads (uniform N = 1M; 200 Gaussian clusters + 20 % uniform, N = 16M, 4 right-hand sides;
the paper's 97^3 Chebyshev points of Section 3.5, whose density does not depend on p),
by the oracle's structure-factor Ewald sum alone (oracle/_native.tp_ewald_targets, pinned against
the pairwise Ewald sum in tests/test_oracle_targets_ewald.py).  The GPU tests read them to state
the method's error against the definition at full size.

python tests/golden/make_tp_exact_subsample.py [c2|c5|paper_cheb ...]   (c5 takes tens of minutes on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W                      # noqa: E402
from oracle import _native                 # noqa: E402

CASES = {
    "c2": (lambda: W.stokes_tp_uniform(), 1000, 20),
    "c5": (lambda: W.stokes_tp_clustered(), 1000, 21),
    "paper_cheb": (lambda: W.stokes_paper_points("chebyshev", W.TP), 300, 22),
}


def main(names):
    for name in names:
        make, n_targets, seed = CASES[name]
        pb = make()
        idx = np.sort(np.random.default_rng(seed).choice(pb.n, n_targets, replace=False))
        t0 = time.time()
        val = _native.tp_ewald_targets(pb.kernel, pb.points[idx], pb.points, pb.density)
        out = os.path.join(HERE, f"tp_exact_{name}.npz")
        np.savez(out, targets=idx, values=val, n=pb.n, seed_targets=seed)
        print(f"{name}: {n_targets} targets x {pb.density.shape[0]} RHS from N = {pb.n} in {time.time() - t0:.0f} s"
              f" -> {out}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
