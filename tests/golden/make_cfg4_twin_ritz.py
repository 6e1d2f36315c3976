"""Write the FP64 oracle's Ritz values for the reduced cfg4 workload (60^3 periodic grid at
h = 0.22, 125 atoms x 4 projectors from a jittered FCC 4^3 lattice, Ns 900, degree 16) after
1..6 CheFSI iterations (Algorithm 1, scaled Chebyshev filter, bounds updated between
iterations) from the seeded X0, to tests/golden/cfg4_twin_ritz.txt (one row per iteration,
written as each iteration ends).

Only the oracle and the seeded input generator are used; the GPU tests compare the
library's whole solves with these values.  Takes about 80 minutes on 8 host cores.

    python tests/golden/make_cfg4_twin_ritz.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import chefsi as oc  # noqa: E402
from paper_2302_09708_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg4_twin_ritz.txt")


def main():
    cfg = inputs.CONFIGS["cfg4_twin"]
    prob = inputs.make_problem(cfg)
    x0 = inputs.initial_block(prob.nd, cfg.ns, cfg.x_seed).T
    lo, cut, hi = oc.spectral_bounds(prob)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle Ritz values (Ha) of the reduced cfg4 workload cfg4_twin\n")
        f.write(f"# grid {cfg.n} h {cfg.h} bc {cfg.bc}, {cfg.n_atoms} atoms x {cfg.nproj_per_atom} projectors, "
                f"Ns {cfg.ns}, degree {cfg.degree}, X0 seed {cfg.x_seed}\n")
        f.write("# bounds of the first step lam_lo lam_cut lam_hi: %.15e %.15e %.15e\n" % (lo, cut, hi))
        f.write("# row k = Ritz values after k+1 iterations (Algorithm 1), ascending\n")
        f.write("# written by tests/golden/make_cfg4_twin_ritz.py (oracle only)\n")

        def record(it, d, x, lam_lo, lam_cut):
            f.write(" ".join(f"{v:.15e}" for v in d) + "\n")
            f.flush()
            print(f"iteration {it + 1}: D_1 = {d[0]:.12f}", flush=True)

        oc.chefsi(prob, x0, cfg.degree, cfg.n_iter, lo, cut, hi, callback=record)


if __name__ == "__main__":
    main()
