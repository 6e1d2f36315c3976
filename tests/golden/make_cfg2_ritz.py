"""Write the FP64 oracle's Ritz values for the cfg2 workload itself (72^3 periodic grid at
h = 0.25, 128 atoms x 4 projectors on a jittered bcc 4^3 lattice, Ns 600, degree 20) after
1..10 CheFSI iterations (Algorithm 1, scaled Chebyshev filter, bounds updated between
iterations as oracle.chefsi.chefsi does) from the seeded X0, to tests/golden/cfg2_ritz.txt
(one row per iteration, written as each iteration ends).

Only the oracle and the seeded input generator are used; the GPU tests compare the
library's whole solves with these values.  The oracle's filter acts on each column on its
own, so it runs here over 8 column blocks in worker processes (the results equal the
one-block filter up to the summation order of the projector products); projection,
diagonalisation and rotation take the whole block.  About 60 minutes on 8 host cores.

    python tests/golden/make_cfg2_ritz.py
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import chefsi as oc  # noqa: E402
from paper_2302_09708_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg2_ritz.txt")
WORKERS = 8
_PROB = None


def _filter_block(args):
    global _PROB
    if _PROB is None:
        _PROB = inputs.make_problem(inputs.CONFIGS["cfg2"])
    x, degree, lo, cut, hi = args
    return oc.chebyshev_filter(_PROB, x, degree, lo, cut, hi)


def main():
    cfg = inputs.CONFIGS["cfg2"]
    prob = inputs.make_problem(cfg)
    x = np.array(inputs.initial_block(prob.nd, cfg.ns, cfg.x_seed).T, dtype=np.float64)
    lo, cut, hi = oc.spectral_bounds(prob)
    with open(OUT, "w") as f, ProcessPoolExecutor(WORKERS) as pool:
        f.write("# FP64 oracle Ritz values (Ha) of the cfg2 workload\n")
        f.write(f"# grid {cfg.n} h {cfg.h} bc {cfg.bc}, {cfg.n_atoms} atoms x {cfg.nproj_per_atom} projectors, "
                f"Ns {cfg.ns}, degree {cfg.degree}, X0 seed {cfg.x_seed}\n")
        f.write("# bounds of the first step lam_lo lam_cut lam_hi: %.15e %.15e %.15e\n" % (lo, cut, hi))
        f.write("# row k = Ritz values after k+1 iterations (Algorithm 1), ascending\n")
        f.write("# written by tests/golden/make_cfg2_ritz.py (oracle only)\n")
        f.flush()
        lam_lo, lam_cut = lo, cut
        for it in range(cfg.n_iter):
            blocks = np.array_split(x, WORKERS, axis=1)
            xf = np.hstack(list(pool.map(_filter_block, [(b, cfg.degree, lam_lo, lam_cut, hi) for b in blocks])))
            hs, ms = oc.project(prob, xf)
            d, z = oc.diagonalize(hs, ms)
            x = oc.rotate(xf, z)
            lam_lo, lam_cut = d[0], d[-1]
            f.write(" ".join(f"{v:.15e}" for v in d) + "\n")
            f.flush()
            print(f"iteration {it + 1}: D_1 = {d[0]:.12f}", flush=True)


if __name__ == "__main__":
    main()
