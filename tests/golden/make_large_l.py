"""Writes the oracle references of the L = 4096 parity tests (tests/golden/l4096_*.npz).

At L = 4096 the oracle's sampled-order transforms (Risbo recursion over full
planes to l = 4095, direct DFT sums) take minutes, so the references are
computed once here, by the oracle alone, from the seeded generators of
``mwsynth``, and stored.  Each file holds the orders, the inverse of the seeded
coefficients on those orders (phi-Fourier coefficients F_m(theta_t) of the
rings, t < L) and the forward of a seeded grid on those orders (f_{l,m},
l = |m| .. L-1).  Run: ``python tests/golden/make_large_l.py``.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import mwsynth  # noqa: E402
import oracle   # noqa: E402

L = 4096
# (name, spin, real, coefficient recipe, orders)
CASES = [
    ("l4096_s0_real", 0, 1, lambda: mwsynth.flm_cl_real(L, seed=1014), [0, 1, L // 2, L - 1]),
    ("l4096_s2", 2, 0, lambda: mwsynth.flm_gaussian(L, 2, seed=1114, decay=1.0), [0, 2, L // 2, L - 1, -1, -(L - 1)]),
]
# seeds of the (not band-limited) forward input grids
GRID_SEED = {"l4096_s0_real": 1214, "l4096_s2": 1314}


def main():
    oracle.build(force=False)
    for name, s, real, make_flm, ms in CASES:
        t0 = time.time()
        flm = make_flm()
        inv = oracle.inverse_orders(flm, L, s, ms)
        t1 = time.time()
        grid = mwsynth.grid_gaussian(L, seed=GRID_SEED[name], real=bool(real)).astype(np.complex128)
        fwd = oracle.forward_orders(grid, L, s, ms)
        t2 = time.time()
        np.savez(os.path.join(HERE, name + ".npz"), L=L, spin=s, real=real, orders=np.array(ms),
                 grid_seed=GRID_SEED[name], inverse_orders=inv, forward_orders=fwd)
        print("%s: inverse %.0f s, forward %.0f s" % (name, t1 - t0, t2 - t1), flush=True)


if __name__ == "__main__":
    main()
