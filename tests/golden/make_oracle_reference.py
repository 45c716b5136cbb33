"""Write tests/golden/oracle_stationary_128x96.npz: the oracle's run of the
stationary-ellipse 128x96 workload (Re 100, dt 1e-3, red-black SOR omega 1.8
to 1e-8 every 10 iterations, seeded 1e-3 noise), 100 steps.

Calls only the oracle.  Stored: per-step pressure iteration counts, residuals,
force coefficients, and u, v, p after steps 10 and 100.
Run:  python tests/golden/make_oracle_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2402_17337_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_stationary_128x96.npz")


def main():
    c = W.stationary_128x96()
    o = O.Oracle(c["nx"], c["ny"], c["xf"], c["yf"], c["u0"], c["v0"], c["p0"], **c["params"])
    keys = ("p_iters", "u_iters", "v_iters", "n_forced_u", "n_forced_v", "n_msrc", "status")
    fkeys = ("p_r0", "p_rel", "cd", "cl", "t")
    hist = {k: [] for k in keys + fkeys}
    snaps = {}
    t0 = time.time()
    for s in range(1, c["steps"] + 1):
        rc, st = o.step(1)
        assert rc == O.OK, st
        for k in keys + fkeys:
            hist[k].append(st[0][k])
        if s in (10, 100):
            u, v, p, phi = o.fields()
            snaps.update({f"u_{s}": u, f"v_{s}": v, f"p_{s}": p})
        print(f"step {s} iters {st[0]['p_iters']} {time.time() - t0:.1f}s", flush=True)
    np.savez_compressed(OUT, **{k: np.array(v) for k, v in hist.items()}, **snaps)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
