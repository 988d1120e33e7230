"""Write the oracle's macro state after 100 steps of the 256^2 x 32^2 cavity
workload (seed 0) for eps in {1e-3, 3e-3, 1e-2, 1e-1, 1}.

Calls only the oracle.  Stored per eps: Q on every 4th cell in x and y
(64 x 64 x 6 values, float64), Q of the whole boundary ring (the first and last
row and column, which hold the lid and the wall cells), and the domain sums of
Q over all cells.
Run:  python tests/golden/make_c3_reference.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mm_workloads as W  # noqa: E402
import oracle  # noqa: E402

EPS = (1e-3, 3e-3, 1e-2, 1e-1, 1.0)
STEPS = 100
STRIDE = 4


def main():
    if len(sys.argv) > 1:
        oracle.set_threads(int(sys.argv[1]))
    out = {}
    for eps in EPS:
        t0 = time.time()
        p, Q, G = W.cavity2d(seed=0, eps=eps)
        Q1, G1, H = oracle.run(p, Q.reshape(-1), G.reshape(-1), STEPS)
        Q1 = Q1.reshape(p["ny"], p["nx"], 6)
        key = f"eps{eps:g}"
        out[key + "_sample"] = Q1[::STRIDE, ::STRIDE, :].copy()
        out[key + "_row_lo"] = Q1[0].copy()
        out[key + "_row_hi"] = Q1[-1].copy()
        out[key + "_col_lo"] = Q1[:, 0].copy()
        out[key + "_col_hi"] = Q1[:, -1].copy()
        out[key + "_sum"] = Q1.reshape(-1, 6).sum(0)
        out[key + "_abssum"] = np.abs(Q1).reshape(-1, 6).sum(0)
        print(f"eps={eps:g}: {time.time() - t0:.1f} s", flush=True)
    out["stride"] = np.array(STRIDE)
    out["steps"] = np.array(STEPS)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_cavity_100steps.npz"), **out)


if __name__ == "__main__":
    main()
