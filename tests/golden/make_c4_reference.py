"""Write the oracle's state after 10 and after 100 steps of the 512^2 x 48^2
Gaussian-blast workload (seed 0, eps = 1e-2, diffuse walls).

Calls only the oracle.  Stored per checkpoint: Q on every 8th cell in x and y
(64 x 64 x 6 values, float64), the domain sums of Q and of |Q| over all cells,
and g (all 2304 velocity nodes) on a fixed set of 16 cells.
Run:  python tests/golden/make_c4_reference.py [threads]
(about 20 GB of host memory; about an hour on 8 cores)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mm_workloads as W  # noqa: E402
import oracle  # noqa: E402

CHECKPOINTS = (10, 100)
STRIDE = 8
# cells (j, i) whose full g is stored: corners, wall-adjacent, the blast core, interior
G_CELLS = np.array([(0, 0), (0, 255), (511, 511), (255, 0), (256, 256), (250, 262), (270, 240), (128, 384),
                    (384, 128), (1, 1), (510, 300), (300, 510), (200, 200), (320, 320), (64, 448), (448, 64)])


def main():
    if len(sys.argv) > 1:
        oracle.set_threads(int(sys.argv[1]))
    p, Q, G = W.blast2d(seed=0)
    Q, G = Q.reshape(-1), G.reshape(-1)
    out = {}
    done = 0
    t0 = time.time()
    for n in CHECKPOINTS:
        Q, G, H = oracle.run(p, Q, G, n - done)
        done = n
        Qc = Q.reshape(p["ny"], p["nx"], 6)
        Gc = G.reshape(p["ny"], p["nx"], p["nv2"] * p["nv1"])
        key = f"step{n}"
        out[key + "_sample"] = Qc[::STRIDE, ::STRIDE, :].copy()
        out[key + "_sum"] = Qc.reshape(-1, 6).sum(0)
        out[key + "_abssum"] = np.abs(Qc).reshape(-1, 6).sum(0)
        out[key + "_g"] = np.stack([Gc[j, i] for j, i in G_CELLS])
        print(f"step {n}: {time.time() - t0:.1f} s", flush=True)
        np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_blast_checkpoints.npz"),
                            stride=np.array(STRIDE), g_cells=G_CELLS, steps=np.array(sorted(out_steps(out))),
                            **out)


def out_steps(out):
    return [int(k[4:-7]) for k in out if k.endswith("_sample")]


if __name__ == "__main__":
    main()
