"""Write tests/golden/mms2d_n80.json: the oracle's 2D manufactured-solution run
(Sec. 6.2, Table tab5-4) at N = 80 (80^4 phase-space points, about 12 minutes on
8 threads), too long for the test suite, which runs N = 20 and 40 live.  Calls
only the oracle.  The oracle source's SHA-256 is stored so a test can tell when
the stored run no longer matches the oracle."""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mm_workloads as W  # noqa: E402
import oracle  # noqa: E402


def oracle_sha():
    with open(os.path.join(ROOT, "oracle", "mm_oracle.c"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def main():
    with open(os.path.join(HERE, "mms2d_tab5_4.json")) as fh:
        gold = json.load(fh)
    n = 80
    p = W.problem2d(n, n, n, n, gold["V"], eps=gold["eps"], cfl=gold["cfl"], nu=gold["nu"], bc=W.periodic2d())
    t = time.time()
    macro, micro = oracle.mms2d(p, gold["t_final"])
    out = {"_source": "oracle.mms2d at N = 80 (tests/golden/make_mms2d_reference.py)",
           "N": n, "macro": macro, "micro": micro, "oracle_sha256": oracle_sha(),
           "seconds": round(time.time() - t, 1)}
    with open(os.path.join(HERE, "mms2d_n80.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


if __name__ == "__main__":
    main()
