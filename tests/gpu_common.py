"""Helpers of the GPU parity tests: run the HIP path (through the C ABI) and
the oracle on the same seeded inputs and compare element by element."""
import math
import os
import sys

import numpy as np

import oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class _env:
    """Set (or clear) one environment variable for the duration of a block."""

    def __init__(self, name, on):
        self.name, self.on = name, on

    def __enter__(self):
        self.old = os.environ.pop(self.name, None)
        if self.on:
            os.environ[self.name] = "1"

    def __exit__(self, *a):
        os.environ.pop(self.name, None)
        if self.old is not None:
            os.environ[self.name] = self.old


def run_gpu(p, Q, G, nsteps, chunks=1, reference=False, generic=False):
    """Run the HIP path.  reference=True selects the unfused phase-space pass
    (the library reads MM_REFERENCE_PASS when a context is created);
    generic=True forces the generic fused kernel where the lane-k one would
    run (MM_GENERIC_FUSED, read at each launch)."""
    from paper_2509_21832_amd import binding as B
    with _env("MM_REFERENCE_PASS", reference):
        s = B.Solver(p, Q, G)
    with s, _env("MM_GENERIC_FUSED", generic):
        per = nsteps // chunks
        done = 0
        while done < nsteps:
            n = min(per, nsteps - done)
            s.step(n)
            done += n
        Qg, Hg = s.moments(with_h=True)
        Gg = s.get_g()
    return Qg, Gg, Hg


def rel_l1(a, b):
    """Pooled relative L1 error sum |a - b| / sum |b|."""
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def maxwell_scale(p, Q):
    """Largest Maxwellian value rho / ((2 pi T)^{d_v/2}) of the state (size of G's round-off)."""
    if p["dim"] == 1:
        Qc = Q.reshape(-1, 3)
        rho = Qc[:, 0]
        u = Qc[:, 1] / rho
        T = 2 * Qc[:, 2] / rho - u * u
        return float(np.max(rho / np.sqrt(2 * math.pi * T)))
    Qc = Q.reshape(-1, 6)
    rho = Qc[:, 0]
    u1, u2 = Qc[:, 1] / rho, Qc[:, 2] / rho
    T = 0.5 * ((Qc[:, 3] - rho * u1 * u1) + (Qc[:, 5] - rho * u2 * u2)) / rho
    return float(np.max(rho / (2 * math.pi * T)))


def compare(p, Q0, Qg, Gg, Hg, Qo, Go, Ho, q_l1=1e-12, q_el=1e-11, g_rel=1e-10, label=""):
    """Element-by-element comparison of the GPU result (g) with the oracle (o)."""
    nc = 6 if p["dim"] == 2 else 3
    Qg = Qg.reshape(-1, nc)
    Qo = Qo.reshape(-1, nc)
    e1 = rel_l1(Qg, Qo)
    scale = np.abs(Qo).mean(0)
    el = np.abs(Qg - Qo) / (np.abs(Qo) + scale)
    gtol = g_rel * np.abs(Go).max() + 1e-13 * maxwell_scale(p, Q0) / p["eps"]
    gerr = np.abs(Gg - Go).max()
    htol = max(1e-9, 10 * g_rel) * np.abs(Ho).max() + 1e-12 * gtol * p["eps"]
    herr = np.abs(Hg - Ho).max()
    log(f"[{label}] Q rel-L1 {e1:.3e}  Q max el {el.max():.3e}  G max abs {gerr:.3e} (tol {gtol:.2e})"
        f"  H max abs {herr:.3e} (tol {htol:.2e})")
    assert np.all(np.isfinite(Qg)) and np.all(np.isfinite(Gg))
    assert e1 <= q_l1, f"Q rel-L1 {e1}"
    assert el.max() <= q_el, f"Q elementwise {el.max()}"
    assert gerr <= gtol, f"G {gerr} > {gtol}"
    assert herr <= htol, f"H {herr} > {htol}"
    return e1


MIXED_TOL = dict(q_l1=1e-5, q_el=1e-4, g_rel=1e-4)


def parity(p, Q, G, nsteps, label="", chunks=1, reference=False, generic=False, **tol):
    log(f"[{label}] start: nx={p['nx']} ny={p.get('ny', 1)} nv={p['nv1']}x{p.get('nv2', 1)} "
        f"steps={nsteps} eps={p['eps']} precision={p.get('precision', 'fp64')} reference={reference} "
        f"generic={generic}")
    if p.get("precision", "fp64") != "fp64":
        for k, v in MIXED_TOL.items():
            tol.setdefault(k, v)
    Qg, Gg, Hg = run_gpu(p, Q, G, nsteps, chunks, reference, generic)
    Qo, Go, Ho = oracle.run(p, Q.reshape(-1), G.reshape(-1), nsteps)
    return compare(p, Q, Qg, Gg, Hg, Qo, Go, Ho, label=label, **tol)
