"""The cylindrical Sod problem of Sec. 6.2 on the GPU: 320^2 x 14^2 phase-space cells,
213 steps to t = 0.07 (the printed step count, which the rule CFL = dt (V1/dx + V2/dy)
reproduces), at the three Knudsen numbers of the section, against the radial Euler
solution (tests/radial_euler.py) as eps -> 0; and a reduced run element by element
against the oracle."""
import numpy as np
import pytest

import mm_workloads as W
import oracle
import radial_euler as RE
from gpu_common import log, rel_l1, run_gpu

pytestmark = pytest.mark.gpu

T_FINAL = 0.07


def test_cylsod_parity_with_oracle():
    p, Q, G = W.cylsod2d(nx=48, nv=14, eps=5e-3)
    log("[cylsod] 48^2 x 14^2, 30 steps")
    Qg, Gg, Hg = run_gpu(p, Q, G, 30)
    Qo, Go, Ho = oracle.run(p, Q.reshape(-1), G.reshape(-1), 30)
    e = rel_l1(Qg, Qo)
    log(f"[cylsod] Q rel-L1 vs oracle {e:.3e}")
    assert e <= 1e-12
    assert np.abs(Gg - Go).max() <= 1e-10 * np.abs(Go).max() + 1e-13 * np.abs(Qo).max() / p["eps"]


def _radial_profiles(p, Q):
    """Per cell: r and (rho, |u|, p, T) of the 2D state."""
    n = p["nx"]
    x = W.centres(-1.0, 1.0, n)
    X, Y = np.meshgrid(x, x)
    Q = Q.reshape(n, n, 6)
    rho = Q[..., 0]
    u1, u2 = Q[..., 1] / rho, Q[..., 2] / rho
    pr = 0.5 * (Q[..., 3] - rho * u1 * u1 + Q[..., 5] - rho * u2 * u2)
    return np.hypot(X, Y).ravel(), np.stack([rho, np.hypot(u1, u2), pr, pr / rho], -1).reshape(-1, 4)


def test_cylsod_printed_run_approaches_euler():
    from paper_2509_21832_amd import binding as B
    rr, rho_r, u_r, p_r, _ = RE.solve(4000, T_FINAL, (1.0, 0.0, 5.0), (0.125, 0.0, 0.5))
    ref = np.stack([rho_r, np.abs(u_r), p_r, p_r / rho_r], -1)
    errs = {}
    for eps in (5e-3, 5e-4, 5e-5):
        p, Q, G = W.cylsod2d(eps=eps)
        dt, n = B.dt(p, T_FINAL)
        assert n == 213
        p["dt"] = dt
        log(f"[cylsod 320^2 x 14^2] eps={eps:g}: {n} steps, dt {dt:.6e}")
        Qg, Gg, Hg = run_gpu(p, Q, G, n)
        r, prof = _radial_profiles(p, Qg)
        keep = r < 0.95
        exact = np.stack([np.interp(r[keep], rr, ref[:, k]) for k in range(4)], -1)
        e = np.abs(prof[keep] - exact).mean(0) / np.abs(exact).mean(0)
        errs[eps] = e
        log(f"[cylsod] eps={eps:g}: relative L1 error of (rho, |u|, p, T) vs radial Euler {np.round(e, 4)}")
        # the data and the scheme are symmetric under x -> -x and y -> -y (the sweeps run
        # x then y, so a swap of x and y is not a symmetry of the discrete step)
        Qq = Qg.reshape(p["nx"], p["nx"], 6)
        assert np.abs(Qq[:, :, 0] - Qq[:, ::-1, 0]).max() <= 1e-10 * Qq[:, :, 0].max()
        assert np.abs(Qq[:, :, 0] - Qq[::-1, :, 0]).max() <= 1e-10 * Qq[:, :, 0].max()
    # the error against the Euler limit shrinks with eps (density and pressure)
    assert errs[5e-5][0] < errs[5e-3][0] and errs[5e-5][2] < errs[5e-3][2]
    assert errs[5e-5][0] < 0.05 and errs[5e-5][2] < 0.05
