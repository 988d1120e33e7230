"""Pins of the radial Euler reference (tests/radial_euler.py) used for the
cylindrical Sod problem of Sec. 6.2 (no GPU):
- without its geometric terms it is a 1D Euler solver: against the exact Riemann
  solution (gamma = 2) of the same data it converges at N = 1000, 2000, 4000;
- with them it conserves the mass int rho r dr to round-off while no wave has
  reached r = R, and a gas at rest stays at rest;
- its cylindrical solution is grid-converged at the resolution the GPU test uses.
"""
import numpy as np
import pytest

import radial_euler as RE
import riemann

IN, OUT = (1.0, 0.0, 5.0), (0.125, 0.0, 0.5)      # (rho, u, p) of the cylindrical Sod data
T_FINAL = 0.07


def test_planar_limit_is_the_riemann_solution():
    errs = []
    for n in (1000, 2000, 4000):
        x, rho, u, p, _ = RE.solve(n, T_FINAL, IN, OUT, planar=True, x_lo=0.0, R=1.0)
        ex = riemann.sample(IN, OUT, 2.0, (x - 0.5) / T_FINAL)
        errs.append(np.abs(rho - ex[:, 0]).mean() / np.abs(ex[:, 0]).mean())
        assert np.abs(p - ex[:, 2]).mean() / np.abs(ex[:, 2]).mean() < 0.01
    assert errs[-1] < 2e-3
    assert errs[0] > errs[1] > errs[2]


def test_cylindrical_mass_and_rest_state():
    x, rho, u, p, vol = RE.solve(800, 0.02, IN, OUT)           # waves still far from r = 1
    x0, rho0, u0, p0, _ = RE.solve(800, 0.0, IN, OUT)
    assert abs((rho * vol).sum() - (rho0 * vol).sum()) <= 1e-13 * (rho0 * vol).sum()
    x, rho, u, p, vol = RE.solve(400, 0.05, (0.7, 0.0, 1.3), (0.7, 0.0, 1.3))
    assert np.abs(rho - 0.7).max() <= 1e-13 and np.abs(u).max() <= 1e-13 and np.abs(p - 1.3).max() <= 1e-13


@pytest.mark.slow
def test_cylindrical_solution_grid_converged():
    x1, r1, u1, p1, _ = RE.solve(2000, T_FINAL, IN, OUT)
    x2, r2, u2, p2, _ = RE.solve(4000, T_FINAL, IN, OUT)
    r2c = 0.5 * (r2[0::2] + r2[1::2])
    assert np.abs(r1 - r2c).mean() / np.abs(r2c).mean() < 5e-3
    # the cylindrical solution differs from the planar one: the shock is weaker
    xp, rp, up, pp, _ = RE.solve(2000, T_FINAL, IN, OUT, planar=True)
    assert np.abs(r1 - rp).mean() > 1e-2
