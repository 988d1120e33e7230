"""Pins of the oracle's 1D diffuse walls (Sec. 4.3: wall_bc_1/2, the wall densities
of zero mass flux, the KFVS wall fluxes, H_{1/2} = H_1 / 2) and of the
heat-transfer runs of that section (walls at T_C = 1 and T_H = 1.2, tau = p,
(x, v) in [0, 1] x [-6, 6], CFL 0.95, t = 100).

What fixes them:
- a gas at rest at the walls' common temperature stays at rest (the wall
  densities and fluxes balance the cell's exactly, up to rounding);
- no mass crosses a wall: the total mass is constant to rounding in any run
  (a wall density taken from the wrong half-range breaks it);
- the mirrored problem (walls swapped, x -> 1 - x) gives the mirrored solution;
- the printed limits of the Knudsen sweep: the scaled heat flux |h_1| at x = 0.5
  tends to the Navier-Stokes-Fourier value kappa (T_H - T_C) = 0.3 as eps -> 0,
  the distribution at eps = 1e30 is the free-molecular one (two half-Maxwellians
  from the walls, zero net mass flux, uniform density), and |h_1| stays near the
  harmonic average of the two limits across the sweep.
"""
import math

import numpy as np
import pytest

import mm_workloads as W
import oracle

TC, TH = 1.0, 1.2
H_FREE = 0.083422728489775170621      # (sqrt(T_H) - sqrt(T_C)) sqrt(2 T_C T_H / pi), printed
H_NSF = 0.3                            # kappa (T_H - T_C) with kappa = 1.5, printed


def heat_problem(n, eps, t_c=TC, t_h=TH, cfl=0.95):
    p = W.problem1d(n, n, 6.0, eps=eps, cfl=cfl, tau_model="p", tau_coef=1.0)
    p["bc"][0] = {"kind": "wall", "T_wall": t_c}
    p["bc"][1] = {"kind": "wall", "T_wall": t_h}
    return p


def test_closed_form_constants():
    """The printed free-molecular constant and the harmonic average's constants."""
    assert (math.sqrt(TH) - math.sqrt(TC)) * math.sqrt(2 * TC * TH / math.pi) == pytest.approx(H_FREE, rel=1e-15)
    # |h_nsf| |h_free| / (|h_nsf| + |h_free|) = H_FREE / (H_FREE / H_NSF + eps)
    assert H_FREE / H_NSF == pytest.approx(0.2780757616325839021, rel=1e-15)


def test_rest_state_at_wall_temperature_is_stationary():
    n = 24
    p = heat_problem(n, 0.05, t_c=0.9, t_h=0.9)
    Q = W.conserved1d(np.full(n, 1.3), np.zeros(n), np.full(n, 0.9))
    G = np.zeros((n, n))
    Q1, G1, H = oracle.run(p, Q.reshape(-1), G.reshape(-1), 50)
    assert np.abs(Q1 - Q.reshape(-1)).max() <= 1e-13
    assert np.abs(G1).max() <= 1e-12


def _flowing_state(n):
    x = W.centres(0.0, 1.0, n)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x) ** 2
    u = 0.2 * np.sin(np.pi * x) + 0.1
    T = 1.0 + 0.2 * x
    return W.conserved1d(rho, u, T)


def test_walls_conserve_mass():
    n = 40
    p = heat_problem(n, 0.05)
    Q = _flowing_state(n)
    m0 = Q[:, 0].sum()
    Q1, G1, H = oracle.run(p, Q.reshape(-1), np.zeros(n * n), 400)
    Q1 = Q1.reshape(n, 3)
    assert abs(Q1[:, 0].sum() - m0) <= 1e-13 * m0
    # the walls did act: the gas is no longer what it was
    assert np.abs(Q1 - Q).max() > 1e-2


def test_mirror_symmetry():
    n, steps = 30, 300
    Q = _flowing_state(n)
    p = heat_problem(n, 0.02)
    Qa, Ga, Ha = oracle.run(p, Q.reshape(-1), np.zeros(n * n), steps)
    # mirrored: x -> 1 - x, u -> -u, walls swapped
    Qm = Q[::-1].copy()
    Qm[:, 1] *= -1.0
    pm = heat_problem(n, 0.02, t_c=TH, t_h=TC)
    Qb, Gb, Hb = oracle.run(pm, Qm.reshape(-1), np.zeros(n * n), steps)
    Qb = Qb.reshape(n, 3)[::-1]
    Qb[:, 1] *= -1.0
    Gb = Gb.reshape(n, n)[::-1, ::-1]
    Qa = Qa.reshape(n, 3)
    Ga = Ga.reshape(n, n)
    assert np.abs(Qa - Qb).max() <= 1e-12 * np.abs(Qa).max()
    assert np.abs(Ga - Gb).max() <= 1e-10 * np.abs(Ga).max()


def knudsen_run(n, eps, t_final=100.0):
    """(|h_1| at x = 0.5, Q, G) after t_final (N_x = N_v = n, odd, so x = 0.5 is a cell centre)."""
    p = heat_problem(n, eps)
    dt, nsteps = oracle.dt(p, t_final)
    p["dt"] = dt
    Q = W.conserved1d(np.ones(n), np.zeros(n), np.ones(n))
    Q1, G1, H = oracle.run(p, Q.reshape(-1), np.zeros(n * n), nsteps)
    # H = (eps / 2) dv sum v^3 G, and |h_1| = (1/2) |dv sum v^3 g| with f = M + eps g
    return abs(H[n // 2]) / eps, Q1.reshape(n, 3), G1.reshape(n, n)


@pytest.mark.slow
def test_free_molecular_limit_distribution():
    """eps = 1e30 (no collisions): at x = 0.5 the distribution f = M + eps g is the free-molecular
    one, the wall Maxwellians at T_C on v > 0 and T_H on v < 0 with rho_C sqrt(T_C) =
    rho_H sqrt(T_H) and mean density 1 (the section's Fig. b comparison)."""
    n, eps = 65, 1e30
    h, Q, G = knudsen_run(n, eps)
    v = W.centres(-6.0, 6.0, n)
    i = n // 2
    rho, m, E = Q[i]
    u = m / rho
    T = 2 * E / rho - u * u
    f = rho / math.sqrt(2 * math.pi * T) * np.exp(-(v - u) ** 2 / (2 * T)) + eps * G[i]
    a = 2 * math.sqrt(TC * TH) / (math.sqrt(TC) + math.sqrt(TH))
    rc, rh = a / math.sqrt(TC), a / math.sqrt(TH)
    fe = np.where(v > 0, rc / math.sqrt(2 * math.pi * TC) * np.exp(-v * v / (2 * TC)),
                  rh / math.sqrt(2 * math.pi * TH) * np.exp(-v * v / (2 * TH)))
    k0 = np.argmin(np.abs(v))                       # the node on the jump at v = 0
    fe[k0] = 0.5 * (rc / math.sqrt(2 * math.pi * TC) + rh / math.sqrt(2 * math.pi * TH))
    assert np.abs(f - fe).max() <= 0.03 * fe.max()
    assert abs(rho - 1.0) <= 1e-3 and abs(u) <= 1e-3
    assert T == pytest.approx(math.sqrt(TC * TH), rel=2e-3)      # (rho_C T_C + rho_H T_H) / 2
    # the heat flux is the free-molecular one's order, from below
    assert 0.65 * H_FREE / eps < h < H_FREE / eps


@pytest.mark.slow
def test_heat_flux_across_the_knudsen_sweep():
    """|h_1| at x = 0.5, t = 100: near kappa (T_H - T_C) = 0.3 at eps = 1e-2 and approaching it
    with resolution; between the harmonic average of the printed limits and 0.7 times it across
    the sweep; decreasing in eps."""
    h33 = {eps: knudsen_run(33, eps)[0] for eps in (1e-2, 1.0, 1e30)}
    h65 = knudsen_run(65, 1e-2)[0]
    assert h33[1e-2] < h65 < H_NSF
    assert h65 >= 0.93 * H_NSF
    for eps, h in h33.items():
        harm = H_FREE / (H_FREE / H_NSF + eps)
        assert 0.7 * harm <= h <= harm, (eps, h, harm)
    assert h33[1e-2] > h33[1.0] > h33[1e30]
