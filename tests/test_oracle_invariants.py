"""Invariants the paper fixes for the whole step: conservation, zero conserved
moments of g, equilibrium, the asymptotic-preserving limit and mirror
symmetries (no GPU)."""
import numpy as np
import pytest

import mm_workloads as W
import oracle


def _mom_g(p, G):
    """dv sum (1, v1, v2, |v|^2) G per cell, and dv sum |G| (scale)."""
    ny, nx, nv2, nv1 = p["ny"], p["nx"], p["nv2"], p["nv1"]
    G = G.reshape(ny * nx, nv2, nv1)
    v1 = W.centres(*p["v1"], nv1)
    v2 = W.centres(*p["v2"], nv2)
    V1, V2 = np.meshgrid(v1, v2)
    m = np.stack([np.einsum("ckl,kl->c", G, f) for f in (np.ones_like(V1), V1, V2, V1 ** 2 + V2 ** 2)], 1)
    s = np.einsum("ckl->c", np.abs(G)) * (1 + np.abs(V1).max() ** 2)
    return m, s


@pytest.mark.parametrize("mode", ["discrete", "paper"])
def test_conservation_periodic_2d(mode):
    p, Q, G = W.smooth2d(seed=1, nx=12, ny=10, nv=16, eps=0.05, proj_mode=mode)
    Q1, G1, H = oracle.run(p, Q.reshape(-1), G.reshape(-1), 60)
    s0 = Q.reshape(-1, 6).sum(0)
    s1 = Q1.reshape(-1, 6).sum(0)
    scale = np.abs(Q).reshape(-1, 6).sum(0)
    for r in (0, 1, 2):
        assert abs(s1[r] - s0[r]) < 1e-13 * scale[r]
    # scalar energy E = (E11 + E22)/2
    assert abs((s1[3] + s1[5]) - (s0[3] + s0[5])) < 1e-13 * (scale[3] + scale[5])
    assert np.abs(G1).max() > 1e-4           # the micro part is not trivially zero


def test_mass_conservation_walls():
    p, Q, G = W.quadrant2d(seed=2, nx=10, ny=12, nv=12)
    Q1, G1, H = oracle.run(p, Q.reshape(-1), G.reshape(-1), 40)
    assert abs(Q1.reshape(-1, 6)[:, 0].sum() - Q.reshape(-1, 6)[:, 0].sum()) < 1e-13 * Q[..., 0].sum()


@pytest.mark.parametrize("case", ["periodic", "walls", "lid"])
def test_g_has_zero_conserved_moments_discrete(case):
    if case == "periodic":
        p, Q, G = W.smooth2d(seed=3, nx=8, ny=8, nv=14, eps=0.1)
    elif case == "walls":
        p, Q, G = W.quadrant2d(seed=3, nx=8, ny=8, nv=14)
    else:
        p, Q, G = W.cavity2d(seed=3, nx=8, ny=8, nv=14, eps=0.1, amp=0.2)
    Q1, G1, H = oracle.run(p, Q.reshape(-1), G.reshape(-1), 25)
    m, s = _mom_g(p, G1)
    assert np.abs(G1).max() > 1e-4
    assert np.all(np.abs(m) <= 1e-13 * s[:, None] + 1e-300)


def test_g_moments_paper_mode_within_quadrature_error():
    """PAPER projector: conserved moments of g vanish only to quadrature error (resolved grid)."""
    p, Q, G = W.smooth2d(seed=3, nx=8, ny=8, nv=40, V=10.0, eps=0.1, proj_mode="paper")
    Q1, G1, H = oracle.run(p, Q.reshape(-1), G.reshape(-1), 10)
    m, s = _mom_g(p, G1)
    assert np.all(np.abs(m) <= 1e-10 * s[:, None])


@pytest.mark.parametrize("bc", ["periodic", "walls"])
def test_equilibrium_is_steady(bc):
    nx, ny, nv = 6, 5, 12
    b = W.periodic2d() if bc == "periodic" else W.walls(T_wall=1.3)
    p = W.problem2d(nx, ny, nv, nv, 8.0, eps=0.02, bc=b)
    Q = W.conserved2d(np.full((ny, nx), 0.8), np.zeros((ny, nx)), np.zeros((ny, nx)), np.full((ny, nx), 1.3))
    G = W.zero_g(p)
    Q1, G1, H = oracle.run(p, Q.reshape(-1), G.reshape(-1), 30)
    np.testing.assert_allclose(Q1.reshape(Q.shape), Q, rtol=1e-13, atol=1e-14)
    # G picks up only the round-off of (Gauss - Maxwell)/eps
    assert np.abs(G1).max() < 1e-12 / 0.02


def test_asymptotic_preserving_limit():
    """eps -> 0: G^{n+1} -> G-hat^n (eqn5-98).  From G^n = 0 the transport
    sub-steps leave G** = 0, so G^{n+1} - G-hat = -eps/(eps + dt tau) G-hat,
    and the distance shrinks linearly with eps."""
    errs = []
    for eps in (1e-8, 1e-10):
        p, Q, G = W.smooth2d(seed=4, nx=8, ny=8, nv=14, eps=eps, nu=0.0)
        Qc = Q.reshape(-1, 6)
        rho = Qc[:, 0]
        u1, u2 = Qc[:, 1] / rho, Qc[:, 2] / rho
        pT = 0.5 * ((Qc[:, 3] - rho * u1 * u1) + (Qc[:, 5] - rho * u2 * u2))
        Qv = W.conserved2d(rho, u1, u2, pT / rho).reshape(-1)   # isotropic P
        G1, H = oracle.micro2d(p, Qv, np.zeros(G.size))
        Gh = oracle.ghat2d(p, Qv)
        dt = oracle.dt(p)[0]
        a = eps / (eps + dt * W.TAU_HS2D * rho)
        want = -(a[:, None] * Gh.reshape(len(rho), -1)).reshape(-1)
        np.testing.assert_allclose(G1 - Gh, want, rtol=1e-6, atol=1e-14 * np.abs(Gh).max())
        errs.append(np.abs(G1 - Gh).max())
    assert 90.0 < errs[0] / errs[1] < 110.0


def _mirror_x(p, Q, G):
    Qm = Q[:, ::-1, :].copy()
    Qm[..., 1] *= -1.0          # rho u1
    Qm[..., 4] *= -1.0          # E12
    Gm = G[:, ::-1, :, ::-1].copy()
    return Qm, Gm


def _mirror_y(p, Q, G):
    Qm = Q[::-1, :, :].copy()
    Qm[..., 2] *= -1.0
    Qm[..., 4] *= -1.0
    Gm = G[::-1, :, ::-1, :].copy()
    return Qm, Gm


@pytest.mark.parametrize("axis", ["x", "y"])
def test_mirror_symmetry_with_moving_lid(axis):
    p, Q, G = W.cavity2d(seed=5, nx=8, ny=6, nv=10, eps=0.05, amp=0.2)
    ny, nx, nv = 6, 8, 10
    Q = Q.copy()
    rng = np.random.default_rng(1)
    Q[..., 1] += 0.05 * rng.standard_normal((ny, nx))           # break every symmetry of the data
    Q[..., 4] += 0.02 * rng.standard_normal((ny, nx))
    Q1, G1, H1 = oracle.run(p, Q.reshape(-1), G.reshape(-1), 12)
    pm = dict(p)
    if axis == "x":
        pm["bc"] = W.walls(1.0, -0.2)                             # the lid moves the other way
        Qm, Gm = _mirror_x(p, Q, G)
        mir = _mirror_x
    else:
        b = W.walls(1.0, 0.2)
        pm["bc"] = [b[0], b[1], b[3], b[2]]                       # moving wall at the bottom
        Qm, Gm = _mirror_y(p, Q, G)
        mir = _mirror_y
    Q2, G2, H2 = oracle.run(pm, Qm.reshape(-1), Gm.reshape(-1), 12)
    Q1m, G1m = mir(p, Q1.reshape(ny, nx, 6), G1.reshape(ny, nx, nv, nv))
    np.testing.assert_allclose(Q2.reshape(ny, nx, 6), Q1m, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(G2.reshape(ny, nx, nv, nv), G1m, rtol=0, atol=1e-11 * np.abs(G1).max())


def test_conservation_and_mirror_1d():
    p, Q, G = W.sod1d(nx=60, nv=32, eps=0.05, bc="periodic")
    Q1, G1, H = oracle.run(p, Q, G, 80)
    s0, s1 = Q.sum(0), Q1.reshape(-1, 3).sum(0)
    assert np.all(np.abs(s1 - s0) <= 1e-13 * np.abs(Q).sum())
    # mirror x -> -x, v -> -v, rho u -> -rho u
    pe, Qe, Ge = W.sod1d(nx=60, nv=32, eps=0.05)
    Qa, Ga, _ = oracle.run(pe, Qe, Ge, 50)
    Qm = Qe[::-1].copy()
    Qm[:, 1] *= -1
    Qb, Gb, _ = oracle.run(pe, Qm, Ge[:, :, :, ::-1].copy(), 50)
    Qa = Qa.reshape(60, 3)[::-1].copy()
    Qa[:, 1] *= -1
    np.testing.assert_allclose(Qb.reshape(60, 3), Qa, rtol=1e-12, atol=1e-14)
