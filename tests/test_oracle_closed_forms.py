"""Pins of the oracle's building blocks against closed forms, brute-force
quadrature and textbook constructions (no GPU)."""
import json
import math
import os

import numpy as np
import pytest

import mm_workloads as W
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _q2d(rho, u1, u2, P11, P12, P22):
    return np.array([rho, rho * u1, rho * u2, rho * u1 * u1 + P11, rho * u1 * u2 + P12, rho * u2 * u2 + P22])


STATES = [
    (1.0, 0.0, 0.0, 1.0, 0.0, 1.0),
    (0.7, 0.31, -0.22, 0.9, 0.13, 0.55),
    (1.9, -0.8, 0.45, 2.4, -0.35, 1.3),
    (0.3, 1.4, 0.05, 0.2, 0.02, 0.35),
]


def _gauss_nodes(lo, hi, n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (hi - lo) * x + 0.5 * (hi + lo), 0.5 * (hi - lo) * w


def _gaussian_pdf(V1, V2, rho, u, S):
    det = S[0, 0] * S[1, 1] - S[0, 1] ** 2
    w1, w2 = V1 - u[0], V2 - u[1]
    quad = (S[1, 1] * w1 * w1 - 2 * S[0, 1] * w1 * w2 + S[0, 0] * w2 * w2) / det
    return rho / (2 * math.pi * math.sqrt(det)) * np.exp(-0.5 * quad)


# ---------------------------------------------------------------------------
# Gaussian moments (Sec. 2.3): <m M> = (rho, rho u, rho u u + rho T I),
# <m G> = (rho, rho u, rho u u + rho calT), calT = (1-nu) T I + nu TT


@pytest.mark.parametrize("st", STATES)
@pytest.mark.parametrize("nu", [-1.0, -0.5, 0.0, 0.6])
def test_gaussian_moments(st, nu):
    rho, u1, u2, P11, P12, P22 = st
    p = W.problem2d(2, 2, 96, 96, 14.0, nu=nu)       # dv = 0.29: quadrature exact to ~1e-15
    M, G = oracle.gaussians2d(p, _q2d(*st))
    v = W.centres(-14.0, 14.0, 96)
    V1, V2 = np.meshgrid(v, v)                        # [l][k] layout: V1 varies along k
    dA = (28.0 / 96) ** 2
    T = 0.5 * (P11 + P22) / rho
    TT = np.array([[P11, P12], [P12, P22]]) / rho
    calT = (1 - nu) * T * np.eye(2) + nu * TT
    for F, S in ((M, T * np.eye(2)), (G, calT)):
        F = F.reshape(96, 96)
        mom = [np.sum(F), np.sum(V1 * F), np.sum(V2 * F), np.sum(V1 * V1 * F), np.sum(V1 * V2 * F), np.sum(V2 * V2 * F)]
        mom = np.array(mom) * dA
        want = [rho, rho * u1, rho * u2, rho * (u1 * u1 + S[0, 0]), rho * (u1 * u2 + S[0, 1]), rho * (u2 * u2 + S[1, 1])]
        np.testing.assert_allclose(mom, want, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# KFVS half-space fluxes (flux-2D-1/2) against brute-force quadrature of
# int_{s v_d > 0} v_d m(v) N(v; u, P/rho) dv, m = (1, v1, v2, v1^2, v1 v2, v2^2)


@pytest.mark.parametrize("st", STATES)
@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("sign", [+1, -1])
def test_kfvs_half2d_quadrature(st, direction, sign):
    rho, u1, u2, P11, P12, P22 = st
    S = np.array([[P11, P12], [P12, P22]]) / rho
    u = np.array([u1, u2])
    L = 14.0 * math.sqrt(max(S[0, 0], S[1, 1])) + 3.0
    a, wa = _gauss_nodes(0.0, L, 160)                 # half line of the normal velocity
    b, wb = _gauss_nodes(-L, L, 240)                  # tangential velocity
    vn = sign * a
    if direction == 0:
        V1, V2 = np.meshgrid(vn, b, indexing="ij")
    else:
        V2, V1 = np.meshgrid(vn, b, indexing="ij")
    Wt = np.outer(wa, wb)
    f = _gaussian_pdf(V1, V2, rho, u, S)
    vd = V1 if direction == 0 else V2
    m = [np.ones_like(V1), V1, V2, V1 * V1, V1 * V2, V2 * V2]
    want = np.array([np.sum(Wt * vd * mm * f) for mm in m])
    got = oracle.kfvs_half2d(_q2d(*st), direction, sign)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("st", STATES)
@pytest.mark.parametrize("direction", [0, 1])
def test_kfvs_split_sums_to_full_flux(st, direction):
    """F+ + F- equals the full 10-moment flux of (eq5-41) without H."""
    rho, u1, u2, P11, P12, P22 = st
    q = _q2d(*st)
    s = oracle.kfvs_half2d(q, direction, +1) + oracle.kfvs_half2d(q, direction, -1)
    if direction == 0:
        f = [rho * u1, rho * u1 ** 2 + P11, rho * u1 * u2 + P12, rho * u1 ** 3 + 3 * u1 * P11,
             rho * u1 ** 2 * u2 + u2 * P11 + 2 * u1 * P12, rho * u1 * u2 ** 2 + 2 * u2 * P12 + u1 * P22]
    else:
        f = [rho * u2, rho * u1 * u2 + P12, rho * u2 ** 2 + P22, rho * u1 ** 2 * u2 + u2 * P11 + 2 * u1 * P12,
             rho * u1 * u2 ** 2 + 2 * u2 * P12 + u1 * P22, rho * u2 ** 3 + 3 * u2 * P22]
    np.testing.assert_allclose(s, f, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("rho,u,T", [(1.0, 0.0, 1.0), (0.125, 0.3, 0.8), (2.0, -1.1, 0.4)])
@pytest.mark.parametrize("sign", [+1, -1])
def test_kfvs_half1d_quadrature(rho, u, T, sign):
    L = 14.0 * math.sqrt(T) + 3.0
    a, wa = _gauss_nodes(0.0, L, 200)
    v = sign * a
    f = rho / math.sqrt(2 * math.pi * T) * np.exp(-(v - u) ** 2 / (2 * T))
    want = np.array([np.sum(wa * v * f), np.sum(wa * v * v * f), np.sum(wa * v * 0.5 * v * v * f)])
    q = np.array([rho, rho * u, 0.5 * rho * T + 0.5 * rho * u * u])
    np.testing.assert_allclose(oracle.kfvs_half1d(q, sign), want, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------
# Projector (eq5-33, eq5-38)


def _span_residual(F, M, V1, V2):
    """Least-squares distance of F from span{1, v1, v2, |v|^2} M (relative)."""
    B = np.stack([M, V1 * M, V2 * M, (V1 ** 2 + V2 ** 2) * M], axis=1)
    c, *_ = np.linalg.lstsq(B, F, rcond=None)
    return np.linalg.norm(B @ c - F) / max(np.linalg.norm(F), 1e-300)


@pytest.mark.parametrize("st", STATES[1:])
def test_discrete_projector_is_orthogonal_projection(st):
    p = W.problem2d(2, 2, 20, 20, 7.0)
    q = _q2d(*st)
    rng = np.random.default_rng(3)
    F = rng.standard_normal(400)
    M, G = oracle.gaussians2d(p, q)
    v = W.centres(-7.0, 7.0, 20)
    V1, V2 = (a.ravel() for a in np.meshgrid(v, v))
    PF = oracle.project2d(p, q, F)
    # idempotent
    np.testing.assert_allclose(oracle.project2d(p, q, PF), PF, rtol=0, atol=1e-13 * np.abs(PF).max())
    # range is span{1, v, |v|^2} M
    assert _span_residual(PF, M, V1, V2) < 1e-12
    # the complement has zero conserved moments (eq5-38: Pi g = 0 for g with zero moments)
    R = F - PF
    for mom in (np.ones_like(V1), V1, V2, V1 ** 2 + V2 ** 2):
        assert abs(np.sum(mom * R)) < 1e-12 * np.sum(np.abs(mom * F))
    # Pi M = M
    np.testing.assert_allclose(oracle.project2d(p, q, M), M, rtol=0, atol=1e-14 * M.max())


@pytest.mark.parametrize("st", STATES[1:])
def test_projector_of_es_gaussian_is_maxwellian(st):
    """Pi_M G = M (eq5-38) up to the quadrature error of a resolved grid, in both modes."""
    for mode in ("discrete", "paper"):
        p = W.problem2d(2, 2, 96, 96, 14.0, nu=-1.0, proj_mode=mode)
        q = _q2d(*st)
        M, G = oracle.gaussians2d(p, q)
        PG = oracle.project2d(p, q, G)
        np.testing.assert_allclose(PG, M, rtol=0, atol=1e-12 * M.max())


def test_paper_projector_matches_discrete_on_resolved_grid():
    st = STATES[2]
    q = _q2d(*st)
    rng = np.random.default_rng(5)
    F = rng.standard_normal(96 * 96)
    pd = W.problem2d(2, 2, 96, 96, 14.0)
    pp = W.problem2d(2, 2, 96, 96, 14.0, proj_mode="paper")
    a, b = oracle.project2d(pd, q, F), oracle.project2d(pp, q, F)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())


def test_paper_projector_coefficients():
    """PAPER mode: A_a = (dv1 dv2 / rho) sum phi_a F, Pi F = sum A_a phi_a M (coeffs-2D-xdir)."""
    p = W.problem2d(2, 2, 12, 10, 5.0, V2=4.0, proj_mode="paper")
    st = STATES[1]
    q = _q2d(*st)
    rho, u1, u2, P11, P12, P22 = st
    T = 0.5 * (P11 + P22) / rho
    rng = np.random.default_rng(9)
    F = rng.standard_normal(120)
    v1 = W.centres(-5, 5, 12)
    v2 = W.centres(-4, 4, 10)
    V1, V2 = (a.ravel() for a in np.meshgrid(v1, v2))
    w1, w2 = V1 - u1, V2 - u2
    phi = [np.ones_like(w1), w1 / math.sqrt(T), w2 / math.sqrt(T), (w1 ** 2 + w2 ** 2) / (2 * T) - 1]
    M = rho / (2 * math.pi * T) * np.exp(-(w1 ** 2 + w2 ** 2) / (2 * T))
    A = [(10 / 12) * (8 / 10) / rho * np.sum(ph * F) for ph in phi]
    want = sum(a * ph for a, ph in zip(A, phi)) * M
    np.testing.assert_allclose(oracle.project2d(p, q, F), want, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------
# Closed form (eq5-69) inside G-hat (eqn5-97): for fields linear in x and y the
# central differences are exact, so tau * G-hat must equal -(I - Pi)[v.grad M]
# with the analytic gradient, to round-off (discrete projector).


def _linear_fields(nx, ny):
    x = W.centres(0, 1, nx)
    y = W.centres(0, 1, ny)
    X, Y = np.meshgrid(x, y)
    rho = 1.0 + 0.3 * X - 0.2 * Y
    u1 = 0.2 - 0.4 * X + 0.3 * Y
    u2 = -0.1 + 0.25 * X + 0.35 * Y
    T = 0.9 + 0.35 * X + 0.15 * Y
    grads = dict(rho=(0.3, -0.2), u1=(-0.4, 0.3), u2=(0.25, 0.35), T=(0.35, 0.15))
    return X, Y, rho, u1, u2, T, grads


@pytest.mark.parametrize("nu", [-0.5, -1.0])
def test_ghat_closed_form_equals_projected_transport(nu):
    nx = ny = 6
    nv = 24
    p = W.problem2d(nx, ny, nv, nv, 8.0, nu=nu, bc=W.extrap2d(), eps=0.37)
    X, Y, rho, u1, u2, T, gr = _linear_fields(nx, ny)
    Q = W.conserved2d(rho, u1, u2, T)                 # isotropic P: the ES term vanishes
    Gh = oracle.ghat2d(p, Q.reshape(-1)).reshape(ny, nx, nv * nv)
    v = W.centres(-8, 8, nv)
    V1, V2 = (a.ravel() for a in np.meshgrid(v, v))
    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            r, a1, a2, t = rho[j, i], u1[j, i], u2[j, i], T[j, i]
            w1, w2 = V1 - a1, V2 - a2
            M = r / (2 * math.pi * t) * np.exp(-(w1 ** 2 + w2 ** 2) / (2 * t))
            vgM = np.zeros_like(M)
            for d, vd in enumerate((V1, V2)):
                dlog = (gr["rho"][d] / r - gr["T"][d] / t + (w1 * gr["u1"][d] + w2 * gr["u2"][d]) / t
                        + (w1 ** 2 + w2 ** 2) * gr["T"][d] / (2 * t * t))
                vgM += vd * dlog * M
            q = Q[j, i]
            want = -(vgM - oracle.project2d(p, q, vgM)) / (W.TAU_HS2D * r)
            np.testing.assert_allclose(Gh[j, i], want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_ghat_es_term():
    """With zero gradients G-hat reduces to (I - Pi)(G - M)/eps (the ES term of eqn5-75)."""
    nx = ny = 4
    nv = 20
    eps = 0.05
    p = W.problem2d(nx, ny, nv, nv, 7.0, nu=-0.5, bc=W.periodic2d(), eps=eps)
    st = STATES[1]
    Q = np.tile(_q2d(*st), (ny, nx, 1))
    Gh = oracle.ghat2d(p, Q.reshape(-1)).reshape(ny * nx, -1)
    M, G = oracle.gaussians2d(p, Q[0, 0])
    D = (G - M) / eps
    want = D - oracle.project2d(p, Q[0, 0], D)
    for c in range(nx * ny):
        np.testing.assert_allclose(Gh[c], want, rtol=0, atol=1e-13 * np.abs(want).max())


# ---------------------------------------------------------------------------
# TR-BDF2 collision factor (macro2d-split1/4)


def _trbdf2_numeric(lam, h):
    """TR-BDF2 with gamma = 1/2 applied stage by stage to y' = lam y, y0 = 1, step h."""
    g = 0.5
    y0 = 1.0
    yg = y0 * (1 + 0.5 * g * h * lam) / (1 - 0.5 * g * h * lam)              # trapezoid to t + g h
    c0 = (1 - g) ** 2 / (g * (2 - g))
    cg = 1.0 / (g * (2 - g))
    ch = (1 - g) / (2 - g)
    return (cg * yg - c0 * y0) / (1 - ch * h * lam)                             # BDF2 to t + h


@pytest.mark.parametrize("eps", [1e-4, 1e-2, 0.3, 5.0])
@pytest.mark.parametrize("tau,nu,dt", [(1.45, -0.5, 1e-3), (0.2, -1.0, 3e-2), (3.0, 0.5, 2e-4)])
def test_trbdf2_factor(eps, tau, nu, dt):
    lam = -tau * (1 - nu) / eps          # decay rate of the deviatoric pressure (eq5-40)
    want = _trbdf2_numeric(lam, 0.5 * dt)
    got = oracle.trbdf2_W(eps, tau, nu, dt)
    assert abs(got - want) <= 1e-14 * max(1.0, abs(want))
    assert abs(got) <= 1.0


def test_trbdf2_limits():
    # L-stable: W -> 0 as eps -> 0; consistent: W ~ exp(z) for small z (third order)
    # R(z) = (12 + 5z)/(12 - 7z + z^2) ~ 5/z as z -> -infinity: |W| ~ 10 eps / (tau (1 - nu) dt)
    for eps in (1e-8, 1e-10, 1e-12):
        w = oracle.trbdf2_W(eps, 1.0, -0.5, 1e-3)
        assert abs(w + 10 * eps / 1.5e-3) < 1e-3 * abs(w)
    for z in (1e-2, 2e-2, 4e-2):
        eps = 1.0
        tau = 1.0
        dt = 2 * z / 1.5
        e = abs(oracle.trbdf2_W(eps, tau, -0.5, dt) - math.exp(-z))
        assert e < 0.05 * z ** 3          # local error constant of this TR-BDF2 is 1/24


def test_collision_step_in_macro_preserves_trace():
    p = W.problem2d(3, 3, 4, 4, 5.0, bc=W.periodic2d(), eps=0.05, dt=1e-3)
    st = STATES[2]
    Q = np.tile(_q2d(*st), (3, 3, 1)).reshape(-1)
    H = np.zeros(9 * 4)
    Q1 = oracle.macro2d(p, Q, H).reshape(9, 6)     # uniform state: fluxes cancel, only collisions act
    rho, u1, u2, P11, P12, P22 = st
    W_ = oracle.trbdf2_W(0.05, W.TAU_HS2D * rho, -0.5, 1e-3)
    pp = 0.5 * (P11 + P22)
    dev = np.array([P11 - pp, P12, P22 - pp]) * W_ * W_
    want = _q2d(rho, u1, u2, pp + dev[0], dev[1], pp + dev[2])
    for c in range(9):
        np.testing.assert_allclose(Q1[c], want, rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------------------
# Wall densities (twodim_wall_densities_1/2): zero net normal mass flux


@pytest.mark.parametrize("st", STATES)
@pytest.mark.parametrize("T_wall", [1.0, 0.7])
@pytest.mark.parametrize("side", ["left", "right", "bottom", "top"])
def test_wall_density_zero_mass_flux(st, T_wall, side):
    rho, u1, u2, P11, P12, P22 = st
    S = np.array([[P11, P12], [P12, P22]]) / rho
    d = 0 if side in ("left", "right") else 1
    inward = +1 if side in ("left", "bottom") else -1
    R = oracle.wall_R([u1, u2][d], S[d, d], T_wall, -1 if inward > 0 else +1)
    rho_w = rho * R
    L = 14.0 * math.sqrt(max(S[0, 0], S[1, 1], T_wall)) + 3.0
    a, wa = _gauss_nodes(0.0, L, 160)
    b, wb = _gauss_nodes(-L, L, 200)
    Wt = np.outer(wa, wb)
    lid = np.array([0.3, 0.0]) if d == 1 else np.array([0.0, -0.2])   # tangential wall motion
    flux = 0.0
    for s, dens, u, Sg in ((inward, rho_w, lid, T_wall * np.eye(2)), (-inward, rho, np.array([u1, u2]), S)):
        A, B = np.meshgrid(s * a, b, indexing="ij")      # normal along axis 0, tangential along 1
        V1, V2 = (A, B) if d == 0 else (B, A)
        vd = A
        flux += np.sum(Wt * vd * _gaussian_pdf(V1, V2, dens, u, Sg))
    assert abs(flux) < 1e-12 * rho


# ---------------------------------------------------------------------------
# Time-step rules against the numbers printed in Sec. 4.2 and Sec. 6.2


def test_dt_rule_printed_examples():
    g = json.load(open(os.path.join(GOLD, "dt_paper.json")))
    s = g["sod1d"]
    p = W.problem1d(s["nx"], 128, s["V"], cfl=s["cfl_in"], x=tuple(s["x"]))
    dt, n = oracle.dt(p, s["t_final"])
    assert n == s["nsteps"]
    assert round(dt, 3 + s["dt_digits"]) == pytest.approx(s["dt"], rel=0, abs=0.5 * 10 ** -(3 + s["dt_digits"]))
    assert abs(s["V"] * dt / ((s["x"][1] - s["x"][0]) / s["nx"]) - s["cfl_out"]) < 5e-4
    c = g["cylsod2d"]
    for rule, key in (("sum", "nsteps_sum_rule"), ("min", "nsteps_min_rule")):
        p = W.problem2d(c["nx"], c["nx"], 14, 14, c["V"], cfl=c["cfl_in"], cfl_rule=rule, x=tuple(c["x"]), y=tuple(c["x"]))
        dt, n = oracle.dt(p, c["t_final"])
        assert n == c[key]
        if rule == "sum":
            assert abs(dt - c["dt"]) < 0.5e-8
            h = (c["x"][1] - c["x"][0]) / c["nx"]
            assert abs(dt * 2 * c["V"] / h - c["cfl_out"]) < 5e-6


def test_dt_rule_workloads():
    assert oracle.dt(W.sod1d()[0])[0] == pytest.approx(3.125e-4, rel=1e-15)
    assert oracle.dt(W.quadrant2d()[0])[0] == pytest.approx(9.765625e-4, rel=1e-15)
    assert oracle.dt(W.cavity2d(nx=256)[0])[0] == pytest.approx(0.5 / 256 / 7, rel=1e-15)
