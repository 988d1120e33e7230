"""Pins of the oracle's wall-cell G-hat (Sec. 6.3, the lid-driven cavity boundary
conditions lid_driven_bc_1..4 and twodim_wall_densities_1/2).

In a cell next to a diffuse wall the oracle replaces the closed form (eqn5-97)
by -(1/tau)(I - Pi)[M_up], M_up an upwind difference of Maxwellians whose ghost
on the wall side is the wall Maxwellian.  Three facts the paper and the
mathematics fix, independently of how the oracle codes it:

1. Consistency.  Where the wall Maxwellian is the smooth field's own
   continuation to the ghost-cell centre (zero normal velocity, T = T_wall and
   the wall's tangential speed there, and a density profile for which the zero
   normal mass flux condition returns the continued density to first order),
   -tau G-hat converges at first order in dx to (I - Pi)(v . grad M), the closed
   form of (eq5-69) taken with the exact gradients.  A ghost on the wrong side,
   a wrong ghost state, the wall speed in the normal component or the wall
   density from the wrong half-range (R+ for R-) leave an O(1) error.
2. The jump.  For a uniform gas against a wall of another temperature and
   speed, only velocities leaving the wall into the gas see the wall: the
   difference is (v.n)^+ (M - M_wall) / dx there, zero on the other half, and
   the wall density is the one for which the normal mass fluxes balance (the
   condition stated with twodim_wall_densities).  (I - Pi) of that, computed
   here from adaptive quadrature of the exact functions with the continuous
   projector, equals -tau G-hat up to the midpoint rule's O(dv^2) error at the
   kink v.n = 0.  Swapped upwind sides, a mirrored ghost, R on the wrong side
   or the scalar T in place of the normal temperature P_nn / rho fail it.
3. The ES term of a wall cell is that of an interior cell with the same state.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import mm_workloads as W
import oracle


def _phi(v1, v2, u1, u2, T):
    """Basis of the collision null space orthogonal under M(u, T) (Sec. 5.3)."""
    w1, w2 = v1 - u1, v2 - u2
    return [np.ones_like(w1 * 1.0), w1 / math.sqrt(T), w2 / math.sqrt(T), (w1 * w1 + w2 * w2) / (2 * T) - 1.0]


def _maxw(rho, u1, u2, T, v1, v2):
    return rho / (2 * math.pi * T) * np.exp(-((v1 - u1) ** 2 + (v2 - u2) ** 2) / (2 * T))


def _q(rho, u1, u2, P11, P12, P22):
    return np.array([rho, rho * u1, rho * u2, rho * u1 * u1 + P11, rho * u1 * u2 + P12, rho * u2 * u2 + P22])


# ----------------------------------------------------------------------------
# 1. consistency with (eq5-69) for a field whose continuation is the wall state

TW = (0.9, 1.15)     # wall temperatures of the low and high side
UW = (0.15, -0.1)    # tangential wall speeds


def _field(x, y, g0, g1):
    """Smooth (rho, u_n, u_t, T), normal coordinate x, tangential y, whose values at the
    ghost-cell centres x = g0 (low side) and x = g1 (high side) are the wall states:
    u_n = 0, T = T_wall and u_t = u_wall there.  d(ln rho)/dx at g0 and g1 is chosen so
    that rho R^-+ of the wall cell, one cell width inside, is the continued density up to
    O(dx^2):  d(ln rho)/dx + T_x / (2 T_w) -+ (du_n/dx) sqrt(pi / (2 T_w)) = 0
    (first-order expansion of twodim_wall_densities_1 about the ghost centre)."""
    L = g1 - g0
    s = (x - g0) / L                              # 0 at the low ghost, 1 at the high one
    a = 0.3 * np.sin(2 * np.pi * y) + 0.2       # T curvature term
    b = 0.25 * np.cos(2 * np.pi * y)            # tangential-speed curvature term
    c = 0.4 + 0.3 * np.sin(2 * np.pi * y + 1.0)  # normal-speed profile
    T = TW[0] + (TW[1] - TW[0]) * s + s * (1 - s) * a
    ut = UW[0] + (UW[1] - UW[0]) * s + s * (1 - s) * b
    un = s * (1 - s) * c
    # x-slopes of T and u_n at the two ghost centres
    Tx0, Tx1 = ((TW[1] - TW[0]) + a) / L, ((TW[1] - TW[0]) - a) / L
    ux0, ux1 = c / L, -c / L
    d0 = -Tx0 / (2 * TW[0]) + ux0 * math.sqrt(math.pi / (2 * TW[0]))
    d1 = -Tx1 / (2 * TW[1]) - ux1 * math.sqrt(math.pi / (2 * TW[1]))
    lnrho = 0.1 * np.cos(2 * np.pi * y) + L * (d0 * s + 0.5 * (d1 - d0) * s * s)
    return np.exp(lnrho), un, ut, T


def _grad(f, x, y, h=1e-5):
    fx = (f(x + h, y) - f(x - h, y)) / (2 * h)
    fy = (f(x, y + h) - f(x, y - h)) / (2 * h)
    return fx, fy


def _consistency_error(n, transpose):
    """max over the wall-column cells of |-tau G-hat - closed form| / max|closed form|,
    on an n x n grid with walls on the x sides (transpose: on the y sides)."""
    nv, V = 20, 6.0
    if not transpose:
        bc = [{"kind": "wall", "T_wall": TW[0], "u_wall": UW[0]}, {"kind": "wall", "T_wall": TW[1], "u_wall": UW[1]},
              {"kind": "periodic"}, {"kind": "periodic"}]
    else:
        bc = [{"kind": "periodic"}, {"kind": "periodic"},
              {"kind": "wall", "T_wall": TW[0], "u_wall": UW[0]}, {"kind": "wall", "T_wall": TW[1], "u_wall": UW[1]}]
    p = W.problem2d(n, n, nv, nv, V, nu=0.0, bc=bc, wall_es_term=False, eps=0.1)
    xc = W.centres(0.0, 1.0, n)
    X, Y = np.meshgrid(xc, xc, indexing="xy")     # X varies along i, Y along j
    # normal coordinate s, tangential coordinate t of every cell
    S, Tt = (X, Y) if not transpose else (Y, X)
    g0, g1 = -0.5 / n, 1.0 + 0.5 / n               # ghost-cell centres
    rho, un, ut, T = _field(S, Tt, g0, g1)
    u1, u2 = (un, ut) if not transpose else (ut, un)
    Q = W.conserved2d(rho, u1, u2, T)
    Gh = oracle.ghat2d(p, Q.reshape(-1)).reshape(n, n, nv, nv)
    tau = W.TAU_HS2D * rho
    v = W.centres(-V, V, nv)
    V1, V2 = np.meshgrid(v, v, indexing="xy")      # [l][k]: v1 along k, v2 along l

    def comp(k):
        return lambda s, t: _field(s, t, g0, g1)[k]

    err, scale = 0.0, 0.0
    cells = [(j, 0) for j in range(n)] + [(j, n - 1) for j in range(n)]
    if transpose:
        cells = [(i, j) for (j, i) in cells]      # rows j = 0 and j = n-1
    for (j, i) in cells:
        s, t = (xc[i], xc[j]) if not transpose else (xc[j], xc[i])
        (un_s, un_t), (ut_s, ut_t), (T_s, T_t) = (_grad(comp(k), s, t) for k in (1, 2, 3))
        if not transpose:
            du1 = (un_s, un_t); du2 = (ut_s, ut_t); dT = (T_s, T_t)
        else:
            du1 = (ut_t, ut_s); du2 = (un_t, un_s); dT = (T_t, T_s)
        r, a1, a2, Tc = rho[j, i], u1[j, i], u2[j, i], T[j, i]
        w1, w2 = V1 - a1, V2 - a2
        s11 = du1[0] - du2[1]
        s12 = du1[1] + du2[0]
        closed = (((w1 ** 2 - w2 ** 2) / 2 * s11 + w1 * w2 * s12) / Tc
                  + ((w1 ** 2 + w2 ** 2) / (2 * Tc) - 2.0) * (w1 * dT[0] + w2 * dT[1]) / Tc) * _maxw(r, a1, a2, Tc, V1, V2)
        got = -tau[j, i] * Gh[j, i]
        err = max(err, np.abs(got - closed).max())
        scale = max(scale, np.abs(closed).max())
    return err / scale


@pytest.mark.parametrize("transpose", [False, True], ids=["x_walls", "y_walls"])
def test_wall_ghat_first_order_consistent(transpose):
    errs = [_consistency_error(n, transpose) for n in (16, 32, 64)]
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    # first order: the error halves with dx (measured 0.29, 0.15, 0.075)
    assert errs[-1] < 0.1, errs
    assert all(0.9 < r < 1.1 for r in rates), (errs, rates)


# ----------------------------------------------------------------------------
# 2. the jump: uniform gas against a wall of another temperature and speed

def _half_flux_out(mu, theta):
    """int_{s<0} s N(s; mu, theta) ds (normal velocity toward the wall; negative)."""
    sd = math.sqrt(theta)
    z = mu / sd
    pdf = math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)
    cdf_neg = 0.5 * math.erfc(z / math.sqrt(2))
    return mu * cdf_neg - sd * pdf


SIDES = {0: ((1.0, 0.0), 0), 1: ((-1.0, 0.0), 0), 2: ((0.0, 1.0), 1), 3: ((0.0, -1.0), 1)}   # inward normal, axis


def _wall_maxwellian(side, cell, T_wall, u_wall):
    """(rho, u1, u2, T) of the wall Maxwellian: tangential speed u_wall, zero normal
    speed, density from the balance of the normal mass fluxes (the gas's Gaussian with
    the normal temperature P_nn / rho against the wall's half-Maxwellian)."""
    rho, u1, u2, P = cell
    n, ax = SIDES[side]
    mu = u1 * n[0] + u2 * n[1]                          # normal speed along the inward normal
    theta = P[ax][ax] / rho
    out = -rho * _half_flux_out(mu, theta)              # mass flux of the gas into the wall
    rho_w = out / math.sqrt(T_wall / (2 * math.pi))     # wall flux per unit density
    uw = (0.0, u_wall) if ax == 0 else (u_wall, 0.0)
    return rho_w, uw[0], uw[1], T_wall


def _expected_jump(sides, cell, walls_, dx, V, nv):
    """(I - Pi_cont)[sum over wall sides of (v.n)^+ (M - M_wall)/dx] at the nodes, with
    the continuous moments of the exact functions from adaptive quadrature."""
    rho, u1, u2, P = cell
    T = 0.5 * (P[0][0] + P[1][1]) / rho

    def F(v1, v2):
        tot = 0.0 * v1
        for s in sides:
            (n1, n2), _ = SIDES[s]
            vn = np.maximum(0.0, v1 * n1 + v2 * n2)
            rw, a1, a2, Tw = _wall_maxwellian(s, cell, *walls_[s])
            tot = tot + vn * (_maxw(rho, u1, u2, T, v1, v2) - _maxw(rw, a1, a2, Tw, v1, v2)) / dx
        return tot

    coef = []
    for a in range(4):
        def integrand(v2, v1, a=a):
            return _phi(v1, v2, u1, u2, T)[a] * F(v1, v2)

        def norm(v2, v1, a=a):
            return _phi(v1, v2, u1, u2, T)[a] ** 2 * _maxw(rho, u1, u2, T, v1, v2)
        num = 0.0
        # split at v1 = 0 and v2 = 0, where F has kinks
        for (l1, h1) in ((-V, 0.0), (0.0, V)):
            for (l2, h2) in ((-V, 0.0), (0.0, V)):
                num += integrate.dblquad(integrand, l1, h1, l2, h2, epsabs=1e-13, epsrel=1e-12)[0]
        den = integrate.dblquad(norm, -V, V, -V, V, epsabs=1e-13, epsrel=1e-12)[0]
        coef.append(num / den)
    v = W.centres(-V, V, nv)
    V1, V2 = np.meshgrid(v, v, indexing="xy")
    ph = _phi(V1, V2, u1, u2, T)
    proj = sum(coef[a] * ph[a] for a in range(4)) * _maxw(rho, u1, u2, T, V1, V2)
    return F(V1, V2) - proj


def _jump_case(sides, nv, V=6.0):
    rho, u1, u2 = 1.2, 0.25, -0.2
    P = [[1.1, 0.12], [0.12, 0.85]]                     # anisotropic: P11/rho != P22/rho != T
    walls_ = {0: (1.5, 0.3), 1: (0.7, -0.25), 2: (1.3, -0.2), 3: (0.8, 0.35)}
    bc = []
    for s in range(4):
        if s in sides or (s ^ 1) in sides:
            Tw, uw = walls_[s]
            bc.append({"kind": "wall", "T_wall": Tw, "u_wall": uw})
        else:
            bc.append({"kind": "periodic"})
    nx, ny = 5, 4
    p = W.problem2d(nx, ny, nv, nv, V, nu=0.0, bc=bc, wall_es_term=False, eps=0.1)
    q = _q(rho, u1, u2, P[0][0], P[0][1], P[1][1])
    Q = np.tile(q, (ny, nx, 1))
    Gh = oracle.ghat2d(p, Q.reshape(-1)).reshape(ny, nx, nv, nv)
    i = {0: 0, 1: nx - 1}.get(next((s for s in sides if s < 2), None), 2)
    j = {2: 0, 3: ny - 1}.get(next((s for s in sides if s >= 2), None), 1)
    tau = W.TAU_HS2D * rho
    got = -tau * Gh[j, i]
    dx = {0: 1.0 / nx, 1: 1.0 / nx, 2: 1.0 / ny, 3: 1.0 / ny}
    # the upwind differences divide by the spacing normal to each wall
    exp = sum(_expected_jump([s], (rho, u1, u2, P), walls_, dx[s], V, nv) for s in sides)
    return np.abs(got - exp).max() / np.abs(exp).max()


@pytest.mark.slow
@pytest.mark.parametrize("sides", [[0], [1], [2], [3], [0, 3], [1, 2]],
                         ids=["x_lo", "x_hi", "y_lo", "y_hi", "corner_x_lo_y_hi", "corner_x_hi_y_lo"])
def test_wall_ghat_jump_against_half_range_integrals(sides):
    e48 = _jump_case(sides, 48)
    e96 = _jump_case(sides, 96)
    # midpoint rule across the kink of (v.n)^+: second order in dv
    assert e96 < 2e-3, (e48, e96)
    assert 3.0 < e48 / e96 < 5.0, (e48, e96)


# ----------------------------------------------------------------------------
# 3. the ES term of a wall cell

def test_wall_ghat_es_term_equals_interior():
    nv, V = 24, 6.0
    nx, ny = 5, 5
    rho, u1, u2 = 0.9, 0.1, -0.15
    q = _q(rho, u1, u2, 1.0, 0.2, 0.7)
    Q = np.tile(q, (ny, nx, 1)).reshape(-1)
    base = dict(nu=-0.5, eps=0.03)
    pw_on = W.problem2d(nx, ny, nv, nv, V, bc=W.walls(T_wall=1.3, lid=0.2), wall_es_term=True, **base)
    pw_off = dict(pw_on, wall_es_term=False)
    on = oracle.ghat2d(pw_on, Q).reshape(ny, nx, -1)
    off = oracle.ghat2d(pw_off, Q).reshape(ny, nx, -1)
    interior = on[2, 2]                                 # uniform state: the ES term alone
    assert np.abs(interior).max() > 0.1                 # the term is not trivially zero
    for (j, i) in [(0, 0), (0, 2), (2, 0), (4, 4), (4, 1)]:
        d = on[j, i] - off[j, i]
        assert np.abs(d - interior).max() <= 1e-12 * np.abs(interior).max() + 1e-12 * np.abs(off[j, i]).max()
