"""Reference for the cylindrical Sod problem: the radially symmetric compressible
Euler equations of a gamma-law gas (Sec. 6.2, eqn:cyl-euler-1d, with the energy
E = p / (gamma - 1) + rho u_r^2 / 2; gamma = 2 for the 2D2V gas),

    d/dt [rho, rho u, E] + d/dr [rho u, rho u^2 + p, u (E + p)] = -(1/r) [rho u, rho u^2, u (E + p)],

solved on r in [0, R] by a second-order finite-volume method written for this
check (the paper's own reference is a discontinuous-Galerkin code that is not
available):
  - the equations in area-weighted form, d/dt (V_i U_i) = -(r F)_{i+1/2} + (r F)_{i-1/2}
    + (0, p_i (r_{i+1/2} - r_{i-1/2}), 0), V_i = (r_{i+1/2}^2 - r_{i-1/2}^2) / 2, which
    conserves mass exactly and keeps a gas at rest at rest;
  - MUSCL reconstruction of the primitive variables with the minmod limiter, the
    HLLC flux (Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics, 10.4)
    and Heun's (SSP RK2) time stepping;
  - reflection at r = 0 and constant extrapolation at r = R.
planar=True drops the geometry (unit areas and volumes, no pressure source): the
plain 1D Euler equations, for checking against the exact Riemann solver.
"""
import numpy as np


def _prim(U, gamma):
    rho = U[0]
    u = U[1] / rho
    p = (gamma - 1.0) * (U[2] - 0.5 * rho * u * u)
    return rho, u, p


def _cons(rho, u, p, gamma):
    return np.array([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def _minmod(a, b):
    return np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def _hllc(rl, ul, pl, rr, ur, pr, gamma):
    cl, cr = np.sqrt(gamma * pl / rl), np.sqrt(gamma * pr / rr)
    sl = np.minimum(ul - cl, ur - cr)
    sr = np.maximum(ul + cl, ur + cr)
    el = pl / (gamma - 1.0) + 0.5 * rl * ul * ul
    er = pr / (gamma - 1.0) + 0.5 * rr * ur * ur
    sm = (pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur)) / (rl * (sl - ul) - rr * (sr - ur))
    fl = np.array([rl * ul, rl * ul * ul + pl, ul * (el + pl)])
    fr = np.array([rr * ur, rr * ur * ur + pr, ur * (er + pr)])

    def star(r, u, p, e, s):
        f = r * (s - u) / (s - sm)
        return np.array([f, f * sm, f * (e / r + (sm - u) * (sm + p / (r * (s - u))))])

    ul_ = np.array([rl, rl * ul, el])
    ur_ = np.array([rr, rr * ur, er])
    fsl = fl + sl * (star(rl, ul, pl, el, sl) - ul_)
    fsr = fr + sr * (star(rr, ur, pr, er, sr) - ur_)
    return np.where(sl >= 0.0, fl, np.where(sm >= 0.0, fsl, np.where(sr > 0.0, fsr, fr)))


def solve(n, t_final, left, right, r0=0.5, R=1.0, gamma=2.0, cfl=0.4, planar=False, x_lo=0.0):
    """Cell centres and (rho, u, p) at t_final.  left / right: (rho, u, p) for r < r0 / r > r0.
    planar=True: the 1D Euler equations on [x_lo, x_lo + R] with extrapolation at both ends."""
    h = R / n
    rf = x_lo + h * np.arange(n + 1)                 # faces
    rc = 0.5 * (rf[:-1] + rf[1:])
    if planar:
        area = np.ones(n + 1)
        vol = np.full(n, h)
    else:
        area = rf
        vol = 0.5 * (rf[1:] ** 2 - rf[:-1] ** 2)
    rho = np.where(rc < r0, left[0], right[0])
    u = np.where(rc < r0, left[1], right[1])
    p = np.where(rc < r0, left[2], right[2])
    U = _cons(rho, u, p, gamma)
    dA = area[1:] - area[:-1]

    def rhs(U):
        rho, u, p = _prim(U, gamma)
        # two ghost cells per side: reflection (or extrapolation when planar) at the left,
        # extrapolation at the right
        if planar:
            gl = [(rho[1], u[1], p[1]), (rho[0], u[0], p[0])]
        else:
            gl = [(rho[1], -u[1], p[1]), (rho[0], -u[0], p[0])]
        W = [np.concatenate([[gl[0][k], gl[1][k]], q, [q[-1], q[-1]]]) for k, q in enumerate((rho, u, p))]
        # limited slopes and face values (MUSCL, primitive variables)
        out = []
        for w in W:
            d = _minmod(w[1:-1] - w[:-2], w[2:] - w[1:-1])      # slopes of cells -1 .. n
            wl = w[1:-2] + 0.5 * d[:-1]                          # left state of faces 0 .. n
            wr = w[2:-1] - 0.5 * d[1:]                           # right state
            out.append((wl, wr))
        F = _hllc(out[0][0], out[1][0], out[2][0], out[0][1], out[1][1], out[2][1], gamma)
        AF = F * area
        dU = -(AF[:, 1:] - AF[:, :-1])
        if not planar:
            dU[1] += p * dA
        return dU / vol

    t = 0.0
    while t < t_final * (1.0 - 1e-14):
        rho, u, p = _prim(U, gamma)
        smax = np.max(np.abs(u) + np.sqrt(gamma * p / rho))
        dt = min(cfl * h / smax, t_final - t)
        U1 = U + dt * rhs(U)
        U = 0.5 * (U + U1 + dt * rhs(U1))
        t += dt
    rho, u, p = _prim(U, gamma)
    return rc, rho, u, p, vol
