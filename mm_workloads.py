"""Seeded synthetic workloads shared by the oracle and the GPU path.

This module holds problem descriptions (plain dictionaries) and initial
states.  It contains none of the scheme's arithmetic: initial data are point
values at cell centres with g = 0 and an isotropic pressure tensor P = rho T I,
written as the conserved vector Q = (rho, rho u1, rho u2, E11, E12, E22) with
E = rho u (x) u + P (2D) or Q = (rho, rho u, rho T/2 + rho u^2/2) (1D).

The workloads are shaped after the paper's examples: the Sod tube of
Sec. 4.2, a quadrant Riemann problem in a walled box, and the lid-driven
cavity of Sec. 6.3 (walls, moving top lid).  The collision parameter of the 2D
cases is the hard-sphere value tau = (3 C25 pi / (2 sqrt 2)) rho, C25 = 0.436,
of (eqn:tau-for-2d-es-bgk); the 1D case uses tau = (16/5) sqrt(T / (2 pi)) of
(eqn:collision_parameter_1d).
"""
import math

import numpy as np

TAU_HS2D = 3.0 * 0.436 * math.pi / (2.0 * math.sqrt(2.0))
TAU_HS1D = 16.0 / 5.0


def _bc(kind, **kw):
    d = {"kind": kind}
    d.update(kw)
    return d


def walls(T_wall=1.0, lid=0.0):
    """Four diffuse walls at T_wall; the top wall moves with speed `lid`."""
    return [_bc("wall", T_wall=T_wall), _bc("wall", T_wall=T_wall),
            _bc("wall", T_wall=T_wall), _bc("wall", T_wall=T_wall, u_wall=lid)]


def periodic2d():
    return [_bc("periodic")] * 4


def extrap2d():
    return [_bc("extrap")] * 4


def problem2d(nx, ny, nv1, nv2, V1, V2=None, eps=0.1, cfl=0.5, nu=-0.5, bc=None,
              x=(0.0, 1.0), y=(0.0, 1.0), tau_model="rho", tau_coef=TAU_HS2D, **kw):
    V2 = V1 if V2 is None else V2
    p = {"dim": 2, "nx": nx, "ny": ny, "nv1": nv1, "nv2": nv2, "x": tuple(x), "y": tuple(y),
         "v1": (-V1, V1), "v2": (-V2, V2), "eps": eps, "cfl": cfl, "cfl_rule": "min", "nu": nu,
         "tau_model": tau_model, "tau_coef": tau_coef, "bc": bc if bc is not None else walls(),
         "proj_mode": "discrete", "wall_es_term": True, "dt": 0.0, "precision": "fp64"}
    p.update(kw)
    return p


def problem1d(nx, nv, V, eps=1e-2, cfl=0.5, bc="extrap", x=(0.0, 1.0), tau_model="hs1d",
              tau_coef=TAU_HS1D, **kw):
    p = {"dim": 1, "nx": nx, "ny": 1, "nv1": nv, "nv2": 1, "x": tuple(x), "y": (0.0, 1.0),
         "v1": (-V, V), "v2": (0.0, 1.0), "eps": eps, "cfl": cfl, "cfl_rule": "min", "nu": 0.0,
         "tau_model": tau_model, "tau_coef": tau_coef,
         "bc": [_bc(bc), _bc(bc), _bc("extrap"), _bc("extrap")],
         "proj_mode": "discrete", "wall_es_term": True, "dt": 0.0, "precision": "fp64"}
    p.update(kw)
    return p


def centres(lo, hi, n):
    h = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * h


def conserved2d(rho, u1, u2, T):
    """Q = (rho, rho u1, rho u2, rho u1^2 + rho T, rho u1 u2, rho u2^2 + rho T) per cell, [ny][nx][6]."""
    rho, u1, u2, T = (np.asarray(a, dtype=np.float64) for a in (rho, u1, u2, T))
    return np.stack([rho, rho * u1, rho * u2, rho * u1 * u1 + rho * T, rho * u1 * u2,
                     rho * u2 * u2 + rho * T], axis=-1)


def conserved1d(rho, u, T):
    rho, u, T = (np.asarray(a, dtype=np.float64) for a in (rho, u, T))
    return np.stack([rho, rho * u, 0.5 * rho * T + 0.5 * rho * u * u], axis=-1)


def zero_g(p, dtype=np.float64):
    return np.zeros((p.get("ny", 1), p["nx"], p.get("nv2", 1), p["nv1"]), dtype=dtype)


# --------------------------------------------------------------------------
# the five workloads


def sod1d(nx=200, nv=64, V=8.0, eps=1e-2, cfl=0.5, **kw):
    """Sod tube on [0, 1]: (rho, u, T) = (1, 0, 1) left of 0.5, (0.125, 0, 0.8) right."""
    p = problem1d(nx, nv, V, eps=eps, cfl=cfl, **kw)
    x = centres(*p["x"], nx)
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    T = np.where(left, 1.0, 0.8)
    Q = conserved1d(rho, np.zeros(nx), T)
    return p, Q, zero_g(p)


def quadrant2d(seed=0, nx=64, ny=64, nv=24, V=8.0, eps=0.1, cfl=0.5, nu=-0.5, bc=None, **kw):
    """Quadrant Riemann problem; per quadrant rho ~ U[0.1,1], |u| ~ U[0,0.5], angle ~ U[0,2pi), T ~ U[0.5,1]."""
    p = problem2d(nx, ny, nv, nv, V, eps=eps, cfl=cfl, nu=nu, bc=bc if bc is not None else walls(), **kw)
    rng = np.random.default_rng(seed)
    st = []
    for _ in range(4):
        r = rng.uniform(0.1, 1.0)
        s = rng.uniform(0.0, 0.5)
        a = rng.uniform(0.0, 2.0 * math.pi)
        T = rng.uniform(0.5, 1.0)
        st.append((r, s * math.cos(a), s * math.sin(a), T))
    x = centres(*p["x"], nx)
    y = centres(*p["y"], ny)
    X, Y = np.meshgrid(x, y)              # [ny][nx]
    xm = 0.5 * (p["x"][0] + p["x"][1])
    ym = 0.5 * (p["y"][0] + p["y"][1])
    quad = (X >= xm).astype(int) + 2 * (Y >= ym).astype(int)
    fields = [np.choose(quad, [st[q][f] for q in range(4)]) for f in range(4)]
    Q = conserved2d(*fields)
    return p, Q, zero_g(p)


def fourier_field(rng, X, Y, modes=4):
    s = np.zeros_like(X)
    for _ in range(modes):
        kx, ky = rng.integers(1, 4, size=2)
        A = rng.uniform(0.5, 1.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        s += A * np.cos(2.0 * math.pi * (kx * X + ky * Y) + ph)
    return s / np.max(np.abs(s))


def cavity2d(seed=0, nx=256, ny=256, nv=32, V=7.0, eps=1e-2, cfl=0.5, nu=-0.5, lid=0.2, amp=0.1, **kw):
    """Cavity-style box: rho = 1 + amp s1, T = 1 + amp s2 (seeded Fourier sums), u = 0, walls, moving lid."""
    p = problem2d(nx, ny, nv, nv, V, eps=eps, cfl=cfl, nu=nu, bc=walls(1.0, lid), **kw)
    rng = np.random.default_rng(seed)
    x = centres(*p["x"], nx)
    y = centres(*p["y"], ny)
    X, Y = np.meshgrid(x, y)
    rho = 1.0 + amp * fourier_field(rng, X, Y)
    T = 1.0 + amp * fourier_field(rng, X, Y)
    Q = conserved2d(rho, np.zeros_like(X), np.zeros_like(X), T)
    return p, Q, zero_g(p)


def blast2d(seed=0, nx=512, ny=512, nv=48, V=8.0, eps=1e-2, cfl=0.5, nu=-0.5, sigma=0.05, **kw):
    """Gaussian blast: rho = 1 + 3 e^{-r^2/2s^2}, T = 1 + 2 e^{-r^2/2s^2}, centre (0.5,0.5) + U[-0.1,0.1]^2."""
    p = problem2d(nx, ny, nv, nv, V, eps=eps, cfl=cfl, nu=nu, bc=walls(1.0, 0.0), **kw)
    rng = np.random.default_rng(seed)
    cx, cy = 0.5 + rng.uniform(-0.1, 0.1, size=2)
    x = centres(*p["x"], nx)
    y = centres(*p["y"], ny)
    X, Y = np.meshgrid(x, y)
    e = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sigma * sigma))
    Q = conserved2d(1.0 + 3.0 * e, np.zeros_like(X), np.zeros_like(X), 1.0 + 2.0 * e)
    return p, Q, zero_g(p)


def smooth2d(seed=0, nx=16, ny=16, nv=16, V=8.0, eps=0.1, bc=None, amp=0.2, u_amp=0.2, **kw):
    """Smooth periodic-compatible state with nonzero velocity and anisotropic pressure (for tests)."""
    p = problem2d(nx, ny, nv, nv, V, eps=eps, bc=bc if bc is not None else periodic2d(), **kw)
    rng = np.random.default_rng(seed)
    x = centres(*p["x"], nx)
    y = centres(*p["y"], ny)
    X, Y = np.meshgrid(x, y)
    rho = 1.0 + amp * fourier_field(rng, X, Y)
    u1 = u_amp * fourier_field(rng, X, Y)
    u2 = u_amp * fourier_field(rng, X, Y)
    T = 1.0 + amp * fourier_field(rng, X, Y)
    Q = conserved2d(rho, u1, u2, T)
    # anisotropic pressure perturbation keeping tr P fixed
    d = 0.1 * amp * fourier_field(rng, X, Y) * rho * T
    o = 0.1 * amp * fourier_field(rng, X, Y) * rho * T
    Q[..., 3] += d
    Q[..., 5] -= d
    Q[..., 4] += o
    return p, Q, zero_g(p)


def cylsod2d(nx=320, nv=14, eps=5e-5, sub=20, **kw):
    """Cylindrical Sod problem (Sec. 6.2): [-1,1]^2 x [-9,9]^2, extrapolation on every side,
    nu = 0 and tau = rho, CFL 0.95 with the rule CFL = dt (V1/dx + V2/dy) the printed run
    follows (213 steps to t = 0.07 at 320^2).  Q_in = (1, 0, 0, 5, 0, 5) inside r = 0.5,
    Q_out = (0.125, 0, 0, 0.5, 0, 0.5) outside; a cell the circle cuts takes
    w Q_in + (1 - w) Q_out, w the fraction of sub x sub points of the cell inside."""
    p = problem2d(nx, nx, nv, nv, 9.0, eps=eps, cfl=0.95, nu=0.0, bc=extrap2d(), x=(-1.0, 1.0), y=(-1.0, 1.0),
                  tau_model="rho", tau_coef=1.0, **kw)
    p["cfl_rule"] = "sum"
    h = 2.0 / nx
    lo = -1.0 + h * np.arange(nx)                          # cell lower edges
    off = (np.arange(sub) + 0.5) * h / sub
    px = (lo[:, None] + off[None, :]).reshape(-1)          # sub points per cell, all cells
    inside = (px[None, :] ** 2 + px[:, None] ** 2) < 0.25   # [y points][x points]
    w = inside.reshape(nx, sub, nx, sub).mean(axis=(1, 3))  # [j][i]
    q_in = np.array([1.0, 0.0, 0.0, 5.0, 0.0, 5.0])
    q_out = np.array([0.125, 0.0, 0.0, 0.5, 0.0, 0.5])
    Q = w[..., None] * q_in + (1.0 - w[..., None]) * q_out
    return p, Q, zero_g(p)


CONFIGS = {
    "c1_sod1d": lambda seed=0: sod1d(),
    "c2_quadrant": lambda seed=0: quadrant2d(seed=seed),
    "c3_cavity": lambda seed=0, eps=1e-2: cavity2d(seed=seed, eps=eps),
    "c4_blast": lambda seed=0: blast2d(seed=seed),
}

STEPS = {"c1_sod1d": 100, "c2_quadrant": 200, "c3_cavity": 100, "c4_blast": 500}
