"""Limits with textbook solutions: free streaming as eps -> infinity and the
exact Euler Riemann solution as eps -> 0 (no GPU)."""
import math

import numpy as np
import pytest

import mm_workloads as W
import oracle
import riemann


def _free_stream_1d(nx, t=0.25, A=0.3, T=1.0):
    p = W.problem1d(nx, 48, 8.0, eps=1e8, bc="periodic")
    x = W.centres(0, 1, nx)
    rho0 = 1.0 + A * np.sin(2 * math.pi * x)
    Q = W.conserved1d(rho0, np.zeros(nx), np.full(nx, T))
    dt, n = oracle.dt(p, t)
    p["dt"] = dt
    Q1, G1, H = oracle.run(p, Q, W.zero_g(p), n)
    exact = 1.0 + A * math.exp(-2 * math.pi ** 2 * T * t * t) * np.sin(2 * math.pi * x)
    return np.abs(Q1.reshape(nx, 3)[:, 0] - exact).mean()


def test_free_streaming_1d():
    """eps -> infinity: rho(x, t) = 1 + A exp(-2 pi^2 T t^2) sin(2 pi x) for f0 = (1 + A sin 2 pi x) M."""
    e = [_free_stream_1d(n) for n in (50, 100, 200)]
    assert e[1] < 0.6 * e[0] and e[2] < 0.6 * e[1]      # first order
    assert e[2] < 0.01


def _free_stream_2d(n, t=0.1, A=0.3, T=1.0):
    p = W.problem2d(n, n, 16, 16, 6.0, eps=1e8, bc=W.periodic2d(), nu=-0.5)
    x = W.centres(0, 1, n)
    X, Y = np.meshgrid(x, x)
    rho0 = 1.0 + A * np.sin(2 * math.pi * (X + Y))
    Q = W.conserved2d(rho0, 0 * X, 0 * X, np.full_like(X, T))
    dt, ns = oracle.dt(p, t)
    p["dt"] = dt
    Q1, G1, H = oracle.run(p, Q.reshape(-1), W.zero_g(p).reshape(-1), ns)
    exact = 1.0 + A * math.exp(-2 * math.pi ** 2 * T * 2 * t * t) * np.sin(2 * math.pi * (X + Y))
    return np.abs(Q1.reshape(n, n, 6)[..., 0] - exact).mean()


def test_free_streaming_2d():
    e = [_free_stream_2d(n) for n in (16, 32)]
    assert e[1] < 0.65 * e[0]
    assert e[1] < 0.02


def _sod_rho(nx, dim, t=0.12):
    if dim == 1:
        p = W.problem1d(nx, 32, 8.0, eps=1e-8)
        x = W.centres(0, 1, nx)
        Q = W.conserved1d(np.where(x < 0.5, 1.0, 0.125), np.zeros(nx), np.where(x < 0.5, 1.0, 0.8))
        G = W.zero_g(p)
    else:
        ny = 3
        b = [{"kind": "extrap"}, {"kind": "extrap"}, {"kind": "periodic"}, {"kind": "periodic"}]
        p = W.problem2d(nx, ny, 10, 10, 8.0, eps=1e-8, bc=b, nu=-0.5, y=(0.0, 3.0 / nx))
        x = W.centres(0, 1, nx)
        X = np.tile(x, (ny, 1))
        Q = W.conserved2d(np.where(X < 0.5, 1.0, 0.125), 0 * X, 0 * X, np.where(X < 0.5, 1.0, 0.8))
        G = W.zero_g(p)
    dt, n = oracle.dt(p, t)
    p["dt"] = dt
    Q1, G1, H = oracle.run(p, Q.reshape(-1), G.reshape(-1), n)
    return x, Q1.reshape(-1, 3 if dim == 1 else 6)[:nx, 0]


def _exact(x, gamma, t=0.12):
    return riemann.sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), gamma, (x - 0.5) / t)[:, 0]


@pytest.mark.parametrize("dim,gamma", [(1, 3.0), (2, 2.0)])
def test_euler_limit_riemann(dim, gamma):
    """eps -> 0: the density converges to the exact Riemann solution of the
    Euler equations with gamma = (d_v + 2)/d_v (order about 1/2 for discontinuous data)."""
    e = []
    for n in (50, 100, 200, 400):
        x, rho = _sod_rho(n, dim)
        e.append(np.abs(rho - _exact(x, gamma)).mean())
    for a, b in zip(e, e[1:]):
        assert b < 0.75 * a
    assert e[-1] < 0.012
    # the solution is clearly closer to its own adiabatic exponent than to the other one
    wrong = 2.0 if gamma == 3.0 else 3.0
    assert np.abs(rho - _exact(x, wrong)).mean() > 2.5 * e[-1]
