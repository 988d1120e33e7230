"""The 1D diffuse walls (Sec. 4.3) on the GPU against the oracle, through the C ABI:
short runs element by element, and the heat-transfer runs of the section to t = 100
(the Knudsen sweep's scaled heat flux at x = 0.5)."""
import numpy as np
import pytest

import mm_workloads as W
import oracle
from gpu_common import log, rel_l1, run_gpu
from test_oracle_wall1d import heat_problem, _flowing_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,eps,steps", [(24, 0.05, 150), (37, 1e-3, 200), (30, 10.0, 120)])
def test_wall1d_parity(n, eps, steps):
    p = heat_problem(n, eps)
    Q = _flowing_state(n)
    G = 1e-3 * np.random.default_rng(n).standard_normal((n, n))
    log(f"[wall1d] n={n} eps={eps} steps={steps}")
    Qg, Gg, Hg = run_gpu(p, Q, G, steps)
    Qo, Go, Ho = oracle.run(p, Q.reshape(-1), G.reshape(-1), steps)
    e = rel_l1(Qg, Qo)
    ge = np.abs(Gg - Go).max() / np.abs(Go).max()
    he = np.abs(Hg - Ho).max() / np.abs(Ho).max()
    log(f"[wall1d] Q rel-L1 {e:.3e}; G max rel {ge:.3e}; H max rel {he:.3e}")
    assert e <= 1e-12
    assert ge <= 1e-10
    assert he <= 1e-10


@pytest.mark.parametrize("eps", [1e-2, 1.0, 1e30])
def test_wall1d_heat_transfer_to_t100(eps):
    """The section's run (N_x = N_v = 33, CFL 0.95, t = 100: 20,843 steps): |h_1| at x = 0.5
    and the final macro state against the oracle."""
    n = 33
    p = heat_problem(n, eps)
    dt, nsteps = oracle.dt(p, 100.0)
    p["dt"] = dt
    Q = W.conserved1d(np.ones(n), np.zeros(n), np.ones(n))
    G = np.zeros((n, n))
    log(f"[heat t=100] eps={eps:g}: {nsteps} steps")
    Qg, Gg, Hg = run_gpu(p, Q, G, nsteps, chunks=8)
    Qo, Go, Ho = oracle.run(p, Q.reshape(-1), G.reshape(-1), nsteps)
    hg, ho = abs(Hg[n // 2]) / eps, abs(Ho[n // 2]) / eps
    log(f"[heat t=100] eps={eps:g}: |h1| GPU {hg:.10f} oracle {ho:.10f}; Q rel-L1 {rel_l1(Qg, Qo):.3e}")
    assert rel_l1(Qg, Qo) <= 1e-11
    assert abs(hg - ho) <= 1e-10 * ho
