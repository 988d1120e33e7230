"""GPU tests of the boundary's helper paths, through the C ABI:
checkpoint / restart (mm_moments + mm_get_g, then mm_set_state), a state that
turns non-physical in the middle of a run (mm_step's status and
mm_failed_step), and the g-moment output of mm_moments against its definition
and the oracle."""
import numpy as np
import pytest

import mm_workloads as W
import oracle
from gpu_common import log, rel_l1

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_checkpoint_restart_bitwise(precision):
    """100 steps in one run equal 50 steps, a checkpoint (Q and G copied to the host),
    a restart of a fresh context from it (mm_set_state), and 50 more, bit for bit."""
    from paper_2509_21832_amd import binding as B
    p, Q, G = W.cavity2d(seed=2, nx=48, ny=40, nv=16, eps=0.02, amp=0.2)
    p["precision"] = precision
    log(f"[restart {precision}] 100 straight")
    with B.Solver(p, Q, G) as s:
        s.step(100)
        Qa = s.moments()
        Ga = s.get_g()
    log(f"[restart {precision}] 50 + checkpoint + 50")
    with B.Solver(p, Q, G) as s:
        s.step(50)
        Qc = s.moments()
        Gc = s.get_g()
    # a different initial state, replaced by the checkpoint
    p2, Q2, G2 = W.cavity2d(seed=9, nx=48, ny=40, nv=16, eps=0.02, amp=0.2)
    with B.Solver(p, Q2, None) as s:
        s.set_state(Qc, Gc)
        s.step(50)
        Qb = s.moments()
        Gb = s.get_g()
    assert np.array_equal(Qa, Qb)
    assert np.array_equal(Ga, Gb)


def test_nonphysical_state_mid_run():
    """An unstable time step (CFL 3, free transport at eps = 1e6) drives the quadrant
    problem to a non-physical state after some steps: mm_step reports MM_ENONPHYS and
    mm_failed_step gives the same first failing step as the oracle."""
    from paper_2509_21832_amd import binding as B
    p, Q, G = W.quadrant2d(seed=0, nx=16, ny=16, nv=16, eps=1e6)
    p["cfl"] = 3.0
    with pytest.raises(oracle.NonPhysical) as eo:
        oracle.run(p, Q.reshape(-1), G.reshape(-1), 40)
    o_step = int(str(eo.value).split()[-1])
    log(f"[nonphys] oracle: first non-physical state after step {o_step}")
    assert 2 <= o_step < 40
    # the steps before are physical and match the oracle
    with B.Solver(p, Q, G) as s:
        s.step(o_step - 1)
        Qg = s.moments()
    Qo, Go, Ho = oracle.run(p, Q.reshape(-1), G.reshape(-1), o_step - 1)
    assert rel_l1(Qg, Qo) <= 1e-12
    with B.Solver(p, Q, G) as s:
        with pytest.raises(B.NonPhysical):
            s.step(40)
        log(f"[nonphys] library: failed step {s.failed_step()}")
        assert s.failed_step() == o_step
        # the context stays usable: a restart from the initial state runs again
        s.set_state(Q, G)
        assert s.failed_step() == -1
        s.step(o_step - 1)
        assert rel_l1(s.moments(), Qo) <= 1e-12


def _gmom_definition(p, Q, G):
    """dv sum (1, v1, v2, |v|^2 / 2) G and eps dv sum (w1^2 - w2^2, 2 w1 w2, |w|^2) G / 2
    with w = v - u of the cell (the g-moment layout of mm_moments)."""
    ny, nx = p["ny"], p["nx"]
    v1 = W.centres(*p["v1"], p["nv1"])
    v2 = W.centres(*p["v2"], p["nv2"])
    V1, V2 = np.meshgrid(v1, v2)                      # [l][k]
    dv = (v1[1] - v1[0]) * (v2[1] - v2[0])
    Q = Q.reshape(ny, nx, 6)
    G = G.reshape(ny, nx, p["nv2"], p["nv1"])
    u1 = (Q[..., 1] / Q[..., 0])[..., None, None]
    u2 = (Q[..., 2] / Q[..., 0])[..., None, None]
    w1, w2 = V1 - u1, V2 - u2
    out = np.empty((ny, nx, 7))
    out[..., 0] = dv * G.sum(axis=(2, 3))
    out[..., 1] = dv * (V1 * G).sum(axis=(2, 3))
    out[..., 2] = dv * (V2 * G).sum(axis=(2, 3))
    out[..., 3] = dv * (0.5 * (V1 * V1 + V2 * V2) * G).sum(axis=(2, 3))
    out[..., 4] = 0.5 * p["eps"] * dv * ((w1 * w1 - w2 * w2) * G).sum(axis=(2, 3))
    out[..., 5] = 0.5 * p["eps"] * dv * (2.0 * w1 * w2 * G).sum(axis=(2, 3))
    out[..., 6] = 0.5 * p["eps"] * dv * ((w1 * w1 + w2 * w2) * G).sum(axis=(2, 3))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gmoments_against_definition_and_oracle(precision):
    from paper_2509_21832_amd import binding as B
    p, Q, G = W.cavity2d(seed=4, nx=24, ny=20, nv=16, eps=0.05, amp=0.2)
    p["precision"] = precision
    steps = 6
    with B.Solver(p, Q, G) as s:
        s.step(steps)
        Qg, Hg, Mg = s.moments(with_h=True, with_gmom=True)
        Gg = s.get_g()
    Mg = Mg.reshape(p["ny"], p["nx"], 7)
    # the library's reduction against the definition on its own G and Q
    Md = _gmom_definition(p, Qg, Gg)
    scale_c = np.abs(Md[..., :4]).max() + 1e-300
    stress = np.abs(Md[..., 4:]).max()
    assert np.abs(Mg[..., 4:] - Md[..., 4:]).max() <= 1e-12 * stress
    assert np.abs(Mg[..., :4] - Md[..., :4]).max() <= 1e-12 * max(scale_c, stress)
    # against the oracle's G after the same steps
    Qo, Go, Ho = oracle.run(p, Q.reshape(-1), G.reshape(-1), steps)
    Mo = _gmom_definition(p, Qo, Go)
    tol = 1e-11 if precision == "fp64" else 1e-5
    log(f"[gmom {precision}] stress scale {stress:.3e}; conserved g-moments max {np.abs(Mg[..., :4]).max():.3e}")
    assert np.abs(Mg[..., 4:] - Mo[..., 4:]).max() <= tol * stress
    # conserved moments of g vanish (discrete projector), to the storage precision
    assert np.abs(Mg[..., :4]).max() <= (1e-13 if precision == "fp64" else 1e-5) * stress / p["eps"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_caller_device_buffers(precision):
    """mm_config.dev_buffers: the state lives in caller-owned GPU tensors (G0, G1, Q).
    Steps give the same results bit for bit as a context with library buffers, the
    tensors hold the state without a copy, and Q0 = NULL takes the state already there."""
    import torch
    from paper_2509_21832_amd import binding as B
    p, Q, G = W.cavity2d(seed=6, nx=30, ny=22, nv=16, eps=0.03, amp=0.2)
    p["precision"] = precision
    rng = np.random.default_rng(1)
    G = 1e-3 * rng.standard_normal(G.shape)
    steps = 7
    with B.Solver(p, Q, G) as s:
        s.step(steps)
        Qa = s.moments()
        Ga = s.get_g()
    gdt = torch.float64 if precision == "fp64" else torch.float32
    n = p["nx"] * p["ny"] * p["nv1"] * p["nv2"]
    g0 = torch.zeros(n, dtype=gdt, device="cuda")
    g1 = torch.zeros(n, dtype=gdt, device="cuda")
    q = torch.zeros(p["nx"] * p["ny"] * 6, dtype=torch.float64, device="cuda")
    # host initial data uploaded into the caller's buffers
    with B.Solver(p, Q, G, dev_buffers=(g0, g1, q)) as s:
        qa, ga, ha, gb = s.device_ptrs()
        assert qa == q.data_ptr() and ga == g0.data_ptr()
        s.step(steps)
        Qb = s.moments()
        Gb = s.get_g()
        assert s.device_ptrs()[1] == g1.data_ptr()        # odd number of steps: G^n in G1
    torch.cuda.synchronize()
    assert np.array_equal(Qa, Qb) and np.array_equal(Ga, Gb)
    assert np.array_equal(q.cpu().numpy(), Qa)
    assert np.array_equal(g1.double().cpu().numpy(), Ga)
    # the state already in the buffers (Q0 = NULL)
    q.copy_(torch.from_numpy(np.ascontiguousarray(Q.reshape(-1))))
    g0.copy_(torch.from_numpy(np.ascontiguousarray(G.reshape(-1))).to(gdt))
    torch.cuda.synchronize()
    with B.Solver(p, None, dev_buffers=(g0, g1, q)) as s:
        s.step(steps)
        Qc = s.moments()
    assert np.array_equal(Qa, Qc)
