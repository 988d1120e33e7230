"""Graph capture of the allocation-free step: with failed_step NULL,
mm_step2d_noalloc enqueues kernel launches only (no memset, copy or
synchronisation), so a caller can capture it in a HIP graph and replay it.  Each
replay, with eager work and synchronisations between replays, is checked against
the same steps run eagerly on copies of the input (identical results)."""
import numpy as np
import pytest

import mm_workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_steps_replayed_from_a_graph(precision):
    import torch
    from paper_2509_21832_amd import binding as B
    p, Q, G = W.cavity2d(seed=6, nx=48, ny=40, nv=16, eps=0.02, amp=0.2)
    p["precision"] = precision
    G = 1e-3 * np.random.default_rng(6).standard_normal(Q.shape[:2] + (p["nv1"] * p["nv2"],))
    gdt = torch.float64 if precision == "fp64" else torch.float32
    steps = 2                                       # even: G^n returns to the first buffer

    def state():
        q = torch.tensor(Q.reshape(-1), dtype=torch.float64, device="cuda")
        g0 = torch.tensor(G.reshape(-1), dtype=gdt, device="cuda")
        return q, g0, torch.zeros_like(g0), torch.zeros(p["nx"] * p["ny"] * 4, dtype=torch.float64, device="cuda")

    qe, ge0, ge1, he = state()                      # eager copy
    qg, gg0, gg1, hg = state()                      # graph copy
    # the first call on a device looks up the static array's address: made outside capture
    qw, gw0, gw1, hw = state()
    assert B.step2d_noalloc(p, qw, gw0, gw1, steps, h=hw) == -1
    torch.cuda.synchronize()
    print(f"[graph] {precision}: capture of {steps} steps", flush=True)
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        B.step2d_noalloc(p, qg, gg0, gg1, steps, h=hg, stream=s.cuda_stream, wait=False)
    torch.cuda.synchronize()
    # capture records the launches without running them
    assert torch.equal(qg, qe) and torch.equal(gg0, ge0)
    for r in range(4):
        graph.replay()
        torch.cuda.synchronize()
        junk = torch.randn(4096, device="cuda").sum()      # eager work between replays
        assert B.step2d_noalloc(p, qe, ge0, ge1, steps, h=he) == -1
        torch.cuda.synchronize()
        same = torch.equal(qg, qe) and torch.equal(gg0, ge0) and torch.equal(gg1, ge1) and torch.equal(hg, he)
        print(f"[graph] {precision} replay {r}: identical to eager {same} ({float(junk):.3f})", flush=True)
        assert same
