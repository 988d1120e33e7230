"""Training recipe of the learned closure (2D): snapshots from the solver's own
full micro solves, then the network trained on the GPU.  Every step runs in
the library's kernels (mm_closure_snapshot, mm_mlp_fit_norm, mm_mlp_train);
this module only chooses the runs and marshals device buffers.

The network learns residual kind 2: the correction of the micro solve's
(q, S, t) / eps to the Navier-Stokes-Fourier values, divided by eps (the leading
correction is first order in eps, so the target is nearly eps-independent and
the features carry no eps).
"""
import numpy as np

import mm_workloads as W

RESIDUAL = 2          # kind of residual the network predicts (see mm_closure_attach)
KN_TRAIN = 0.1        # snapshot cells up to twice the default threshold of the closure form
KN_MAX = 0.05         # threshold of the closure form


def training_runs(eps_list=(1e-3, 2e-3, 5e-3, 1e-2), nx=64, nv=16, seed0=20):
    """Cavity-box and quadrant-Riemann states, one of each per eps (seeded)."""
    runs = []
    for k, eps in enumerate(eps_list):
        runs.append(W.cavity2d(seed=seed0 + k, nx=nx, ny=nx, nv=nv, eps=eps, amp=0.2))
        runs.append(W.quadrant2d(seed=seed0 + 10 + k, nx=nx, ny=nx, nv=nv, eps=eps))
    return runs


def snapshots(runs, steps=160, first=40, every=6, kn_max=KN_TRAIN, residual=RESIDUAL, cap=4_000_000):
    """Training rows (device tensors X [n, 21], Y [n, 7]) from full micro solves with g in
    FP32: a snapshot every `every` steps from step `first` on (the first steps relax g from
    its zero initial value)."""
    import torch
    from . import binding as B
    X = torch.zeros((cap, B.N_FEAT), dtype=torch.float32, device="cuda")
    Y = torch.zeros((cap, B.N_OUT), dtype=torch.float32, device="cuda")
    count = 0
    for p, Q, G in runs:
        with B.Solver(dict(p, precision="mixed"), Q, G) as s:
            for k in range(steps):
                if k >= first and (k - first) % every == 0:
                    count = s.closure_snapshot(kn_max, X, Y, count, residual=residual)
                else:
                    s.step(1)
    return X[:count].contiguous(), Y[:count].contiguous()


def train(X, Y, epochs=30, batch=512, lr=2e-3, seed=3):
    """A network fitted to (X, Y) on the GPU; returns (net, per-epoch losses)."""
    from . import binding as B
    net = B.Mlp(seed=seed)
    net.fit_norm(X, Y)
    losses = net.train(X, Y, epochs=epochs, batch=batch, lr=lr, seed=seed + 1)
    return net, np.asarray(losses)


def trained_closure(**kw):
    """Snapshots of the default training runs and the trained network."""
    X, Y = snapshots(training_runs(**kw))
    net, losses = train(X, Y)
    return net, losses, int(X.shape[0])
