"""The learned-closure form on the GPU (through the C ABI) against the oracle:
features and indicator, the network's forward pass and gradient (bf16 matrix
cores vs an FP64 evaluation at the same rounding points), the rebuilt micro
part, two hybrid steps assembled from oracle pieces, and the trained closure
checked against the full micro solve."""
import numpy as np
import pytest

import mm_workloads as W
import oracle
from gpu_common import log, rel_l1

pytestmark = pytest.mark.gpu

NF, NO = 30, 7


def _torch():
    import torch
    return torch


def _B():
    from paper_2509_21832_amd import binding as B
    return B


def _cavity(seed=3, nx=13, ny=11, nv=16, eps=0.01, amp=0.2):
    return W.cavity2d(seed=seed, nx=nx, ny=ny, nv=nv, eps=eps, amp=amp)


def _developed(p, Q, G, steps=5):
    """A state with nonzero velocity and g: a few oracle steps."""
    Qo, Go, Ho = oracle.run(p, Q.reshape(-1), G.reshape(-1), steps)
    return Qo, Go


# ---------------------------------------------------------------- features

@pytest.mark.parametrize("case", ["cavity_walls", "periodic"])
def test_features_vs_oracle(case):
    if case == "cavity_walls":
        p, Q, G = _cavity()
    else:
        p, Q, G = W.smooth2d(seed=4, nx=12, ny=10, nv=16, eps=0.05)
    Q, G = _developed(p, Q, G)
    B = _B()
    with B.Solver(p, Q, G) as s:
        F, kn, edge = s.closure_features()
    Fo, kno, edgeo = oracle.features2d(p, Q)
    scale = np.abs(Fo).mean(0) + 1e-30
    err = np.abs(F - Fo) / (np.abs(Fo) + scale)
    log(f"[features {case}] max rel {err.max():.3e}; kn max rel {np.max(np.abs(kn - kno) / kno):.3e}")
    assert err.max() <= 1e-6
    assert np.allclose(kn, kno, rtol=1e-5, atol=1e-12)
    assert np.array_equal(edge, edgeo)


# ---------------------------------------------------------------- network

def _net(seed, scale=0.25):
    rng = np.random.default_rng(seed)
    P = (rng.standard_normal(oracle.mlp_nparam()) * scale).astype(np.float32)
    N = np.concatenate([rng.standard_normal(NF), rng.uniform(0.5, 2.0, NF), rng.standard_normal(NO),
                        rng.uniform(0.5, 2.0, NO)]).astype(np.float32)
    return P, N


def _oracle_params(P):
    """The parameters as the kernels see them: weight matrices rounded to bf16, biases FP32."""
    P64 = P.astype(np.float64)
    nw1, nb1, nw2, nb2, nw3 = 64 * NF, 64, 64 * 64, 64, NO * 64
    o = 0
    out = P64.copy()
    for n, is_w in ((nw1, True), (nb1, False), (nw2, True), (nb2, False), (nw3, True)):
        if is_w:
            out[o:o + n] = [oracle.bf16(v) for v in P64[o:o + n]]
        o += n
    return out


def _norm_dict(N):
    N = N.astype(np.float64)
    return {"in_mean": N[:NF], "in_std": N[NF:2 * NF], "out_mean": N[2 * NF:2 * NF + NO],
            "out_std": N[2 * NF + NO:]}


def _inputs(N, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, NF)) * N[NF:2 * NF] + N[:NF]
    return X.astype(np.float32)


def test_mlp_forward_vs_oracle():
    torch = _torch()
    B = _B()
    P, N = _net(1)
    n = 1000                                  # 31 full tiles of 32 and a ragged tail of 8
    X = _inputs(N, n, 2)
    net = B.Mlp(seed=0)
    net.set(P, N)
    Y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    Yo = oracle.mlp_forward(_oracle_params(P), _norm_dict(N), X.astype(np.float64), bf16=True)
    e = np.abs(Y - Yo) / N[2 * NF + NO:]
    log(f"[mlp forward] max {e.max():.3e} mean {e.mean():.3e} (in units of out_std)")
    # the two sides round the same quantities to bf16; they differ by FP32 vs FP64
    # sums and rare one-ulp (2^-8) flips of an activation at a rounding boundary
    assert e.mean() <= 1e-4
    assert e.max() <= 1e-2


def test_mlp_forward_empty_and_tiny():
    torch = _torch()
    B = _B()
    P, N = _net(3)
    net = B.Mlp(seed=0)
    net.set(P, N)
    for n in (1, 31, 33):
        X = _inputs(N, n, 4)
        Y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
        Yo = oracle.mlp_forward(_oracle_params(P), _norm_dict(N), X.astype(np.float64), bf16=True)
        assert np.abs(Y - Yo).max() <= 1e-2 * N[2 * NF + NO:].max()
    Y0 = net.forward(torch.empty((0, NF), dtype=torch.float32, device="cuda"))
    assert Y0.shape == (0, NO)


def test_mlp_grad_vs_oracle():
    torch = _torch()
    B = _B()
    P, N = _net(5)
    n = 777
    X = _inputs(N, n, 6)
    rng = np.random.default_rng(7)
    Yt = (rng.standard_normal((n, NO)) * N[2 * NF + NO:] + N[2 * NF:2 * NF + NO]).astype(np.float32)
    net = B.Mlp(seed=0)
    net.set(P, N)
    g, L = net.grad(torch.from_numpy(X).cuda(), torch.from_numpy(Yt).cuda())
    go, Lo = oracle.mlp_grad(_oracle_params(P), _norm_dict(N), X.astype(np.float64), Yt.astype(np.float64),
                             bf16=True)
    e = np.linalg.norm(g - go) / np.linalg.norm(go)
    o = np.cumsum([0, 64 * NF, 64, 64 * 64, 64, NO * 64, NO])
    blocks = {k: (o[i], o[i + 1]) for i, k in enumerate(("W1", "b1", "W2", "b2", "W3", "b3"))}
    eb = {k: np.linalg.norm(g[a:b] - go[a:b]) / np.linalg.norm(go[a:b]) for k, (a, b) in blocks.items()}
    log(f"[mlp grad] rel L2 {e:.3e}; per block " + " ".join(f"{k} {v:.2e}" for k, v in eb.items()) +
        f"; loss {L:.6f} vs {Lo:.6f}")
    assert abs(L - Lo) <= 1e-4 * Lo
    assert e <= 1e-3
    assert max(eb.values()) <= 3e-3


def test_mlp_fit_norm_mean_and_std():
    """mm_mlp_fit_norm: population mean and standard deviation of every feature and target
    column (FP64 sums); a constant column gets the floor 1e-6 x its root mean square."""
    torch = _torch()
    B = _B()
    rng = np.random.default_rng(12)
    n = 3001
    X = (rng.standard_normal((n, NF)) * rng.uniform(0.01, 100.0, NF) + rng.standard_normal(NF) * 10).astype(np.float32)
    Y = (rng.standard_normal((n, NO)) * rng.uniform(0.1, 5.0, NO) + rng.standard_normal(NO)).astype(np.float32)
    X[:, 3] = 2.5                     # a constant feature
    net = B.Mlp(seed=0)
    net.fit_norm(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda())
    _, N = net.get()
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    sx, sy = X64.std(0), Y64.std(0)
    sx[3] = 1e-6 * 2.5
    ref = np.concatenate([X64.mean(0), sx, Y64.mean(0), sy])
    err = np.abs(N - ref) / np.abs(ref)
    log(f"[fit_norm] max rel {err.max():.3e}")
    assert err.max() <= 1e-5


def test_mlp_train_reduces_loss():
    """Adam on the GPU fits a smooth map of real features."""
    torch = _torch()
    B = _B()
    p, Q, G = W.cavity2d(seed=8, nx=48, ny=48, nv=16, eps=0.01, amp=0.3)
    with B.Solver(p, Q, G) as s:
        s.step(5)
        F, kn, edge = s.closure_features()
    X = F.astype(np.float64)
    # targets: a smooth function of the features (stand-in for the micro moments)
    Yt = np.stack([X[:, 10] * X[:, 0], X[:, 17] * X[:, 3], X[:, 8] - X[:, 16], np.tanh(X[:, 15] + X[:, 9]),
                   X[:, 4] - X[:, 6], X[:, 1] * X[:, 2], np.tanh(X[:, 11] - X[:, 18])], 1).astype(np.float32)
    Xt = torch.from_numpy(F).cuda()
    Yd = torch.from_numpy(Yt).cuda()
    net = B.Mlp(seed=1)
    net.fit_norm(Xt, Yd)
    _, L0 = net.grad(Xt, Yd)
    losses = net.train(Xt, Yd, epochs=30, batch=256, lr=3e-3, seed=2)
    _, L1 = net.grad(Xt, Yd)
    log(f"[mlp train] loss {L0:.4f} -> {L1:.5f}; epochs {np.round(losses[[0, 9, 19, 29]], 5)}")
    assert np.all(np.isfinite(losses))
    assert L1 < 0.05 * L0


# ---------------------------------------------------------------- rebuilt micro part

@pytest.mark.parametrize("proj", ["discrete", "paper"])
def test_closure_rebuild_vs_oracle(proj):
    B = _B()
    p, Q, G = _cavity(seed=9, nx=9, ny=7, nv=16)
    p["proj_mode"] = proj
    Q, G = _developed(p, Q, G, 3)
    p["precision"] = "mixed"
    ncell = p["nx"] * p["ny"]
    rng = np.random.default_rng(10)
    out = (rng.standard_normal((ncell, NO)) * 0.3).astype(np.float32)
    mask = rng.uniform(size=ncell) < 0.4
    with B.Solver(p, Q, G) as s:
        s.closure_rebuild(out, mask)
        cells = np.nonzero(mask)[0]
        Gg = s.get_g_cells(cells)
        keep = s.get_g_cells(np.nonzero(~mask)[0])
    Qc = Q.reshape(ncell, 6)
    o64 = out.astype(np.float64)
    ref = np.stack([oracle.closure_grec(p, Qc[c], o64[c, :2], o64[c, 2:5], o64[c, 5:7]) for c in cells])
    e = np.abs(Gg - ref).max() / np.abs(ref).max()
    log(f"[rebuild {proj}] {len(cells)} cells, max rel {e:.3e}")
    assert e <= 1e-6
    # untouched cells keep their g (FP32 copy of the input)
    Gc = G.reshape(ncell, -1)[~mask]
    assert np.abs(keep - Gc).max() <= 1e-6 * np.abs(Gc).max()


# ---------------------------------------------------------------- training snapshots

@pytest.mark.parametrize("residual", [0, 1, 2])
def test_closure_snapshot_vs_oracle(residual):
    """mm_closure_snapshot on an FP64 context: features of Q^n and one step, then the rows of
    the cells with kn <= kn_max not next to a wall, in cell order, with targets
    (q1, q2, S11, S12, S22, t1, t2) / eps of g^{n+1} (w = v - u^n): q and t from the oracle's
    H, S = dv sum w w^T g; minus the NSF values (residual 1), divided by eps (residual 2)."""
    torch = _torch()
    B = _B()
    p, Q, G = _cavity(seed=21, nx=13, ny=11, nv=16, eps=0.02)
    Q, G = _developed(p, Q, G, 4)
    F, kn, edge = oracle.features2d(p, Q)
    # the NSF baseline from the features as the kernels hold them (FP32)
    nsf = np.array([np.concatenate(oracle.nsf_closure(p, f)) for f in F.astype(np.float32).astype(np.float64)])
    ks = np.sort(kn[~edge])
    kn_max = float(0.5 * (ks[len(ks) // 2] + ks[len(ks) // 2 + 1]))   # between two cells' values
    sel = (~edge) & (kn <= kn_max)
    cap = p["nx"] * p["ny"] + 5
    X = torch.zeros((cap, NF), dtype=torch.float32, device="cuda")
    Y = torch.zeros((cap, NO), dtype=torch.float32, device="cuda")
    with B.Solver(p, Q, G) as s:
        n = s.closure_snapshot(kn_max, X, Y, 2, residual=residual)      # appended after two rows
    Xg, Yg = X.cpu().numpy(), Y.cpu().numpy()
    # the oracle: one step, H and the stress of g^{n+1} about u^n
    Qo, Go, Ho = oracle.run(p, Q.reshape(-1), G.reshape(-1), 1)
    ncell = p["nx"] * p["ny"]
    Go = Go.reshape(ncell, p["nv2"], p["nv1"])
    Ho = Ho.reshape(ncell, 4)
    v1 = W.centres(*p["v1"], p["nv1"])
    v2 = W.centres(*p["v2"], p["nv2"])
    V1, V2 = np.meshgrid(v1, v2)
    dv = (v1[1] - v1[0]) * (v2[1] - v2[0])
    Qc = Q.reshape(ncell, 6)
    eps = p["eps"]
    T = np.zeros((ncell, NO))
    for c in range(ncell):
        w1, w2 = V1 - Qc[c, 1] / Qc[c, 0], V2 - Qc[c, 2] / Qc[c, 0]
        g, h = Go[c], Ho[c]
        T[c] = [0.5 * (h[0] + h[2]) / eps, 0.5 * (h[1] + h[3]) / eps, dv * np.sum(w1 * w1 * g),
                dv * np.sum(w1 * w2 * g), dv * np.sum(w2 * w2 * g), (h[0] - 3 * h[2]) / eps, (3 * h[1] - h[3]) / eps]
    if residual:
        T = (T - nsf) / (eps if residual == 2 else 1.0)
    rows = np.nonzero(sel)[0]
    log(f"[snapshot r={residual}] {len(rows)} rows of {ncell} cells (kn_max {kn_max:.3e})")
    assert n == 2 + len(rows)
    assert np.all(Xg[:2] == 0) and np.all(Yg[:2] == 0) and np.all(Xg[n:] == 0)
    fs = np.abs(F).mean(0) + 1e-30
    assert np.max(np.abs(Xg[2:n] - F[rows]) / (np.abs(F[rows]) + fs)) <= 1e-6
    ys = np.abs(T[rows]).mean(0) + 1e-30
    ey = np.abs(Yg[2:n] - T[rows]) / (np.abs(T[rows]) + ys)
    log(f"[snapshot r={residual}] targets max rel {ey.max():.3e}")
    assert ey.max() <= 1e-5


# ---------------------------------------------------------------- hybrid steps

def test_closure_with_all_cells_solved_equals_mixed():
    """kn_max = 0 on a non-uniform state: every cell keeps its micro solve, so the closure
    form must reproduce the FP32-storage form exactly."""
    B = _B()
    p, Q, G = _cavity(seed=11, nx=14, ny=12, nv=16)
    pm = dict(p, precision="mixed")
    pc = dict(p, precision="closure")
    with B.Solver(pm, Q, G) as s:
        s.step(10)
        Qm, Hm = s.moments(with_h=True)
        Gm = s.get_g()
    with B.Solver(pc, Q, G) as s:
        s.closure_attach(None, 0.0)
        s.step(10)
        Qc, Hc = s.moments(with_h=True)
        Gc = s.get_g()
        ncl, cls = s.closure_cells()
    log(f"[all solved] closure cells {ncl}; max |dQ| {np.abs(Qc - Qm).max():.3e}")
    assert ncl == 0 and cls.all()
    assert np.array_equal(Qc, Qm) and np.array_equal(Hc, Hm) and np.array_equal(Gc, Gm)


def test_closure_without_closure_attached_is_rejected():
    B = _B()
    p, Q, G = _cavity(seed=12, nx=8, ny=8, nv=16)
    p["precision"] = "closure"
    with B.Solver(p, Q, G) as s:
        with pytest.raises(B.MMError):
            s.step(1)


def _nsf_out(p, Q):
    F, kn, edge = oracle.features2d(p, Q)
    out = np.array([np.concatenate(oracle.nsf_closure(p, f)) for f in F])
    return F, kn, edge, out


def _dilate(cls, p):
    """cells within the 3 x 3 block of a solved cell (walls: no wrap)"""
    c = cls.reshape(p["ny"], p["nx"]).astype(bool)
    per_x = p["bc"][0]["kind"] == "periodic"
    per_y = p["bc"][2]["kind"] == "periodic"
    out = np.zeros_like(c)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            s = np.roll(np.roll(c, dj, 0), di, 1)
            if not per_y:
                if dj == 1:
                    s[0, :] = False
                if dj == -1:
                    s[-1, :] = False
            if not per_x:
                if di == 1:
                    s[:, 0] = False
                if di == -1:
                    s[:, -1] = False
            out |= s
    return out.reshape(-1)


@pytest.mark.parametrize("case", ["cavity_walls", "periodic"])
def test_two_hybrid_steps_vs_oracle_pieces(case):
    """Two closure steps (NSF closure, threshold at the median indicator) against the oracle
    composed the same way: classes from the oracle indicator, H of eps (q, t) in closure
    cells (t = 0: the isotropic form), the oracle micro step on the cells it solves with the rebuilt micro parts
    of the closure cells they need, and the oracle macro step with the assembled H."""
    B = _B()
    if case == "cavity_walls":
        p, Q, G = _cavity(seed=13, nx=16, ny=13, nv=16, eps=0.01)
    else:
        p, Q, G = W.smooth2d(seed=14, nx=14, ny=12, nv=16, eps=0.02)
    Q, G = _developed(p, Q, G, 4)
    ncell = p["nx"] * p["ny"]
    F0, kn0, edge0, out0 = _nsf_out(p, Q)
    thr = float(np.median(kn0[~edge0]))
    pc = dict(p, precision="closure")
    with B.Solver(pc, Q, G) as s:
        s.closure_attach(None, thr)
        s.step(1)
        Q1, H1 = s.moments(with_h=True)
        _, cls1 = s.closure_cells()
        G1 = s.get_g()
        s.step(1)
        Q2, H2 = s.moments(with_h=True)
        _, cls2 = s.closure_cells()
        G2 = s.get_g()
    nv = p["nv1"] * p["nv2"]
    tol_gap = 1e-5 * thr

    def check_step(Qn, Gn_valid, valid, out_or, kn_or, edge_or, cls_gpu, Qg, Hg, Gg, label):
        clear = np.abs(kn_or - thr) > tol_gap          # cells not at the threshold
        cls_or = edge_or | (kn_or > thr)
        assert np.array_equal(cls_gpu.astype(bool)[clear], cls_or[clear]), label
        cls = cls_gpu.astype(bool)
        need = _dilate(cls, p)
        Gmod = Gn_valid.reshape(ncell, nv).copy()
        Qc = Qn.reshape(ncell, 6)
        for c in np.nonzero(need & ~valid)[0]:
            Gmod[c] = oracle.closure_grec(p, Qc[c], out_or[c, :2], out_or[c, 2:5], out_or[c, 5:7])
        Go, Ho = oracle.micro2d(p, Qn, Gmod.reshape(-1))
        Go = Go.reshape(ncell, nv)
        Ho = Ho.reshape(ncell, 4)
        Hg = Hg.reshape(ncell, 4)
        # closure cells: H of eps (q, t) (t = 0 for NSF: the isotropic form)
        hc = np.array([oracle.closure_H(p["eps"] * out_or[c, :2], p["eps"] * out_or[c, 5:7])
                       for c in range(ncell)])
        ecl = np.abs(Hg[~cls] - hc[~cls]).max() / (np.abs(hc[~cls]).max() + 1e-300) if (~cls).any() else 0.0
        # solved cells: the micro step
        gsc = np.abs(Go[cls]).max()
        eg = np.abs(Gg.reshape(ncell, nv)[cls] - Go[cls]).max() / gsc
        eh = np.abs(Hg[cls] - Ho[cls]).max() / np.abs(Ho[cls]).max()
        # macro step with the assembled H
        Qo = oracle.macro2d(p, Qn, Hg.reshape(-1))
        eq = rel_l1(Qg.reshape(-1), Qo)
        log(f"[{label}] closure cells {int((~cls).sum())}/{ncell}; H closure rel {ecl:.2e}; g solved rel "
            f"{eg:.2e}; H solved rel {eh:.2e}; Q rel-L1 {eq:.2e}")
        assert ecl <= 1e-5
        assert eg <= 1e-4 and eh <= 1e-4
        assert eq <= 1e-12
        return cls

    cls1b = check_step(Q, G, np.ones(ncell, bool), out0, kn0, edge0, cls1, Q1, H1, G1, f"{case} step 1")
    assert (~cls1b).sum() > 0 and cls1b.sum() > 0
    F1, kn1, edge1, out1 = _nsf_out(p, Q1)
    check_step(Q1, G1, cls1b, out1, kn1, edge1, cls2, Q2, H2, G2, f"{case} step 2")


# ---------------------------------------------------------------- trained closure

def _snapshots(B, torch, cases, steps, first, every, kn_max, cap, residual):
    from paper_2509_21832_amd import closure as CL
    return CL.snapshots(cases, steps=steps, first=first, every=every, kn_max=kn_max, residual=residual, cap=cap)


@pytest.fixture(scope="module")
def trained():
    """The closure network trained on the GPU on snapshots of cavity and quadrant runs at
    eps = 1e-3, 2e-3, 5e-3, 1e-2 on the grid of its use (256^2 cells, 32^2 velocity
    nodes): it learns the correction of the micro solve's (q, S, t) / eps to the
    Navier-Stokes-Fourier values, divided by eps."""
    from paper_2509_21832_amd import closure as CL
    net, losses, n = CL.trained_closure()
    log(f"[train] {n} samples; epoch losses {np.round(losses[[0, 4, 9, 19, 29]], 5)}")
    return net, losses


@pytest.mark.parametrize("eps", [1e-3, 3e-3, 1e-2])
def test_trained_closure_against_micro_solve(trained, eps):
    """Held-out cavity (another seed than the training runs) at 256^2 x 32^2: the closure
    form runs its initial layer with every cell solved (40 steps), then 100 steps with the
    closure; macro rel-L1 against the FP64 full micro solve over the same 140 steps at
    least 30 % below that of the Navier-Stokes-Fourier closure (the method without the
    network) run the same way, with at least 90 % of the cells on the closure.  On
    held-out snapshots of the same run, the network's heat flux, stress and traceless
    third moments each at least 20 % closer to the micro solve than the NSF values."""
    torch = _torch()
    B = _B()
    from paper_2509_21832_amd import closure as CL
    net, losses = trained
    assert losses[-1] < 0.5 * losses[0]
    p, Q, G = W.cavity2d(seed=41, eps=eps)
    steps = 100
    with B.Solver(p, Q, G) as s:                                    # reference: FP64 full solve
        s.step(CL.INITIAL_LAYER + steps)
        Qref = s.moments()
    res = {}
    for name, closure in (("net", net), ("nsf", None)):
        with B.Solver(dict(p, precision="closure"), Q, G) as s:
            CL.start(s, closure)
            s.closure_cells()
            s.step(steps)
            ncl, _ = s.closure_cells()
            res[name] = (rel_l1(s.moments(), Qref), ncl / (steps * p["nx"] * p["ny"]))
    gain = 1.0 - res["net"][0] / res["nsf"][0]
    log(f"[reference eps={eps:g}] macro rel-L1 vs FP64 full solve: net {res['net'][0]:.3e} (closure fraction "
        f"{res['net'][1]:.2f}), NSF {res['nsf'][0]:.3e}; gain {gain:.2f}")
    assert res["net"][0] <= 1e-2
    assert res["net"][1] >= 0.9
    assert gain >= 0.30

    # offline, on held-out snapshots after the initial layer: raw targets of the micro
    # solve vs NSF and vs NSF + network correction
    kw = dict(steps=CL.INITIAL_LAYER + steps, first=CL.INITIAL_LAYER, every=10, kn_max=CL.KN_MAX, cap=2_000_000)
    Xh, Yh = _snapshots(B, torch, [(p, Q, G)], residual=0, **kw)
    Xr, Yr = _snapshots(B, torch, [(p, Q, G)], residual=1, **kw)
    Yh = Yh.cpu().numpy().astype(np.float64)
    nsf = Yh - Yr.cpu().numpy()                      # the NSF values the kernels used
    Yn = nsf + p["eps"] * net.forward(Xh).cpu().numpy()
    rms = lambda a: float(np.sqrt(np.mean(a ** 2)))  # noqa: E731
    e = {k: (rms(Yn[:, a:b] - Yh[:, a:b]), rms(nsf[:, a:b] - Yh[:, a:b]), rms(Yh[:, a:b]))
         for k, (a, b) in (("heat flux", (0, 2)), ("stress", (2, 5)), ("traceless third moments", (5, 7)))}
    log(f"[gain eps={eps:g}] held-out RMS error, " + "; ".join(
        f"{k}: net {v[0]:.3e} NSF {v[1]:.3e} (target rms {v[2]:.3e})" for k, v in e.items()))
    for k, v in e.items():
        assert v[0] <= 0.8 * v[1], k


@pytest.mark.parametrize("seed,eps", [(45, 1e-3), (45, 3e-3), (46, 1e-3), (46, 3e-3)])
def test_trained_closure_on_held_out_quadrant_flows(trained, seed, eps):
    """The network on quadrant Riemann flows it has not seen (other seeds than the training
    runs) at 256^2 x 32^2: after the initial layer and 100 closure steps, macro rel-L1
    against the FP64 full solve at least 25 % below that of the NSF closure.  (At eps = 1e-2
    the gain depends on the flow: measured -2 % and +34 % for these two seeds.)"""
    B = _B()
    from paper_2509_21832_amd import closure as CL
    net, _ = trained
    p, Q, G = W.quadrant2d(seed=seed, nx=256, ny=256, nv=32, eps=eps)
    with B.Solver(p, Q, G) as s:
        s.step(CL.INITIAL_LAYER + 100)
        Qref = s.moments()
    res = {}
    for name, closure in (("net", net), ("nsf", None)):
        with B.Solver(dict(p, precision="closure"), Q, G) as s:
            CL.start(s, closure)
            s.step(100)
            res[name] = rel_l1(s.moments(), Qref)
    gain = 1.0 - res["net"] / res["nsf"]
    log(f"[quadrant seed={seed} eps={eps:g}] macro rel-L1: net {res['net']:.3e}, NSF {res['nsf']:.3e}; gain {gain:.2f}")
    assert gain >= 0.25


def test_trained_closure_speedup_at_full_size(trained):
    """256^2 cells x 32^2 velocity nodes, eps = 3e-3: the closure form against the
    FP32-storage full micro solve on the same GPU (wall time of 30 synchronised steps),
    its macro error against the FP64 full solve after its initial layer and 30 steps."""
    import time
    B = _B()
    from paper_2509_21832_amd import closure as CL
    net, _ = trained
    p, Q, G = W.cavity2d(seed=41, eps=3e-3)
    steps = 30
    with B.Solver(p, Q, G) as s:
        s.step(CL.INITIAL_LAYER + steps)
        Qref = s.moments()
    times, errs = {}, {}
    for form in ("mixed", "closure"):
        with B.Solver(dict(p, precision=form), Q, G) as s:
            if form == "closure":
                CL.start(s, net)
                s.closure_cells()
            else:
                s.step(CL.INITIAL_LAYER)
            s.step(steps)
            errs[form] = rel_l1(s.moments(), Qref)
            s.step(3)
            t0 = time.perf_counter()
            s.step(steps)
            times[form] = (time.perf_counter() - t0) / steps
            s.timing(True)
            s.step(5)
            parts = {k: s.timing_get(c)[1] / 5 for k, c in
                     (("pass", 0), ("prep", 1), ("macro", 2), ("wall", 3), ("closure", 4))}
            s.timing(False)
            log(f"[speed {form}] per step (ms): " + " ".join(f"{k} {v:.4f}" for k, v in parts.items()))
            if form == "closure":
                ncl, _ = s.closure_cells()
                frac = ncl / ((steps + 3 + steps + 5) * p["nx"] * p["ny"])
    sp = times["mixed"] / times["closure"]
    log(f"[speed] ms/step mixed {1e3 * times['mixed']:.3f}, closure {1e3 * times['closure']:.3f} "
        f"(x{sp:.2f}, closure fraction {frac:.2f}); macro rel-L1 vs FP64: mixed {errs['mixed']:.2e}, "
        f"closure {errs['closure']:.2e}")
    assert errs["closure"] <= 1e-2
    assert sp >= 1.5
