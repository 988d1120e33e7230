"""Pins of the closure part of the oracle (features, indicator, network, closure
moments, rebuilt micro part, NSF values) against closed forms, independent
implementations and invariants."""
import math

import numpy as np
import pytest

import mm_workloads as W
import oracle

NF, NH, NO = 30, 64, 7


def _problem(nx=12, ny=10, nv=16, V=8.0, bc=None, eps=0.01, **kw):
    return W.problem2d(nx, ny, nv, nv, V, eps=eps, bc=bc if bc is not None else W.walls(), **kw)


# ------------------------------------------------------------------ GELU, bf16

def test_gelu_values():
    # gelu(x) = x Phi(x): Phi(1) = 0.841344746068543 (standard normal CDF)
    assert oracle.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-15)
    assert oracle.gelu(0.0) == 0.0
    assert oracle.gelu_d(0.0) == pytest.approx(0.5, rel=1e-15)
    for x in (-3.0, -0.7, 0.3, 2.5):
        # x Phi(x) - (-x) Phi(-x) = x
        assert oracle.gelu(x) - oracle.gelu(-x) == pytest.approx(x, rel=1e-14)
        h = 1e-5
        fd = (oracle.gelu(x + h) - oracle.gelu(x - h)) / (2 * h)
        assert oracle.gelu_d(x) == pytest.approx(fd, rel=1e-8)
    assert oracle.gelu(12.0) == pytest.approx(12.0, rel=1e-15)
    assert abs(oracle.gelu(-12.0)) < 1e-30


def _bf16_bits(x):
    """bfloat16 of float32 values by integer rounding of the bit pattern (to nearest, ties to even)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_rounding_matches_bit_rounding():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(4000) * np.exp(rng.uniform(-20, 20, 4000))).astype(np.float32)
    ref = _bf16_bits(x)
    got = np.array([oracle.bf16(float(v)) for v in x])
    assert np.array_equal(got, ref)
    # ties go to the even significand
    assert oracle.bf16(1.0 + 2.0 ** -8) == 1.0
    assert oracle.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


# ------------------------------------------------------------------ the network

def _random_net(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal(oracle.mlp_nparam()) * scale
    norm = {"in_mean": rng.standard_normal(NF), "in_std": rng.uniform(0.5, 2.0, NF),
            "out_mean": rng.standard_normal(NO), "out_std": rng.uniform(0.5, 2.0, NO)}
    return P, norm


def _split(P):
    o = 0
    out = []
    for shape in ((NH, NF), (NH,), (NH, NH), (NH,), (NO, NH), (NO,)):
        n = int(np.prod(shape))
        out.append(P[o:o + n].reshape(shape))
        o += n
    return out


def _join(parts):
    return np.concatenate([np.ravel(p) for p in parts])


def test_mlp_zero_weights_give_bias():
    P, norm = _random_net(1)
    W1, b1, W2, b2, W3, b3 = _split(P.copy())
    P0 = _join([W1, b1, W2, b2, np.zeros_like(W3), b3])
    X = np.random.default_rng(2).standard_normal((7, NF))
    Y = oracle.mlp_forward(P0, norm, X)
    assert np.allclose(Y, b3 * norm["out_std"] + norm["out_mean"], rtol=0, atol=1e-14)


def test_mlp_single_path_is_scalar_chain():
    """Only weights W1[3,5], W2[7,3], W3[2,7] nonzero: output 2 is a chain of scalar GELUs."""
    P = np.zeros(oracle.mlp_nparam())
    W1, b1, W2, b2, W3, b3 = _split(P)
    W1[3, 5], b1[3] = 0.8, -0.1
    W2[7, 3], b2[7] = -1.3, 0.4
    W3[2, 7], b3[2] = 0.9, 0.05
    norm = {"in_mean": np.zeros(NF), "in_std": np.ones(NF), "out_mean": np.zeros(NO), "out_std": np.ones(NO)}
    x = np.zeros(NF)
    x[5] = 1.7
    Phi = lambda t: 0.5 * (1 + math.erf(t / math.sqrt(2)))  # noqa: E731
    g = lambda t: t * Phi(t)  # noqa: E731
    a1 = g(0.8 * 1.7 - 0.1)
    # every other hidden unit of layer 1 has zero input: gelu(0) = 0; layer 2 units other
    # than 7 see only zeros as well
    a2 = g(-1.3 * a1 + 0.4)
    y = oracle.mlp_forward(_join([W1, b1, W2, b2, W3, b3]), norm, x[None, :])[0]
    assert y[2] == pytest.approx(0.9 * a2 + 0.05, rel=1e-14)
    assert np.all(y[[0, 1, 3, 4]] == 0.0)


def test_mlp_hidden_permutation_invariance():
    """Relabelling hidden units consistently leaves the function unchanged (catches a
    transposed weight index)."""
    P, norm = _random_net(3)
    W1, b1, W2, b2, W3, b3 = _split(P)
    rng = np.random.default_rng(4)
    p1, p2 = rng.permutation(NH), rng.permutation(NH)
    Pp = _join([W1[p1], b1[p1], W2[p2][:, p1], b2[p2], W3[:, p2], b3])
    X = rng.standard_normal((9, NF))
    assert np.allclose(oracle.mlp_forward(P, norm, X), oracle.mlp_forward(Pp, norm, X), rtol=1e-13, atol=1e-13)


def test_mlp_input_normalisation():
    """Shifting/scaling the inputs and the input statistics together changes nothing."""
    P, norm = _random_net(5)
    X = np.random.default_rng(6).standard_normal((5, NF))
    a, b = 3.0, -2.0
    n2 = dict(norm, in_mean=a * norm["in_mean"] + b, in_std=a * norm["in_std"])
    assert np.allclose(oracle.mlp_forward(P, norm, X), oracle.mlp_forward(P, n2, a * X + b), rtol=1e-12, atol=1e-12)


def test_mlp_gradient_vs_central_differences():
    P, norm = _random_net(7, scale=0.4)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((6, NF)) * norm["in_std"] + norm["in_mean"]
    Y = rng.standard_normal((6, NO))
    g, L = oracle.mlp_grad(P, norm, X, Y)
    # the loss itself from the forward pass
    yh = (oracle.mlp_forward(P, norm, X) - norm["out_mean"]) / norm["out_std"]
    t = (Y - norm["out_mean"]) / norm["out_std"]
    assert L == pytest.approx(np.mean((yh - t) ** 2), rel=1e-13)
    idx = np.concatenate([rng.choice(NH * NF, 25, replace=False),                      # W1
                          NH * NF + rng.choice(NH, 5, replace=False),                  # b1
                          NH * NF + NH + rng.choice(NH * NH, 25, replace=False),        # W2
                          NH * NF + NH + NH * NH + rng.choice(NH, 5, replace=False),    # b2
                          NH * NF + 2 * NH + NH * NH + rng.choice(NO * NH, 15, replace=False),  # W3
                          oracle.mlp_nparam() - NO + np.arange(NO)])                    # b3
    h = 1e-6
    # central differences carry round-off of about 1e-16 L / h
    fd_abs = 1e-16 * max(L, 1.0) / h * 10
    for k in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (oracle.mlp_grad(Pp, norm, X, Y)[1] - oracle.mlp_grad(Pm, norm, X, Y)[1]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=fd_abs), k


def test_mlp_bf16_mode_rounds_only_product_inputs():
    """With weights and inputs that are already bf16 values, the bf16 mode differs from the
    FP64 forward only through the rounding of the two hidden activation vectors: a small
    but nonzero change."""
    P, norm = _random_net(9)
    Pb = np.array([oracle.bf16(v) for v in P])
    norm0 = {"in_mean": np.zeros(NF), "in_std": np.ones(NF), "out_mean": np.zeros(NO), "out_std": np.ones(NO)}
    X = np.array([[oracle.bf16(v) for v in row] for row in np.random.default_rng(10).standard_normal((4, NF))])
    y64 = oracle.mlp_forward(Pb, norm0, X, bf16=False)
    y16 = oracle.mlp_forward(Pb, norm0, X, bf16=True)
    # rounding two 64-wide activation vectors to 8 significant bits moves the output by at
    # most about sum |W3| |W2| 2^-9 |a|; well below 5 %
    assert np.all(np.abs(y16 - y64) <= 0.05 * (np.abs(y64) + 1.0))
    assert not np.array_equal(y16, y64)


# ------------------------------------------------------------------ features

def _linear_state(p, a=(1.0, 0.3, -0.2), u=(0.1, 0.2, -0.05, 0.15, 0.1, -0.1), T=(1.0, 0.2, 0.1)):
    """rho, u1, u2, T linear in (x, y); isotropic pressure P = rho T I."""
    x = W.centres(*p["x"], p["nx"])
    y = W.centres(*p["y"], p["ny"])
    X, Y = np.meshgrid(x, y)
    rho = a[0] + a[1] * X + a[2] * Y
    u1 = u[0] + u[1] * X + u[2] * Y
    u2 = u[3] + u[4] * X + u[5] * Y
    Tf = T[0] + T[1] * X + T[2] * Y
    return W.conserved2d(rho, u1, u2, Tf), rho, u1, u2, Tf


def test_features_of_linear_fields_are_exact():
    p = _problem(nx=9, ny=7)
    Q, rho, u1, u2, T = _linear_state(p)
    F, kn, edge = oracle.features2d(p, Q.reshape(-1))
    F = F.reshape(p["ny"], p["nx"], NF)
    assert np.allclose(F[..., 0], rho, rtol=1e-14)
    assert np.allclose(F[..., 1], u1, rtol=1e-13, atol=1e-15)
    assert np.allclose(F[..., 3], T, rtol=1e-13)
    # P = rho T I: P11 = P22 = rho T, P12 = 0 (up to cancellation in E - rho u u)
    assert np.allclose(F[..., 4], rho * T, rtol=1e-12)
    assert np.allclose(F[..., 5], 0.0, atol=1e-13)
    # gradients of the linear fields, everywhere (one-sided differences at the edges are exact too)
    assert np.allclose(F[..., 7], 0.3, rtol=1e-10)
    assert np.allclose(F[..., 14], -0.2, rtol=1e-10)
    assert np.allclose(F[..., 8], 0.2, rtol=1e-9)
    assert np.allclose(F[..., 15], -0.05, rtol=1e-9)
    assert np.allclose(F[..., 9], 0.1, rtol=1e-9)
    assert np.allclose(F[..., 16], -0.1, rtol=1e-9)
    assert np.allclose(F[..., 10], 0.2, rtol=1e-9)
    assert np.allclose(F[..., 17], 0.1, rtol=1e-9)
    # indicator from the exact gradients (tau = tau_coef rho)
    gr = np.hypot(0.3, -0.2) / rho
    gT = np.hypot(0.2, 0.1) / T
    gu = np.sqrt(0.2 ** 2 + 0.05 ** 2 + 0.1 ** 2 + 0.1 ** 2) / np.sqrt(T)
    ref = p["eps"] * np.sqrt(T) / (p["tau_coef"] * rho) * np.maximum(np.maximum(gr, gT), gu)
    assert np.allclose(kn.reshape(p["ny"], p["nx"]), ref, rtol=1e-9)
    # the local mean free path eps sqrt(T) / tau, tau = tau_coef rho
    assert np.allclose(F[..., 21], p["eps"] * np.sqrt(T) / (p["tau_coef"] * rho), rtol=1e-13)
    # second differences of linear fields vanish; next to the walls they are set to zero
    scale = max(p["nx"] / (p["x"][1] - p["x"][0]), p["ny"] / (p["y"][1] - p["y"][0])) ** 2
    assert np.abs(F[..., 22:30]).max() <= 1e-12 * scale
    assert np.all(F[:, 0, 22:26] == 0) and np.all(F[:, -1, 22:26] == 0)
    assert np.all(F[0, :, 26:30] == 0) and np.all(F[-1, :, 26:30] == 0)
    # walls on all four sides: the outer ring is always micro
    e = edge.reshape(p["ny"], p["nx"])
    assert e[0].all() and e[-1].all() and e[:, 0].all() and e[:, -1].all()
    assert not e[1:-1, 1:-1].any()


def test_features_second_differences_of_quadratic_fields_are_exact():
    """The central second difference is exact for quadratics: d2/dx2 and d2/dy2 of
    (rho, u1, u2, T) in the interior, zero where a neighbour is missing."""
    p = _problem(nx=9, ny=8)
    x = W.centres(*p["x"], p["nx"])
    y = W.centres(*p["y"], p["ny"])
    X, Y = np.meshgrid(x, y)
    c = {"rho": (1.0, 0.3, -0.2), "u1": (0.1, 0.4, 0.25), "u2": (-0.05, -0.3, 0.2), "T": (1.0, 0.15, 0.35)}
    f = {k: a + b * X * X + d * Y * Y + 0.1 * X * Y for k, (a, b, d) in c.items()}
    Q = W.conserved2d(f["rho"], f["u1"], f["u2"], f["T"])
    F, kn, edge = oracle.features2d(p, Q.reshape(-1))
    F = F.reshape(p["ny"], p["nx"], NF)
    for a, k in enumerate(("rho", "u1", "u2", "T")):
        assert np.allclose(F[1:-1, 1:-1, 22 + a], 2 * c[k][1], rtol=1e-8), k
        assert np.allclose(F[1:-1, 1:-1, 26 + a], 2 * c[k][2], rtol=1e-8), k
        assert np.all(F[:, 0, 22 + a] == 0) and np.all(F[:, -1, 22 + a] == 0)
        assert np.all(F[0, :, 26 + a] == 0) and np.all(F[-1, :, 26 + a] == 0)
    # the mixed term x y adds nothing to either second difference; first differences
    # stay the centred ones: d rho / dx = 2 b x + 0.1 y exactly for a quadratic
    assert np.allclose(F[1:-1, 1:-1, 7], (2 * 0.3 * X + 0.1 * Y)[1:-1, 1:-1], rtol=1e-9, atol=1e-12)


def test_features_periodic_wrap_second_order():
    errs = []
    for n in (16, 32):
        p = _problem(nx=n, ny=n, bc=W.periodic2d())
        x = W.centres(*p["x"], n)
        X, Y = np.meshgrid(x, x)
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
        Q = W.conserved2d(rho, 0 * X, 0 * X, 1.0 + 0 * X)
        F, kn, edge = oracle.features2d(p, Q.reshape(-1))
        F = F.reshape(n, n, NF)
        exact = 0.2 * 2 * np.pi * np.cos(2 * np.pi * X) * np.cos(2 * np.pi * Y)
        exact2 = -0.2 * (2 * np.pi) ** 2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
        errs.append((np.abs(F[..., 7] - exact).max(), np.abs(F[..., 22] - exact2).max(),
                     np.abs(F[..., 26] - exact2).max()))
        assert not edge.any()
    for k in range(3):                 # second order including the wrapped cells
        assert errs[1][k] < errs[0][k] / 3.5, (k, errs)


# ------------------------------------------------------------------ closure moments

def test_closure_H_contracts_to_q():
    q = np.array([0.37, -1.2])
    H = oracle.closure_H(q)
    # heat-flux vector of Sec. 6.3: h = (H111 + H122, H112 + H222) / 2
    assert 0.5 * (H[0] + H[2]) == pytest.approx(q[0], rel=1e-15)
    assert 0.5 * (H[1] + H[3]) == pytest.approx(q[1], rel=1e-15)
    # isotropic (Grad) form: H111 = 3 H122, H222 = 3 H112
    assert H[0] == pytest.approx(3 * H[2]) and H[3] == pytest.approx(3 * H[1])
    assert np.array_equal(oracle.closure_H(q, np.zeros(2)), H)


def test_closure_H_is_inverted_by_contractions_and_traceless_part():
    """Any symmetric 2D third-order tensor (four free components) is rebuilt from its
    contraction q and its traceless combinations t: the map is one to one."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        Hin = rng.normal(size=4)                 # (H111, H112, H122, H222)
        q = 0.5 * np.array([Hin[0] + Hin[2], Hin[1] + Hin[3]])
        t = np.array([Hin[0] - 3 * Hin[2], 3 * Hin[1] - Hin[3]])
        assert np.allclose(oracle.closure_H(q, t), Hin, rtol=0, atol=1e-14)
    # the traceless part alone has zero contraction
    Ht = oracle.closure_H(np.zeros(2), np.array([0.8, -0.3]))
    assert abs(Ht[0] + Ht[2]) < 1e-16 and abs(Ht[1] + Ht[3]) < 1e-16


@pytest.mark.parametrize("proj,with_t", [("discrete", False), ("paper", False), ("discrete", True),
                                         ("paper", True)])
def test_closure_grec_moments(proj, with_t):
    """The rebuilt micro part has the requested stress deviation, heat flux and traceless
    third moments and no conserved moments (fine, wide velocity grid so quadrature
    errors are negligible)."""
    p = _problem(nx=2, ny=2, nv=96, V=11.0, proj_mode=proj)
    q = W.conserved2d(np.array(1.3), np.array(0.2), np.array(-0.15), np.array(0.9)).reshape(-1)
    qt = np.array([0.4, -0.25])
    St = np.array([0.3, -0.12, -0.2])          # not traceless: its traceless part is used
    tt = np.array([0.35, -0.6]) if with_t else None
    g = oracle.closure_grec(p, q, qt, St, tt).reshape(p["nv2"], p["nv1"])
    v1 = W.centres(*p["v1"], p["nv1"])
    v2 = W.centres(*p["v2"], p["nv2"])
    V1, V2 = np.meshgrid(v1, v2)
    dv = (v1[1] - v1[0]) * (v2[1] - v2[0])
    rho, u1, u2 = 1.3, 0.2, -0.15
    w1, w2 = V1 - u1, V2 - u2
    m = lambda f: dv * np.sum(f * g)  # noqa: E731
    cons = [m(1.0), m(V1), m(V2), m(V1 ** 2 + V2 ** 2)]
    tol_c = 1e-13 if proj == "discrete" else 1e-9
    assert np.max(np.abs(cons)) <= tol_c * dv * np.abs(g).sum() / dv
    tr = 0.5 * (St[0] + St[2])
    assert m(w1 * w1) == pytest.approx(St[0] - tr, abs=1e-10)
    assert m(w1 * w2) == pytest.approx(St[1], abs=1e-10)
    assert m(w2 * w2) == pytest.approx(St[2] - tr, abs=1e-10)
    ww = w1 ** 2 + w2 ** 2
    assert 0.5 * m(w1 * ww) == pytest.approx(qt[0], abs=1e-10)
    assert 0.5 * m(w2 * ww) == pytest.approx(qt[1], abs=1e-10)
    # third central moments: the H of the closure, divided by eps
    H = oracle.closure_H(qt, tt)
    H3 = [m(w1 ** 3), m(w1 ** 2 * w2), m(w1 * w2 ** 2), m(w2 ** 3)]
    assert np.allclose(H3, H, atol=1e-10)
    t_exp = tt if with_t else np.zeros(2)
    assert H3[0] - 3 * H3[2] == pytest.approx(t_exp[0], abs=1e-10)
    assert 3 * H3[1] - H3[3] == pytest.approx(t_exp[1], abs=1e-10)


def test_nsf_closure_matches_moments_of_first_order_micro_part():
    """(q, S) / eps of the NSF closure equal the heat flux and stress of the oracle's G-hat
    (eqn5-97, evaluated independently) for smooth fields on a fine velocity grid."""
    p = _problem(nx=8, ny=8, nv=80, V=10.0, bc=W.periodic2d(), eps=0.05, nu=-0.5)
    x = W.centres(*p["x"], 8)
    X, Y = np.meshgrid(x, x)
    s = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    c = np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    Q = W.conserved2d(1.0 + 0.1 * s, 0.1 * c, 0.05 * s, 1.0 + 0.1 * c)
    Qf = Q.reshape(-1, 6).copy()
    # an anisotropic pressure deviation so the ES term contributes
    Qf[:, 3] += 0.01 * s.ravel()
    Qf[:, 5] -= 0.01 * s.ravel()
    Qf[:, 4] += 0.004 * c.ravel()
    Gh = oracle.ghat2d(p, Qf.reshape(-1)).reshape(64, p["nv2"], p["nv1"])
    F, kn, edge = oracle.features2d(p, Qf.reshape(-1))
    v1 = W.centres(*p["v1"], p["nv1"])
    V1, V2 = np.meshgrid(v1, v1)
    dv = (v1[1] - v1[0]) ** 2
    for cell in (0, 9, 27, 45, 63):
        f = F[cell]
        qt, St, tt = oracle.nsf_closure(p, f)
        w1, w2 = V1 - f[1], V2 - f[2]
        ww = w1 ** 2 + w2 ** 2
        g = Gh[cell]
        assert 0.5 * dv * np.sum(w1 * ww * g) == pytest.approx(qt[0], rel=1e-8, abs=1e-9)
        assert 0.5 * dv * np.sum(w2 * ww * g) == pytest.approx(qt[1], rel=1e-8, abs=1e-9)
        assert dv * np.sum(w1 * w1 * g) == pytest.approx(St[0], rel=1e-8, abs=1e-9)
        assert dv * np.sum(w1 * w2 * g) == pytest.approx(St[1], rel=1e-8, abs=1e-9)
        assert dv * np.sum(w2 * w2 * g) == pytest.approx(St[2], rel=1e-8, abs=1e-9)
        # G-hat's third central moments are of the isotropic form: its traceless part is 0
        h111, h112 = dv * np.sum(w1 ** 3 * g), dv * np.sum(w1 * w1 * w2 * g)
        h122, h222 = dv * np.sum(w1 * w2 * w2 * g), dv * np.sum(w2 ** 3 * g)
        scale = 1e-8 * (abs(h111) + abs(h122) + abs(h112) + abs(h222)) + 1e-9
        assert abs(h111 - 3 * h122 - tt[0]) <= scale
        assert abs(3 * h112 - h222 - tt[1]) <= scale
