"""GPU FP64 path vs the oracle, element by element, through the C ABI."""
import numpy as np
import pytest

import mm_workloads as W
import oracle
from gpu_common import log, parity, rel_l1, run_gpu

pytestmark = pytest.mark.gpu


def _inflow_box(seed=0):
    b = [{"kind": "inflow", "rho": 1.2, "u1": 0.3, "u2": 0.05, "T": 1.1}, {"kind": "extrap"},
         {"kind": "wall", "T_wall": 0.9}, {"kind": "wall", "T_wall": 1.2, "u_wall": -0.15}]
    return W.smooth2d(seed=seed, nx=14, ny=9, nv=12, eps=0.07, bc=b)


def _nonsquare_v():
    """nv1 != nv2 and different velocity boxes: catches a swapped k/l index."""
    p, Q, G = W.quadrant2d(seed=2, nx=9, ny=12, nv=12, eps=0.03)
    p["nv2"], p["v2"] = 9, (-6.0, 6.0)
    return p, Q, W.zero_g(p)


SMALL = {
    # ragged sizes, every boundary kind, both projector modes, several nu
    "walls_quadrant": lambda: W.quadrant2d(seed=1, nx=13, ny=11, nv=10, eps=0.1),
    "walls_nonsquare_v": lambda: _nonsquare_v(),
    "lid_cavity": lambda: W.cavity2d(seed=3, nx=17, ny=10, nv=14, eps=0.02, amp=0.2),
    "periodic_smooth": lambda: W.smooth2d(seed=4, nx=12, ny=10, nv=16, eps=0.05),
    "periodic_paper_proj": lambda: W.smooth2d(seed=5, nx=10, ny=12, nv=13, eps=0.2, proj_mode="paper"),
    "extrap_nu_minus1": lambda: W.smooth2d(seed=6, nx=11, ny=8, nv=12, eps=0.01, bc=W.extrap2d(), nu=-1.0),
    "extrap_bgk_nu0": lambda: W.smooth2d(seed=7, nx=8, ny=11, nv=11, eps=1.0, bc=W.extrap2d(), nu=0.0),
    "inflow_mixed_sides": lambda: _inflow_box(8),
    "walls_no_es_term": lambda: W.quadrant2d(seed=9, nx=10, ny=10, nv=10, eps=0.1, wall_es_term=False),
    "walls_paper_proj": lambda: W.cavity2d(seed=10, nx=12, ny=12, nv=12, eps=0.05, amp=0.2, proj_mode="paper"),
    "tiny_2x2": lambda: W.smooth2d(seed=11, nx=2, ny=2, nv=4, eps=0.3),
    "small_eps": lambda: W.cavity2d(seed=12, nx=10, ny=9, nv=16, eps=1e-3, amp=0.1),
    "tau_p_model": lambda: W.quadrant2d(seed=13, nx=8, ny=8, nv=12, eps=0.05, tau_model="p", tau_coef=1.0),
}


def _v2_box(case, lo, hi):
    """The same case on an asymmetric v2 box (the pass's general y-upwind form)."""
    p, Q, G = case
    p["v2"] = (lo, hi)
    return p, Q, G


def _velocity(gen, nv1, nv2, V1=8.0, V2=8.0):
    """A generated problem on another velocity grid (g starts at zero)."""
    p, Q, _ = gen()
    p["nv1"], p["nv2"], p["v1"], p["v2"] = nv1, nv2, (-V1, V1), (-V2, V2)
    return p, Q, W.zero_g(p)


# velocity grids the lane-k kernel takes (nv1 divides 64): one to sixteen
# nodes per lane, one wavefront per SIMD (FP64) and the chunked FP32 form at
# 1024 nodes per cell; ragged spatial sizes with several row segments
LANE_K = {
    "lk_8x8_periodic": lambda: _velocity(lambda: W.smooth2d(seed=20, nx=13, ny=11, eps=0.05), 8, 8),
    "lk_2x32_extrap": lambda: _velocity(lambda: W.smooth2d(seed=21, nx=7, ny=9, eps=0.2, bc=W.extrap2d()),
                                        2, 32, V1=6.0),
    "lk_16x8_walls": lambda: _velocity(lambda: W.quadrant2d(seed=22, nx=11, ny=9, eps=0.1), 16, 8),
    "lk_4x64_inflow": lambda: _velocity(lambda: _inflow_box(23), 4, 64, V1=5.0, V2=9.0),
    "lk_32x32_cavity": lambda: W.cavity2d(seed=24, nx=9, ny=37, nv=32, eps=0.02, amp=0.2),
    "lk_64x16_walls": lambda: _velocity(lambda: W.quadrant2d(seed=25, nx=6, ny=19, eps=0.03), 64, 16,
                                        V1=9.0, V2=7.0),
    "lk_32x16_paper_proj": lambda: _velocity(
        lambda: W.smooth2d(seed=26, nx=10, ny=18, eps=0.1, proj_mode="paper"), 32, 16),
    # an asymmetric v2 box: the y-upwind direction is decided per node at run time
    "lk_32x32_asym_v2": lambda: _asym_v2(),
    # nu = -1 (the paper's value for its 2D studies): the ES tensor 2T I - P/rho at the
    # edge of admissibility, on a periodic box
    "lk_32x32_nu_minus1": lambda: W.smooth2d(seed=28, nx=10, ny=11, nv=32, V=6.0, eps=0.08, nu=-1.0),
    # a small Knudsen number: the ES term (calG - M)/eps is amplified most
    "lk_32x32_eps_1e-4": lambda: W.cavity2d(seed=29, nx=9, ny=13, nv=32, eps=1e-4, amp=0.1),
}


# 48 active lanes (nv1 = 24 or 48; 16 idle lanes): 12 nodes per lane in both precisions,
# 48 nodes per lane with g in FP32 (the 512^2 x 48^2 blast's velocity grid)
LANE_K48 = {
    "lk48_24x24_walls": (lambda: _velocity(lambda: W.quadrant2d(seed=30, nx=11, ny=13, eps=0.05), 24, 24),
                         ("fp64", "mixed")),
    "lk48_24x24_asym_periodic": (lambda: _velocity(lambda: W.smooth2d(seed=31, nx=9, ny=10, eps=0.1), 24, 24,
                                                   V1=7.0, V2=5.0), ("fp64", "mixed")),
    "lk48_48x48_blast": (lambda: W.blast2d(seed=32, nx=18, ny=15, eps=0.02, sigma=0.2), ("fp64", "mixed")),
    "lk48_48x48_lid_paper_proj": (lambda: W.cavity2d(seed=33, nx=10, ny=17, nv=48, V=8.0, eps=0.05, amp=0.2,
                                                     proj_mode="paper"), ("fp64", "mixed")),
    "lk48_48x48_asym_v2": (lambda: _v2_box(_velocity(lambda: W.blast2d(seed=35, nx=12, ny=11, eps=0.03,
                                                                        sigma=0.2), 48, 48), -7.0, 8.0),
                           ("fp64", "mixed")),
    "lk48_48x24_inflow": (lambda: _velocity(lambda: _inflow_box(34), 48, 24, V1=9.0, V2=6.0), ("fp64", "mixed")),
}


@pytest.mark.parametrize("name,precision", [(n, pr) for n in sorted(LANE_K48) for pr in LANE_K48[n][1]])
def test_lane_k_48_lanes(name, precision):
    """The lane-k kernel with 48 active lanes on its velocity grids, against the oracle
    (walls go through the wall-ring kernel of the same layout)."""
    p, Q, G = LANE_K48[name][0]()
    p["precision"] = precision
    parity(p, Q, G, 20, label=f"{name}_{precision}")


def _asym_v2():
    p, Q, G = W.cavity2d(seed=27, nx=9, ny=21, nv=32, eps=0.05, amp=0.2)
    p["v2"] = (-6.0, 8.0)
    return p, Q, W.zero_g(p)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", sorted(LANE_K))
def test_lane_k_2d(name, precision):
    """The lane-k fused kernel on its whole range of velocity grids."""
    p, Q, G = LANE_K[name]()
    p["precision"] = precision
    parity(p, Q, G, 25, label=f"{name}_{precision}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["lk_32x32_cavity", "lk_32x32_asym_v2"])
def test_lane_k_2d_bitwise_repeatable(name, precision):
    """Two runs of the same case give the same bits (every reduction in the
    step has a fixed order, so any difference is a defect of the kernel)."""
    from paper_2509_21832_amd import binding as B
    p, Q, G = LANE_K[name]()
    p["precision"] = precision
    out = []
    for _ in range(2):
        with B.Solver(p, Q, G) as s:
            s.step(25)
            out.append((s.moments(), s.get_g()))
    log(f"repeat {name} {precision}")
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["lk_32x32_cavity", "lk_16x8_walls", "lk_4x64_inflow"])
def test_generic_fused_on_lane_k_shapes(name, precision):
    """The generic fused kernel, forced where the lane-k kernel would run."""
    p, Q, G = LANE_K[name]()
    p["precision"] = precision
    parity(p, Q, G, 25, label=f"{name}_{precision}_generic", generic=True)


@pytest.mark.parametrize("name", sorted(SMALL))
def test_small_2d(name):
    """The launch configuration of the benchmark: fused phase-space pass."""
    p, Q, G = SMALL[name]()
    parity(p, Q, G, 30, label=name)


@pytest.mark.parametrize("name", ["walls_quadrant", "lid_cavity", "periodic_paper_proj", "inflow_mixed_sides",
                                  "extrap_nu_minus1", "walls_nonsquare_v"])
def test_small_2d_reference_pass(name):
    """The unfused phase-space pass (one workgroup per cell), used for shapes the fused pass
    does not cover."""
    p, Q, G = SMALL[name]()
    parity(p, Q, G, 30, label=name + "_ref", reference=True)


@pytest.mark.parametrize("gen", ["walls", "periodic"])
@pytest.mark.parametrize("shape", [(520, 3), (3, 520)])
def test_long_lines_macro(shape, gen):
    """Lines of more than 512 cells along a sweep take the four-lanes-per-cell macro
    kernel; the other direction takes the one-workgroup-per-line kernel."""
    nx, ny = shape
    if gen == "walls":
        p, Q, G = W.quadrant2d(seed=16, nx=nx, ny=ny, nv=8, eps=0.1)
    else:
        p, Q, G = W.smooth2d(seed=17, nx=nx, ny=ny, nv=8, eps=0.05)
    parity(p, Q, G, 10, label=f"long_{gen}_{nx}x{ny}")


def test_large_velocity_grid_uses_reference_pass():
    """nv1 > 64 is outside the fused pass; the library falls back to the unfused pass."""
    p, Q, G = W.quadrant2d(seed=15, nx=6, ny=5, nv=12, eps=0.1)
    p["nv1"], p["v1"] = 72, (-9.0, 9.0)
    parity(p, Q, W.zero_g(p), 10, label="nv1_72")


@pytest.mark.parametrize("name", ["walls_quadrant", "lid_cavity", "periodic_smooth", "inflow_mixed_sides",
                                  "small_eps", "walls_paper_proj"])
def test_small_2d_mixed(name):
    """g stored in FP32: macro rel-L1 <= 1e-5 against the FP64 oracle."""
    p, Q, G = SMALL[name]()
    p["precision"] = "mixed"
    parity(p, Q, G, 30, label=name + "_mixed")


def test_small_2d_nonzero_g0():
    """Start from a micro part with nonzero (projected) values."""
    p, Q, G = W.smooth2d(seed=14, nx=9, ny=9, nv=12, eps=0.1)
    Qo, Go, Ho = oracle.run(p, Q.reshape(-1), G.reshape(-1), 5)     # a valid g from 5 oracle steps
    parity(p, Qo, Go, 20, label="nonzero_g0")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_generic_pass_padding_slots_add_nothing(precision):
    """The generic fused kernel pads a lane's last node slots when 64 does not divide nv
    (10 x 10 = 100 nodes in 128 slots).  On a small velocity box (|v| <= 3.5) the Maxwellian at
    every node is far from negligible, so a padding slot that carried a Maxwellian value into
    the G-hat moments or into H would show at once."""
    p, Q, G = W.smooth2d(seed=21, nx=10, ny=9, nv=10, V=3.5, eps=0.05)
    Qo, Go, Ho = oracle.run(p, Q.reshape(-1), G.reshape(-1), 3)     # a nonzero valid g
    p["precision"] = precision
    parity(p, Qo, Go, 12, label=f"padding_{precision}")


@pytest.mark.parametrize("bc,mode", [("extrap", "discrete"), ("periodic", "discrete"), ("periodic", "paper")])
def test_small_1d(bc, mode):
    p, Q, G = W.sod1d(nx=37, nv=20, eps=0.05, bc=bc, proj_mode=mode)
    parity(p, Q, G, 60, label=f"1d_{bc}_{mode}")


def test_c1_sod1d_full():
    """Config 1: Nx = 200, Nv = 64, eps = 1e-2, outflow, 100 steps."""
    p, Q, G = W.sod1d()
    parity(p, Q, G, 100, label="c1_full")


def test_c2_quadrant_full():
    """Config 2: 64^2 x 24^2 quadrant Riemann problem with walls, eps = 0.1, 200 steps (seed 0)."""
    p, Q, G = W.quadrant2d(seed=0)
    parity(p, Q, G, 200, label="c2_full", chunks=4)


@pytest.mark.parametrize("eps", [1e-3, 1.0])
def test_c3_full_one_step_all_outputs(eps):
    """Config 3 at full size (256^2 x 32^2): one step, every output element."""
    p, Q, G = W.cavity2d(seed=0, eps=eps)
    parity(p, Q, G, 1, label=f"c3_one_step_eps{eps:g}")


def test_c3_full_two_steps_from_nonzero_g():
    """Config 3 at full size from a developed state (g != 0, u != 0): the state after
    2 oracle steps is advanced 1 step by both sides."""
    p, Q, G = W.cavity2d(seed=1, eps=1e-2)
    Qo, Go, Ho = oracle.run(p, Q.reshape(-1), G.reshape(-1), 2)
    parity(p, Qo, Go, 1, label="c3_developed")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_c3_full_100_steps_vs_golden(precision, tol):
    """Config 3, 100 steps, every eps of its sweep (and 3e-3 of config 5): macro rel-L1
    against the oracle's stored result (tests/golden/make_c3_reference.py) on every 4th cell
    and, element by element, on the whole boundary ring (the lid and wall cells):
    <= 1e-12 in FP64, <= 1e-5 with g in FP32."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c3_cavity_100steps.npz")
    ref = np.load(path)
    st = int(ref["stride"])
    for eps in (1e-3, 3e-3, 1e-2, 1e-1, 1.0):
        key = f"eps{eps:g}"
        p, Q, G = W.cavity2d(seed=0, eps=eps)
        p["precision"] = precision
        log(f"[c3_100 {key} {precision}] start")
        Qg, Gg, Hg = run_gpu(p, Q, G, int(ref["steps"]), chunks=4)
        Qg = Qg.reshape(p["ny"], p["nx"], 6)
        e = rel_l1(Qg[::st, ::st, :], ref[key + "_sample"])
        sums = Qg.reshape(-1, 6).sum(0)
        es = np.abs(sums - ref[key + "_sum"]) / ref[key + "_abssum"]
        ring = np.concatenate([Qg[0], Qg[-1], Qg[:, 0], Qg[:, -1]])
        ring_ref = np.concatenate([ref[key + "_row_lo"], ref[key + "_row_hi"], ref[key + "_col_lo"],
                                   ref[key + "_col_hi"]])
        er = rel_l1(ring, ring_ref)
        emax = (np.abs(ring - ring_ref) / np.abs(ring_ref).max(axis=0)).max()
        log(f"[c3_100 {key} {precision}] sampled Q rel-L1 {e:.3e}; domain sums rel {es.max():.3e}; "
            f"boundary ring rel-L1 {er:.3e}, max per component {emax:.3e}")
        assert e <= tol
        assert es.max() <= tol
        assert er <= tol
        assert emax <= 10 * tol


def _c4_reference():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c4_blast_checkpoints.npz")
    return np.load(path)


def _c4_vs_golden(precision, tol_q, tol_g):
    from paper_2509_21832_amd import binding as B
    ref = _c4_reference()
    st = int(ref["stride"])
    p, Q, G = W.blast2d(seed=0)
    p["precision"] = precision
    cells = ref["g_cells"][:, 0] * p["nx"] + ref["g_cells"][:, 1]
    with B.Solver(p, Q, G) as s:
        done = 0
        for n in ref["steps"]:
            log(f"[c4 {precision}] to step {n}")
            s.step(int(n) - done)
            done = int(n)
            Qg = s.moments().reshape(p["ny"], p["nx"], 6)
            e = rel_l1(Qg[::st, ::st, :], ref[f"step{n}_sample"])
            sums = Qg.reshape(-1, 6).sum(0)
            es = np.abs(sums - ref[f"step{n}_sum"]) / ref[f"step{n}_abssum"]
            gg = s.get_g_cells(cells)
            gr = ref[f"step{n}_g"]
            ge = np.abs(gg - gr).max() / np.abs(gr).max()
            log(f"[c4 {precision} step {n}] sampled Q rel-L1 {e:.3e}; sums rel {es.max():.3e}; g max rel {ge:.3e}")
            assert e <= tol_q and es.max() <= tol_q
            assert ge <= tol_g


def test_c4_blast_mixed_vs_golden():
    """Config 4 at full size (512^2 x 48^2 = 604M points, g in FP32): macro state after 10 and
    100 steps against the oracle's stored result (tests/golden/make_c4_reference.py), sampled
    every 8th cell, domain sums over all cells, and g of 16 cells (corners, wall rows, blast core)."""
    _c4_vs_golden("mixed", 1e-5, 1e-4)


def test_c4_blast_fp64_vs_golden():
    """Config 4 at full size in FP64 (the lane-k pass with 48 nodes per lane): the same stored
    oracle result, to the FP64 bar."""
    _c4_vs_golden("fp64", 1e-12, 1e-10)


def test_c4_blast_mixed_500_steps_properties():
    """Config 4's full run (500 steps, g in FP32): no non-physical state, total mass conserved to
    round-off (diffuse walls have zero net mass flux), conserved moments of g zero to FP32 rounding."""
    from paper_2509_21832_amd import binding as B
    p, Q, G = W.blast2d(seed=0)
    p["precision"] = "mixed"
    with B.Solver(p, Q, G) as s:
        s.step(500)
        Qg, H, M = s.moments(with_h=True, with_gmom=True)
    Q0 = Q.reshape(-1, 6)
    Qg = Qg.reshape(-1, 6)
    M = M.reshape(-1, 7)
    dm = abs(Qg[:, 0].sum() - Q0[:, 0].sum()) / Q0[:, 0].sum()
    stress = np.abs(M[:, 4:7]).max() / p["eps"]
    cons = np.abs(M[:, 0:4]).max()
    log(f"[c4 500] mass drift {dm:.3e}; max |conserved g-moment| {cons:.3e} vs stress scale {stress:.3e}")
    assert np.all(np.isfinite(Qg)) and np.all(np.isfinite(H))
    assert dm <= 1e-12
    assert cons <= 1e-5 * stress
