"""The C-ABI library: it loads without a GPU, exports every entry point the
header declares, and rejects invalid input before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import mm_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_four_core_calls():
    d = _declared()
    for name in ("mm_init", "mm_step", "mm_moments", "mm_free"):
        assert name in d


def test_library_exports_every_declared_symbol():
    from paper_2509_21832_amd import binding as B
    lib = C.CDLL(B.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(B.EXPORTS)


def test_binding_sizes_match_the_header():
    """The closure network's sizes in the binding are the header's."""
    import re
    from paper_2509_21832_amd import binding as B
    text = open(os.path.join(ROOT, "include", "mm.h")).read()
    val = {k: int(re.search(rf"#define {k} (\d+)", text).group(1))
           for k in ("MM_MLP_NPARAM", "MM_MLP_NNORM", "MM_NOALLOC_MAX_CELLS")}
    assert B.MLP_NPARAM == val["MM_MLP_NPARAM"] and B.MLP_NNORM == val["MM_MLP_NNORM"]
    assert B.NOALLOC_MAX_CELLS == val["MM_NOALLOC_MAX_CELLS"]
    assert B.MLP_NPARAM == 64 * B.N_FEAT + 64 + 64 * 64 + 64 + B.N_OUT * 64 + B.N_OUT
    assert B.MLP_NNORM == 2 * B.N_FEAT + 2 * B.N_OUT


def test_dt_rule_matches_oracle():
    import oracle
    from paper_2509_21832_amd import binding as B
    for p in (W.sod1d()[0], W.quadrant2d()[0], W.cavity2d(nx=256)[0], W.blast2d()[0]):
        assert B.dt(p)[0] == oracle.dt(p)[0]
        assert B.dt(p, 0.37) == oracle.dt(p, 0.37)
    p = W.quadrant2d()[0]
    p["cfl_rule"] = "sum"
    assert B.dt(p)[0] == oracle.dt(p)[0]


@pytest.mark.parametrize("field,value", [("eps", 0.0), ("eps", -1.0), ("cfl", 0.0), ("nu", 1.0), ("nu", -1.5),
                                         ("nx", 1), ("nv1", 1), ("tau_coef", 0.0)])
def test_invalid_config_rejected(field, value):
    from paper_2509_21832_amd import binding as B
    p, Q, G = W.quadrant2d(nx=4, ny=4, nv=4)
    p[field] = value
    Q = np.tile(Q.reshape(-1, 6)[0], p["nx"] * p["ny"])     # a valid state of the (possibly bad) size
    with pytest.raises(B.MMError) as e:
        B.Solver(p, Q)
    assert e.value.code == B.MM_EINVAL


def test_unpaired_periodic_and_1d_inflow_rejected():
    from paper_2509_21832_amd import binding as B
    p, Q, G = W.quadrant2d(nx=4, ny=4, nv=4)
    p["bc"] = [{"kind": "periodic"}, {"kind": "wall"}, {"kind": "wall"}, {"kind": "wall"}]
    with pytest.raises(B.MMError) as e:
        B.Solver(p, Q)
    assert e.value.code == B.MM_EINVAL
    p1, Q1, G1 = W.sod1d(nx=8, nv=8)
    p1["bc"][0] = {"kind": "inflow"}
    with pytest.raises(B.MMError) as e:
        B.Solver(p1, Q1)
    assert e.value.code == B.MM_EINVAL
    p1["bc"][0] = {"kind": "wall", "T_wall": 0.0}
    with pytest.raises(B.MMError) as e:
        B.Solver(p1, Q1)
    assert e.value.code == B.MM_EINVAL


@pytest.mark.parametrize("what", ["rho", "T", "es_det", "cold"])
def test_nonphysical_initial_state_rejected(what):
    from paper_2509_21832_amd import binding as B
    p, Q, G = W.quadrant2d(nx=4, ny=4, nv=4, nu=-1.0)
    Q = Q.copy()
    if what == "rho":
        Q[1, 2, 0] = -0.1
    elif what == "T":
        Q[0, 0, 3] = Q[0, 0, 1] ** 2 / Q[0, 0, 0] - 0.5
        Q[0, 0, 5] = Q[0, 0, 2] ** 2 / Q[0, 0, 0] - 0.5
    elif what == "cold":
        # T = 1e-3 on a velocity grid of half-width 8: the Maxwellian's exponent
        # reaches about 6e4 at the grid corners, beyond the solver's range rule
        rho = Q[1, 1, 0]
        u1, u2 = Q[1, 1, 1] / rho, Q[1, 1, 2] / rho
        Q[1, 1, 3] = rho * u1 * u1 + rho * 1e-3
        Q[1, 1, 5] = rho * u2 * u2 + rho * 1e-3
        Q[1, 1, 4] = rho * u1 * u2
    else:
        # P11 > 0 and P22 > 0 but nu = -1 makes calT = 2 T I - TT singular when P12^2 >= ...
        rho = Q[2, 2, 0]
        u1, u2 = Q[2, 2, 1] / rho, Q[2, 2, 2] / rho
        Q[2, 2, 3] = rho * u1 * u1 + 1.0
        Q[2, 2, 5] = rho * u2 * u2 + 1.0
        Q[2, 2, 4] = rho * u1 * u2 + 1.0
    with pytest.raises(B.NonPhysical):
        B.Solver(p, Q)
