"""The 1D and 2D steps against the printed convergence studies of the
manufactured solutions (Sec. 3.4, Table tab5-2, and Sec. 6.2, Table tab5-4;
fixtures tests/golden/mms1d_tab5_2.json and mms2d_tab5_4.json).

1D:

The micro errors are pinned to the printed digits within 5% at every N; the
printed log2 error ratios are pinned within 0.1 in both columns.  The macro
errors follow the printed ones with one fixed factor (1.30-1.33 here, the same
at every N): the section does not fix enough of the run to place the leading
error constant of the momentum component, which dominates that column, so the
macro digits are only pinned up to that constant factor.

2D: the table starts at 40^4 points, which the oracle runs in about 30 s; the
macro error there is pinned within 6% of the printed one and the micro error
within 35% (it is 1.30 times the printed one at N = 40 and 1.12 times at N = 80,
where the macro rate 40 -> 80 is 0.68 against the printed 0.67) (no GPU)."""
import json
import math
import os

import numpy as np
import pytest

import mm_workloads as W
import oracle

FIX = os.path.join(os.path.dirname(__file__), "golden", "mms1d_tab5_2.json")
NS = (10, 20, 40, 80, 160)


@pytest.fixture(scope="module")
def study():
    with open(FIX) as fh:
        gold = json.load(fh)
    printed = {n: (gold["macro"][i], gold["micro"][i]) for i, n in enumerate(gold["N"])}
    ours = {}
    for n in NS:
        p = W.problem1d(n, n, gold["V"], eps=gold["eps"], bc="periodic", cfl=gold["cfl"])
        ours[n] = oracle.mms1d(p, gold["t_final"])
    return printed, ours


def test_mms1d_micro_errors_match_printed(study):
    printed, ours = study
    for n in NS:
        assert ours[n][1] == pytest.approx(printed[n][1], rel=0.05), n


def test_mms1d_first_order_rates_match_printed(study):
    printed, ours = study
    for a, b in zip(NS[:-1], NS[1:]):
        for col in (0, 1):
            r_ours = math.log2(ours[a][col] / ours[b][col])
            r_paper = math.log2(printed[a][col] / printed[b][col])
            assert abs(r_ours - r_paper) < 0.1, (a, b, col, r_ours, r_paper)
    # the asymptotic order is one in both columns
    assert 0.9 < math.log2(ours[80][0] / ours[160][0]) < 1.05
    assert 0.9 < math.log2(ours[80][1] / ours[160][1]) < 1.05


def test_mms1d_macro_errors_one_constant_factor_from_printed(study):
    printed, ours = study
    ratios = np.array([ours[n][0] / printed[n][0] for n in NS])
    assert np.all((ratios > 1.0) & (ratios < 1.4)), ratios
    assert ratios.max() / ratios.min() < 1.03, ratios



FIX2 = os.path.join(os.path.dirname(__file__), "golden", "mms2d_tab5_4.json")


@pytest.fixture(scope="module")
def study2d():
    with open(FIX2) as fh:
        gold = json.load(fh)
    ours = {}
    for n in (20, 40):
        p = W.problem2d(n, n, n, n, gold["V"], eps=gold["eps"], cfl=gold["cfl"], nu=gold["nu"],
                        bc=W.periodic2d())
        ours[n] = oracle.mms2d(p, gold["t_final"])
    return gold, ours


def test_mms2d_errors_at_40_match_printed(study2d):
    gold, ours = study2d
    assert gold["N"][0] == 40
    assert ours[40][0] == pytest.approx(gold["macro"][0], rel=0.06)
    assert ours[40][1] == pytest.approx(gold["micro"][0], rel=0.35)


def test_mms2d_errors_decrease_with_resolution(study2d):
    _, ours = study2d
    assert ours[40][0] < 0.8 * ours[20][0]
    assert ours[40][1] < 0.8 * ours[20][1]


FIX2_N80 = os.path.join(os.path.dirname(__file__), "golden", "mms2d_n80.json")


def _oracle_sha():
    import hashlib
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "mm_oracle.c")
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def test_mms2d_rate_40_to_80_matches_printed(study2d):
    """The stored N = 80 run (tests/golden/make_mms2d_reference.py, oracle only)
    with the live N = 40 run: the macro rate 40 -> 80 is the printed one within
    0.05, and the N = 80 errors are the printed ones within 5% (macro) and 15%
    (micro)."""
    gold, ours = study2d
    with open(FIX2_N80) as fh:
        ref = json.load(fh)
    if ref["oracle_sha256"] != _oracle_sha():
        pytest.skip("the stored N = 80 run predates this oracle source: rerun "
                    "tests/golden/make_mms2d_reference.py")
    i80 = gold["N"].index(80)
    rate_ours = math.log2(ours[40][0] / ref["macro"])
    rate_paper = math.log2(gold["macro"][0] / gold["macro"][i80])
    assert abs(rate_ours - rate_paper) < 0.05, (rate_ours, rate_paper)
    assert ref["macro"] == pytest.approx(gold["macro"][i80], rel=0.05)
    assert ref["micro"] == pytest.approx(gold["micro"][i80], rel=0.15)
