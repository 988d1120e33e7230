"""The 1D step against the printed convergence study of the manufactured
solution (Sec. 3.4, Table tab5-2; fixture tests/golden/mms1d_tab5_2.json).

The micro errors are pinned to the printed digits within 5% at every N; the
printed log2 error ratios are pinned within 0.1 in both columns.  The macro
errors follow the printed ones with one fixed factor (1.30-1.33 here, the same
at every N): the section does not fix enough of the run to place the leading
error constant of the momentum component, which dominates that column, so the
macro digits are only pinned up to that constant factor (no GPU)."""
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

