"""Pins of the selection rule and the indicator against the paper's own tables.

These checks use only the tables' internal consistency (the oracle run on the
paper's own experiment is in test_oracle_paper_elasticity.py); they fix the
semantics:
  * Table 6 at tau = 10 adds 4805 - 4794 = 11 coarse dofs over 4512 edges,
    which rules out taking "up to and including the first eigenvalue <= tau"
    (that adds at least one dof per edge) and fits the strict rule lambda > tau;
  * omega-tilde of Table 7 (tau = 10) is the product of the level-1 value of
    Table 6 and the largest unselected level-2 eigenvalue of Table 5;
  * the level-1 value 8.67 of Table 6 is the largest unselected eigenvalue of
    Table 3 (8.7, printed to one decimal).
Printed values carry their rounding: a value printed with one decimal is
taken as an interval of half a unit of the last digit.
"""

import json
import os

import pytest

from oracle.adaptive import count_selected, indicator_from_tables

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _interval(x, decimals):
    h = 0.5 * 10.0 ** (-decimals)
    return x - h, x + h


def _pairs(table):
    return [lam for _, _, lam in G[table]["pairs"]]


def test_strict_selection_fits_table6_count():
    tau = 10.0
    added = G["table6"]["rows"][1]["nc"] - G["table6"]["rows"][0]["nc"]
    dpn = G["experiment"]["dofs_per_node"]
    ns = G["experiment"]["level1_per_side"]
    n_edges = 2 * ns * (ns - 1)                     # pinned against Table 1 elsewhere
    listed = sum(count_selected(lam, tau) for lam in _pairs("table3"))
    # strict rule: the listed pairs already account for all but a few of the added dofs
    assert listed <= added
    assert added - listed <= 8 * len(_pairs("table3"))
    # inclusive rule would add one dof per edge at least, per displacement component
    assert n_edges > added and n_edges * 1 > added // dpn


def test_indicator_three_level_tau10_is_product_of_level_maxima():
    tau = G["table5"]["tau"]
    lo1, hi1 = _interval(max(x for lam in _pairs("table3") for x in lam if not x > tau), 1)
    lo2, hi2 = _interval(max(x for lam in _pairs("table5") for x in lam if not x > tau), 1)
    omega3 = G["table7"]["rows"][1]["omega"]
    assert lo1 * lo2 <= omega3 <= hi1 * hi2
    # same through the oracle's indicator routine (point values)
    ind = indicator_from_tables([_pairs("table3"), _pairs("table5")], tau)
    assert abs(ind - omega3) <= (hi1 * hi2 - lo1 * lo2)
    # the level-1 factor is Table 6's omega-tilde at tau = 10
    om1 = G["table6"]["rows"][1]["omega"]
    assert lo1 <= om1 <= hi1
    assert abs(omega3 / om1 - 9.8) <= 0.05


def test_indicator_respects_theorem_bound_in_tables():
    # Theorem "adaptive": omega-tilde <= tau^(L-1)
    for row in G["table6"]["rows"][1:]:
        assert row["omega"] <= row["tau"]
    for row in G["table7"]["rows"][1:]:
        assert row["omega"] <= row["tau"] ** 2


@pytest.mark.parametrize("tau", [2.0, 10.0])
def test_listed_level2_pairs_lower_bound_reported_indicator(tau):
    table = "table4" if tau == 2.0 else "table5"
    row = [r for r in G["table7"]["rows"] if r["tau"] == tau][0]
    row2 = [r for r in G["table6"]["rows"] if r["tau"] == tau][0]
    lo2, _ = _interval(max(x for lam in _pairs(table) for x in lam if not x > tau), 1)
    # the listed pairs are a subset of all pairs: their maximum cannot exceed
    # the level-2 factor of the reported indicator (level 1 = Table 6)
    lo_om1, hi_om1 = _interval(row2["omega"], 2)
    _, hi3 = _interval(row["omega"], 2)
    assert lo2 <= hi3 / lo_om1
