"""Pins of the oracle's corner/edge classification (no GPU).

The paper's experiment (Section 6, Tables 1-2) counts coarse dofs on a
48 x 48 partition of a 768 x 768 mesh with a 3 x 3 partition at level 2.  Its
boundary conditions are not stated and its corner count includes substructure
vertices on the domain boundary (4794 / 2 = 49^2 - 4), while the model here
has zero Dirichlet data on the whole boundary; the edge counts do not depend
on that difference and are pinned exactly.
"""

import json
import os

import numpy as np
import pytest

import synth
from oracle import fem
from oracle.topology import classify

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _level1_topology(nx, ns):
    dofs = fem.element_dofs(nx, nx)
    elems = [(d[d >= 0], None) for d in dofs]
    touches = (dofs < 0).any(axis=1)
    part = synth.square_partition(nx, nx, ns, ns)
    return classify((nx - 1) ** 2, elems, part, ns * ns, ~touches)


def test_config1_counts():
    top = _level1_topology(32, 4)
    assert len(top.corners) == 9
    assert len(top.edges) == 24
    assert all(len(E) == 7 for E in top.edges.values())
    assert top.interior.sum() == 16 * 49
    assert top.sub_floating.sum() == 4          # the 2x2 block of inner substructures


@pytest.mark.slow
def test_paper_partition_edge_and_corner_counts():
    g = GOLD
    ns = g["experiment"]["level1_per_side"]
    dpn = g["experiment"]["dofs_per_node"]
    nx = ns * g["experiment"]["ratio"]
    top = _level1_topology(nx, ns)
    # Table 1: c+e adds one average per edge and per component
    n_edges_paper = (g["table1"]["ce"]["nc"] - g["table1"]["c"]["nc"]) // dpn
    assert len(top.edges) == n_edges_paper == 4512
    assert all(len(E) == 15 for E in top.edges.values())
    # Table 1 corner count = ours + vertices on the boundary shared by two substructures
    assert len(top.corners) + 4 * (ns - 1) == g["table1"]["c"]["nc"] // dpn

    # level 2: level-1 substructures are elements, level-1 corners are the dofs
    ns2 = g["experiment"]["level2_per_side"]
    cid = {int(c): k for k, c in enumerate(top.corners)}
    elems2 = []
    for s in range(ns * ns):
        loc = top.local[s]
        elems2.append((np.array([cid[int(d)] for d in loc if int(d) in cid]), None))
    agg = synth.square_agglomeration(ns, ns, ns2, ns2)
    top2 = classify(len(cid), elems2, agg, ns2 * ns2, top.sub_floating)
    n_edges2_paper = (g["table2"]["ce"]["nc2"] - g["table2"]["c"]["nc2"]) // dpn
    assert len(top2.edges) == n_edges2_paper == 12
    assert len(top2.corners) + 4 * (ns2 - 1) == g["table2"]["c"]["nc2"] // dpn


def test_corner_promotion_for_floating_pair_without_corner():
    # an island substructure inside another one: the pair shares a closed-loop
    # edge and no node with |N| >= 3, so the rule must promote one edge node
    nx = 12
    dofs = fem.element_dofs(nx, nx)
    elems = [(d[d >= 0], None) for d in dofs]
    touches = (dofs < 0).any(axis=1)
    part = np.zeros((nx, nx), dtype=np.int32)
    part[3:9, 3:9] = 1
    top = classify((nx - 1) ** 2, elems, part.reshape(-1), 2, ~touches)
    assert top.sub_floating.tolist() == [False, True]
    assert len(top.corners) == 1
    E = top.edges[(0, 1)]
    assert len(E) == 4 * 6 - 1
    assert top.corners[0] < E.min()
