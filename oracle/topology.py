"""Oracle: substructure topology at one level (plain Python/NumPy).

TEST INFRASTRUCTURE ONLY (see oracle/fem.py).

The same classification is used at every level (Section 2 and Section 2.1):
level-l elements carry level-l dofs; level-l substructures are sets of
elements.  For each dof d, N_d is the set of substructures whose elements
touch d.

Reading of the paper (it assumes a conforming triangulation and only asks for
"sufficient" corners, Section 5):
  * interface dofs: |N_d| >= 2; interior dofs: |N_d| = 1;
  * corner: every dof with |N_d| >= 3;
  * edge of the adjacent pair (s, t): all dofs with N_d = {s, t};
  * if s or t floats (has no Dirichlet contact) and s, t share no corner,
    the lowest-index dof of their edge becomes a corner;
  * a floating substructure with no corner at all promotes the lowest-index
    dof of its largest edge (ties: the smaller pair).
On square partitions with at least two elements per substructure side the two
promotion rules never fire.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np


@dataclass
class Topology:
    n: int
    N: List[Tuple[int, ...]]                 # substructures touching each dof
    local: List[np.ndarray]                  # sorted global dofs of each substructure
    interior: np.ndarray                     # bool per dof
    corners: np.ndarray                      # sorted corner dofs
    edges: Dict[Tuple[int, int], np.ndarray] # (s, t), s < t -> sorted edge dofs
    sub_floating: np.ndarray                 # bool per substructure


def classify(n: int, elems, elem_sub: np.ndarray, nsub: int,
             elem_floating: np.ndarray) -> Topology:
    sets = [set() for _ in range(n)]
    local_sets = [set() for _ in range(nsub)]
    floating = np.ones(nsub, dtype=bool)
    for e, (dofs, _) in enumerate(elems):
        s = int(elem_sub[e])
        if not elem_floating[e]:
            floating[s] = False
        for d in dofs:
            sets[int(d)].add(s)
            local_sets[s].add(int(d))
    N = [tuple(sorted(x)) for x in sets]
    local = [np.array(sorted(x), dtype=np.int64) for x in local_sets]
    interior = np.array([len(x) == 1 for x in N], dtype=bool)

    corner_set = {d for d in range(n) if len(N[d]) >= 3}
    edge_lists: Dict[Tuple[int, int], list] = {}
    for d in range(n):
        if len(N[d]) == 2:
            edge_lists.setdefault(N[d], []).append(d)

    # a pair with a floating member must share at least one corner
    covered = set()
    for c in corner_set:
        for a in N[c]:
            for b in N[c]:
                if a < b:
                    covered.add((a, b))
    for key in sorted(edge_lists):
        s, t = key
        if not (floating[s] or floating[t]) or not edge_lists[key]:
            continue
        if key not in covered:
            d = min(edge_lists[key])
            corner_set.add(d)
            covered.add(key)
            edge_lists[key].remove(d)

    # a floating substructure must own at least one corner
    for s in range(nsub):
        if not floating[s]:
            continue
        if any(s in N[c] for c in corner_set):
            continue
        cand = [(-len(v), k) for k, v in edge_lists.items() if s in k and v]
        if not cand:
            raise ValueError(f"floating substructure {s} has no interface")
        _, key = min(cand)
        d = min(edge_lists[key])
        corner_set.add(d)
        edge_lists[key].remove(d)

    edges = {k: np.array(sorted(v), dtype=np.int64) for k, v in sorted(edge_lists.items()) if v}
    corners = np.array(sorted(corner_set), dtype=np.int64)
    return Topology(n=n, N=N, local=local, interior=interior, corners=corners,
                    edges=edges, sub_floating=floating)
