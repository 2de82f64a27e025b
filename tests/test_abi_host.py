"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol the header declares, validates its inputs, and its host topology
agrees exactly with the oracle's classification."""

import os
import re

import numpy as np
import pytest

import synth
from oracle import fem
from oracle.topology import classify

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bddc.h")

P = pytest.importorskip("paper_0911_5730_amd")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const char\*|void|bddc_status)\s+(bddc_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    import ctypes
    lib = P.load_library()
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert isinstance(ctypes.CDLL(P.bddc.LIB_PATH).bddc_status_string, object)


def test_tuning_entry_points_validate_without_a_device():
    import ctypes
    lib = P.load_library()
    t = P.bddc.BddcTuningC()
    assert lib.bddc_get_tuning(None, ctypes.byref(t)) == -1
    assert lib.bddc_set_tuning(None, ctypes.byref(t)) == -1
    assert lib.bddc_autotune(None, None, None, 1, 1, 1e-8, 1, None, None) == -1


def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert P.status_string(code) != "unknown status"
    assert P.status_string(-99) == "unknown status"


def _oracle_counts(prob):
    dofs = fem.element_dofs(prob.nx, prob.ny, prob.element)
    elems = [(d[d >= 0], None) for d in dofs]
    touches = (dofs < 0).any(axis=1)
    top = classify(prob.n_free, elems, prob.part, prob.nsub, ~touches)
    return dict(n_interface=int((~top.interior).sum()), n_corners=len(top.corners),
                n_edges=len(top.edges))


@pytest.mark.parametrize("case", [
    dict(nx=32, nsx=4),
    dict(nx=18, nsx=4),                       # ragged blocks
    dict(nx=20, ny=12, nsx=5, nsy=3),         # rectangular mesh and partition
    dict(nx=256, nsx=16),                     # config-2 partition
    dict(nx=12, nsx=1),                       # a single substructure
])
def test_plan_topology_matches_oracle(case):
    prob = synth.square_problem(case["nx"], case["nsx"], ny=case.get("ny"), nsy=case.get("nsy"))
    got = P.plan(prob)
    want = _oracle_counts(prob)
    assert got["n_free"] == prob.n_free
    for k, v in want.items():
        assert got[k] == v, (k, got[k], v)


@pytest.mark.parametrize("case", [dict(nx=24, nsx=3), dict(nx=26, nsx=4), dict(nx=20, ny=12, nsx=5, nsy=3)])
def test_plan_topology_matches_oracle_elasticity(case):
    """Plane elasticity: two dofs per free node (2 f + c); the host's dof
    topology (node classes expanded to both components) against the oracle's
    classification of the elasticity element dofs."""
    prob = synth.square_problem(case["nx"], case["nsx"], ny=case.get("ny"), nsy=case.get("nsy"), element="Q1E")
    got = P.plan(prob)
    want = _oracle_counts(prob)
    assert got["n_free"] == prob.n_free == 2 * (prob.nx - 1) * (prob.ny - 1)
    for k, v in want.items():
        assert got[k] == v, (k, got[k], v)


def test_plan_promotes_corner_for_island():
    nx = 12
    prob = synth.square_problem(nx, 1)
    part = np.zeros((nx, nx), dtype=np.int32)
    part[3:9, 3:9] = 1
    prob.part = part.reshape(-1)
    prob.nsub = 2
    got = P.plan(prob)
    want = _oracle_counts(prob)
    assert got["n_corners"] == want["n_corners"] == 1
    assert got["n_edges"] == want["n_edges"] == 1


def _expect(code, prob, **kw):
    with pytest.raises(P.BDDCError) as ei:
        P.plan(prob, **kw)
    assert ei.value.name == code


def test_validation_errors():
    base = synth.config(1)
    bad = synth.config(1)
    bad.coeff = bad.coeff.copy()
    bad.coeff[5] = 0.0
    _expect("BDDC_EINVAL", bad)
    bad.coeff[5] = np.nan
    _expect("BDDC_EINVAL", bad)
    bad = synth.config(1)
    bad.part = bad.part.copy()
    bad.part[0] = 16
    _expect("BDDC_EPARTITION", bad)
    bad = synth.config(1)
    bad.nsub = 17                                       # substructure 16 owns nothing
    _expect("BDDC_EPARTITION", bad)
    bad = synth.config(1)
    bad.levels = 1
    _expect("BDDC_EINVAL", bad)
    bad = synth.config(1)
    bad.levels = 3
    bad.agglom = []
    _expect("BDDC_EINVAL", bad)
    _expect("BDDC_EINVAL", base, precision=7)
    for prec in ("fp32", "bf16"):
        assert P.plan(base, precision=prec)["n_corners"] == 9
    bad = synth.config(1)
    bad.nx = 1
    _expect("BDDC_EINVAL", bad)
    assert P.plan(base)["n_corners"] == 9


def _random_partition(nx, nsub, seed):
    """Irregular partition: each element takes the part of its nearest seed point."""
    rng = np.random.default_rng(seed)
    pts = rng.random((nsub, 2))
    c = (np.arange(nx) + 0.5) / nx
    X, Y = np.meshgrid(c, c)
    d = (X.reshape(-1, 1) - pts[:, 0]) ** 2 + (Y.reshape(-1, 1) - pts[:, 1]) ** 2
    part = np.argmin(d, axis=1).astype(np.int32)
    used = np.unique(part)
    remap = np.full(nsub, -1, dtype=np.int32)
    remap[used] = np.arange(used.size, dtype=np.int32)
    return remap[part], int(used.size)


@pytest.mark.parametrize("nx,nsub,seed", [(24, 9, 1), (40, 23, 2), (17, 6, 3), (64, 50, 4)])
def test_grid_and_element_list_classifications_agree(nx, nsub, seed, monkeypatch):
    """Level 1 is classified node by node on the grid; the general
    element-list classification (used at levels >= 2) must give the same
    topology, and both must match the oracle, on irregular partitions."""
    prob = synth.square_problem(nx, 1)
    prob.part, prob.nsub = _random_partition(nx, nsub, seed)
    grid = P.plan(prob)
    monkeypatch.setenv("BDDC_CLASSIFY", "elements")
    general = P.plan(prob)
    for k in ("n_free", "nsub", "n_dof", "n_interface", "n_corners", "n_edges"):
        assert grid[k] == general[k], (k, grid[k], general[k])
    want = _oracle_counts(prob)
    for k, v in want.items():
        assert grid[k] == v, (k, grid[k], v)


def test_plan_paper_elasticity_topology():
    """Host-only plan of the paper's experiment (768 x 768 elasticity, 48 x 48
    substructures, one jagged edge per level): the edge count is Table 1's
    (13818 - 4794 = 2 x 4512 edge averages), the corners are the interior cross
    points with both components, and the jagged edge adds two interface nodes
    per one-element tooth (fourteen teeth)."""
    p = synth.paper_elasticity_problem(768, 48, levels=3, groups=3, constraints="adaptive", tau=3.0)
    info = P.plan(p)
    assert info["n_free"] == 2 * 767 * 767
    assert info["nsub"] == 48 * 48 and info["levels"] == 3
    assert info["n_edges"] == 2 * 48 * 47 == 4512
    assert info["n_corners"] == 2 * 47 * 47
    straight_nodes = 2 * 47 * 767 - 47 * 47
    assert info["n_interface"] == 2 * (straight_nodes + 2 * 14)
