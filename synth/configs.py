"""Seeded problem generators.

The model problem is scalar diffusion  -div(k grad u) = f  on the unit square
with zero Dirichlet data on the whole boundary, discretised on an nx x ny grid
of square (or rectangular) elements.  Element e = j*nx + i covers
[i/nx, (i+1)/nx] x [j/ny, (j+1)/ny].  Free node (i, j), 1 <= i <= nx-1,
1 <= j <= ny-1, has index (j-1)*(nx-1) + (i-1).

Every random draw goes through one numpy Generator(PCG64(seed)) in a fixed
order: coefficient, channels, partition seeds, right-hand side.

Workload shapes follow the numerical section of the paper (unit square,
H/h = 16, coarsening ratio 16 between levels, about a million unknowns at
the largest size); the paper's own experiment is elasticity on a jagged
partition whose geometry is not available, so these seeded scalar problems
stand in for it.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

CONSTRAINT_KINDS = ("corners", "corners_edges", "adaptive")


@dataclass
class Problem:
    nx: int
    ny: int
    coeff: np.ndarray            # float64, nx*ny, element-wise k_e > 0
    part: np.ndarray             # int32, nx*ny, level-1 substructure of each element
    nsub: int
    levels: int                  # L >= 2
    agglom: List[np.ndarray]     # agglom[l-2][s] = level-l substructure of level-(l-1) substructure s
    constraints: str = "corners"
    tau: float = float("inf")
    f: Optional[np.ndarray] = None   # float64 (nrhs, n_free) dual load vectors
    element: str = "Q1"
    rtol: float = 1e-8
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_free(self) -> int:
        return (2 if self.element == "Q1E" else 1) * (self.nx - 1) * (self.ny - 1)


def square_partition(nx: int, ny: int, nsx: int, nsy: int) -> np.ndarray:
    """Element -> substructure id for an nsx x nsy grid of rectangular blocks."""
    i = np.arange(nx)
    j = np.arange(ny)
    bi = (i * nsx) // nx
    bj = (j * nsy) // ny
    part = bj[:, None] * nsx + bi[None, :]
    return part.reshape(-1).astype(np.int32)


def square_agglomeration(nsx: int, nsy: int, gx: int, gy: int) -> np.ndarray:
    """Substructure (I, J) of an nsx x nsy grid -> group of a gx x gy grid."""
    I = np.arange(nsx)
    J = np.arange(nsy)
    gi = (I * gx) // nsx
    gj = (J * gy) // nsy
    return (gj[:, None] * gx + gi[None, :]).reshape(-1).astype(np.int32)


def add_channels(rng: np.random.Generator, nx: int, ny: int, coeff: np.ndarray,
                 count: int = 8, kval: float = 1e6) -> list:
    """Straight high-coefficient channels two elements wide across the domain.

    Each channel draws its orientation (0 = horizontal, 1 = vertical) and then
    an offset t in {0, ..., n-2}; rows (or columns) t and t+1 get k = kval.
    """
    k2 = coeff.reshape(ny, nx)
    drawn = []
    for _ in range(count):
        orient = int(rng.integers(0, 2))
        if orient == 0:
            t = int(rng.integers(0, ny - 1))
            k2[t:t + 2, :] = kval
        else:
            t = int(rng.integers(0, nx - 1))
            k2[:, t:t + 2] = kval
        drawn.append((orient, t))
    return drawn


def _levels_agglom(nsx, nsy, levels, groups):
    agg = []
    if levels >= 3:
        gx, gy = groups
        agg.append(square_agglomeration(nsx, nsy, gx, gy))
        cx, cy = gx, gy
        for _ in range(levels - 3):
            nx2, ny2 = max(1, cx // 4), max(1, cy // 4)
            agg.append(square_agglomeration(cx, cy, nx2, ny2))
            cx, cy = nx2, ny2
    return agg


def square_problem(nx: int, nsx: int, *, ny: Optional[int] = None, nsy: Optional[int] = None,
                   levels: int = 2, groups=(1, 1), constraints: str = "corners",
                   tau: float = float("inf"), kmode: str = "one", kmax_exp: float = 0.0,
                   channels: int = 0, nrhs: int = 1, seed: int = 0,
                   element: str = "Q1", name: str = "") -> Problem:
    """A seeded problem on a square partition.

    kmode: "one" (k = 1), "loguniform" (k = 10**U(0, kmax_exp) per element).
    groups: level-2 groups per side (gx, gy), used when levels >= 3.
    """
    ny = nx if ny is None else ny
    nsy = nsx if nsy is None else nsy
    assert constraints in CONSTRAINT_KINDS
    rng = np.random.Generator(np.random.PCG64(seed))
    if kmode == "one":
        coeff = np.ones(nx * ny)
    elif kmode == "loguniform":
        coeff = 10.0 ** rng.uniform(0.0, kmax_exp, size=nx * ny)
    else:
        raise ValueError(kmode)
    ch = add_channels(rng, nx, ny, coeff, count=channels) if channels else []
    part = square_partition(nx, ny, nsx, nsy)
    agg = _levels_agglom(nsx, nsy, levels, groups)
    nfree = (2 if element == "Q1E" else 1) * (nx - 1) * (ny - 1)
    f = rng.uniform(-1.0, 1.0, size=(nrhs, nfree))
    return Problem(nx=nx, ny=ny, coeff=coeff, part=part, nsub=nsx * nsy, levels=levels,
                   agglom=agg, constraints=constraints, tau=tau, f=f, element=element,
                   name=name, meta={"channels": ch, "nsx": nsx, "nsy": nsy, "groups": groups})


def voronoi_partition(rng: np.random.Generator, nx: int, ny: int, nsub: int, jitter: bool = False,
                      lloyd: int = 0):
    """Element -> region of the nearest of `nsub` seed points drawn uniformly in
    the unit square (nearest to the element centre, ties to the lower seed).
    With `jitter` (nsub a square q^2), one seed is drawn uniformly in each cell
    of a q x q grid of the unit square instead, which bounds the spread of the
    region sizes.  `lloyd` relaxation steps then move every seed to the mean
    element centre of its region and reassign (no random draws).  Seeds whose
    region holds no element are dropped and the ids renumbered in seed order.
    Returns (part, seed points of the kept regions)."""
    from scipy.spatial import cKDTree

    if jitter:
        q = int(round(np.sqrt(nsub)))
        assert q * q == nsub, "jittered seeds need a square count"
        cell = np.stack(np.meshgrid(np.arange(q), np.arange(q)), axis=-1).reshape(-1, 2)
        pts = (cell + rng.uniform(0.0, 1.0, size=(nsub, 2))) / q
    else:
        pts = rng.uniform(0.0, 1.0, size=(nsub, 2))
    cx = (np.arange(nx) + 0.5) / nx
    cy = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(cx, cy)
    centres = np.column_stack([X.reshape(-1), Y.reshape(-1)])
    _, near = cKDTree(pts).query(centres)
    for _ in range(lloyd):
        cnt = np.bincount(near, minlength=len(pts)).astype(np.float64)
        keep = cnt > 0
        moved = pts.copy()
        moved[keep] = np.column_stack([np.bincount(near, centres[:, 0], len(pts))[keep] / cnt[keep],
                                       np.bincount(near, centres[:, 1], len(pts))[keep] / cnt[keep]])
        pts = moved
        _, near = cKDTree(pts).query(centres)
    used = np.unique(near)
    remap = np.full(nsub, -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    return remap[near].astype(np.int32), pts[used]


def voronoi_agglomeration(rng: np.random.Generator, nx: int, ny: int, part: np.ndarray, nsub: int,
                          ngroups: int, jitter: bool = False) -> np.ndarray:
    """Level-1 region -> group of the nearest of `ngroups` seed points (uniform,
    or jittered as in voronoi_partition) to the region's centroid (mean element
    centre); empty groups dropped."""
    from scipy.spatial import cKDTree

    if jitter:
        q = int(round(np.sqrt(ngroups)))
        assert q * q == ngroups, "jittered seeds need a square count"
        cell = np.stack(np.meshgrid(np.arange(q), np.arange(q)), axis=-1).reshape(-1, 2)
        pts = (cell + rng.uniform(0.0, 1.0, size=(ngroups, 2))) / q
    else:
        pts = rng.uniform(0.0, 1.0, size=(ngroups, 2))
    cx = np.tile((np.arange(nx) + 0.5) / nx, ny)
    cy = np.repeat((np.arange(ny) + 0.5) / ny, nx)
    cnt = np.bincount(part, minlength=nsub).astype(np.float64)
    cen = np.column_stack([np.bincount(part, cx, nsub) / cnt, np.bincount(part, cy, nsub) / cnt])
    _, near = cKDTree(pts).query(cen)
    near = _connected_groups(part.reshape(ny, nx), nsub, near)
    used = np.unique(near)
    remap = np.full(int(near.max()) + 1, -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    return remap[near].astype(np.int32)


def _connected_groups(part2d: np.ndarray, nsub: int, group: np.ndarray) -> np.ndarray:
    """Make every group of regions connected (regions adjacent when they share
    a mesh node): a piece of a group cut off from its largest piece joins the
    adjacent group it touches most, until no group is cut."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    q = np.stack([part2d[:-1, :-1], part2d[:-1, 1:], part2d[1:, :-1], part2d[1:, 1:]], 0).reshape(4, -1)
    a, b = [], []
    for i in range(4):
        for j in range(i + 1, 4):
            m = q[i] != q[j]
            a.append(q[i][m])
            b.append(q[j][m])
    a, b = np.concatenate(a), np.concatenate(b)
    adj = coo_matrix((np.ones(a.size), (a, b)), shape=(nsub, nsub)).tocsr()
    adj = ((adj + adj.T) > 0).astype(np.int8).tocsr()
    group = group.copy()
    for _ in range(50):
        r, c = adj.nonzero()
        keep = group[r] == group[c]
        inner = coo_matrix((np.ones(keep.sum()), (r[keep], c[keep])), shape=(nsub, nsub))
        ncomp, lab = connected_components(inner, directed=False)
        size = np.bincount(lab, minlength=ncomp)
        # the largest piece of each group stays
        best = {}
        for comp in np.argsort(-size, kind="stable"):
            g = int(group[np.argmax(lab == comp)])
            best.setdefault(g, comp)
        stray = [comp for comp in range(ncomp) if best[int(group[np.argmax(lab == comp)])] != comp]
        if not stray:
            return group
        for comp in stray:
            members = np.where(lab == comp)[0]
            nb = adj[members].nonzero()[1]
            nb = nb[group[nb] != group[members[0]]]
            if nb.size:
                group[members] = np.bincount(group[nb]).argmax()
    return group


def voronoi_problem(nx: int, nsub: int, *, levels: int = 2, ngroups: int = 1, constraints: str = "corners",
                    tau: float = float("inf"), kmode: str = "one", kmax_exp: float = 0.0, channels: int = 0,
                    nrhs: int = 1, seed: int = 0, element: str = "Q1", name: str = "",
                    jitter: bool = False, lloyd: int = 0) -> Problem:
    """A seeded problem on an irregular partition of uneven substructures:
    Voronoi regions of `nsub` uniform seed points (level 1) and, for three
    levels, Voronoi groups of their centroids around `ngroups` further seeds.
    Draw order: coefficient, channels, partition seeds, group seeds, loads."""
    assert constraints in CONSTRAINT_KINDS and levels in (2, 3)
    ny = nx
    rng = np.random.Generator(np.random.PCG64(seed))
    if kmode == "one":
        coeff = np.ones(nx * ny)
    elif kmode == "loguniform":
        coeff = 10.0 ** rng.uniform(0.0, kmax_exp, size=nx * ny)
    else:
        raise ValueError(kmode)
    ch = add_channels(rng, nx, ny, coeff, count=channels) if channels else []
    part, _ = voronoi_partition(rng, nx, ny, nsub, jitter=jitter, lloyd=lloyd)
    nkept = int(part.max()) + 1
    agg = [voronoi_agglomeration(rng, nx, ny, part, nkept, ngroups, jitter=jitter)] if levels == 3 else []
    nfree = (nx - 1) * (ny - 1)
    f = rng.uniform(-1.0, 1.0, size=(nrhs, nfree))
    sizes = np.bincount(part, minlength=nkept)
    return Problem(nx=nx, ny=ny, coeff=coeff, part=part, nsub=nkept, levels=levels, agglom=agg,
                   constraints=constraints, tau=tau, f=f, element=element, name=name,
                   meta={"channels": ch, "voronoi": True, "elements_min": int(sizes.min()),
                         "elements_max": int(sizes.max())})


def jag_edge(owner2d: np.ndarray, split: int, lo: int, hi: int, s: int, t: int, width: int, depth: int) -> int:
    """Make the straight horizontal edge between owners s (rows below `split`)
    and t (rows from `split` on), over columns lo..hi-1, jagged in place: the
    columns lo+1 .. hi-2 (so both end points keep their neighbours) are cut
    into teeth `width` columns wide that alternate, starting with a tooth of s
    reaching `depth` rows into t, then one of t reaching `depth` rows into s.
    Each tooth stays attached to its owner, so both stay connected, and every
    node on the new edge is still shared by s and t alone.  Returns the number
    of cells that changed owner."""
    moved = 0
    for c in range(lo + 1, hi - 1):
        if ((c - lo - 1) // width) % 2 == 0:
            rows, src, dst = slice(split, split + depth), t, s
        else:
            rows, src, dst = slice(split - depth, split), s, t
        col = owner2d[rows, c]
        assert (col == src).all(), "the teeth must lie inside the two owners"
        owner2d[rows, c] = dst
        moved += col.size
    return moved


def paper_elasticity_problem(nx: int = 768, nsx: int = 48, *, levels: int = 2, groups: int = 3,
                             constraints: str = "corners", tau: float = float("inf"), jagged: bool = True,
                             teeth=None, nrhs: int = 1, seed: int = 0, name: str = "") -> Problem:
    """The shape of the paper's experiment (Section 6): plane elasticity
    (lambda = 1, mu = 2, k = 1) on the unit square, an nx x nx mesh cut into
    nsx x nsx square substructures (768 / 48: H/h = 16, 2304 substructures)
    and, for three levels, groups x groups level-2 substructures (3 x 3:
    coarsening ratio 16), with one jagged edge on each decomposition level:
    at level 1 between substructures (1, 0) and (1, 1) (x-block, y-block;
    numbers 2 and 50 counted from one), at level 2 between groups (1, 0) and
    (1, 1) (numbers 2 and 5).  The figure that draws the jagged edges is not
    in the text, so the teeth are a reading: one unit wide and one deep
    (elements at level 1, level-1 substructures at level 2), a zigzag that
    starts with a tooth of the lower substructure; at level 1 this shape
    gives the pair eigenvalues printed for the jagged pair and its
    neighbours (Table 3) to within a few percent.  `teeth` = (width, depth)
    overrides it at level 1.  The only random draw is the load."""
    assert constraints in CONSTRAINT_KINDS and levels in (2, 3) and nx % nsx == 0
    assert levels == 2 or nsx % groups == 0
    hh = nx // nsx
    part2d = square_partition(nx, nx, nsx, nsx).reshape(nx, nx)
    moved = [0, 0]
    if jagged:
        assert nsx >= 2 and hh >= 3
        w, d = teeth or (1, 1)
        moved[0] = jag_edge(part2d, hh, hh, 2 * hh, 1, nsx + 1, w, d)
    agg = []
    if levels == 3:
        g2d = square_agglomeration(nsx, nsx, groups, groups).reshape(nsx, nsx)
        m = nsx // groups
        if jagged:
            assert groups >= 2 and m >= 3
            moved[1] = jag_edge(g2d, m, m, 2 * m, 1, groups + 1, 1, 1)
        agg.append(g2d.reshape(-1).astype(np.int32))
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.uniform(-1.0, 1.0, size=(nrhs, 2 * (nx - 1) * (nx - 1)))
    return Problem(nx=nx, ny=nx, coeff=np.ones(nx * nx), part=part2d.reshape(-1).astype(np.int32),
                   nsub=nsx * nsx, levels=levels, agglom=agg, constraints=constraints, tau=tau, f=f,
                   element="Q1E", name=name,
                   meta={"nsx": nsx, "nsy": nsx, "groups": (groups, groups), "jagged": jagged,
                         "moved": moved, "jagged_pairs": [(1, nsx + 1), (1, groups + 1)]})


CONFIG_NAMES = {
    1: "two-level c+e, 32x32 Q1, 4x4 subs (H/h=8), k=1",
    2: "adaptive three-level, 256x256 Q1, 16x16 subs (H/h=16), 4x4 groups, "
       "k=10^U(0,6) + 8 channels k=1e6, tau=10",
    3: "adaptive three-level, 1024x1024 Q1, 64x64 subs (H/h=16), 16x16 groups, k=1, tau=10",
    4: "adaptive three-level, 2048x2048 Q1, 1024 Voronoi regions (jittered seeds, 3 Lloyd steps; about "
       "3000-5700 local dofs), 16 Voronoi groups, k=10^U(0,4), tau=10",
}


def config(cid: int, nrhs: int = 1) -> Problem:
    """The seeded workloads; config c uses seed 1000*c."""
    seed = 1000 * cid
    if cid == 1:
        return square_problem(32, 4, levels=2, constraints="corners_edges", kmode="one",
                              nrhs=nrhs, seed=seed, name="config1")
    if cid == 2:
        return square_problem(256, 16, levels=3, groups=(4, 4), constraints="adaptive",
                              tau=10.0, kmode="loguniform", kmax_exp=6.0, channels=8,
                              nrhs=nrhs, seed=seed, name="config2")
    if cid == 3:
        return square_problem(1024, 64, levels=3, groups=(4, 4), constraints="adaptive",
                              tau=10.0, kmode="one", nrhs=nrhs, seed=seed, name="config3")
    if cid == 4:
        # the batching form: about 1024 uneven substructures of 1500-6000
        # local dofs (one seed uniform in each of 32 x 32 cells, then three
        # Lloyd steps), 16 level-2 groups
        return voronoi_problem(2048, 32 * 32, levels=3, ngroups=4 * 4, constraints="adaptive", tau=10.0,
                               kmode="loguniform", kmax_exp=4.0, nrhs=nrhs, seed=seed, jitter=True, lloyd=3,
                               name="config4")
    raise ValueError(f"unknown config {cid}")


def request_stream(count: int, *, rate: float = 200.0, sides=(128, 256), hh=(8, 16), seed: int = 5000,
                   max_rhs: int = 4, problems: Optional[int] = None):
    """A seeded stream of independent solve requests shaped like the serving
    workload: Poisson arrivals (mean `rate` per second), grid side and H/h
    drawn uniformly from `sides` and `hh` (H/h above the side is skipped:
    the draw is repeated), levels: 3 (level-2 substructures of 4 x 4 level-1
    substructures) from 16 x 16 substructures on, 2 or 3 at random from
    8 x 8 (3: 2 x 2 groups), else 2; k = 10^U(0, m) with m uniform in 0..6,
    adaptive tau = 10, 1 to `max_rhs` right-hand sides U[-1, 1].  Returns
    [(arrival_seconds, Problem)].  The serving workload itself is
    `serving_stream`.

    With `problems`, that many distinct problems are drawn first and every
    request takes one of them uniformly with loads of its own (seeded):
    requests of one problem share its mesh, coefficient field and partition
    (`meta["problem"]` is the problem's index), as repeated solves against
    one discretization do."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if problems:
        base = request_stream(problems, rate=rate, sides=sides, hh=hh, seed=seed + 1, max_rhs=max_rhs)
        t = 0.0
        out = []
        for r in range(count):
            t += rng.exponential(1.0 / rate)
            j = int(rng.integers(0, problems))
            src = base[j][1]
            nrhs = int(rng.integers(1, max_rhs + 1))
            f = rng.uniform(-1.0, 1.0, size=(nrhs, src.n_free))
            prob = Problem(nx=src.nx, ny=src.ny, coeff=src.coeff, part=src.part, nsub=src.nsub, levels=src.levels,
                           agglom=src.agglom, constraints=src.constraints, tau=src.tau, f=f, element=src.element,
                           rtol=src.rtol, name=f"request{r}", meta=dict(src.meta, problem=j))
            out.append((t, prob))
        return out
    t = 0.0
    out = []
    for r in range(count):
        t += rng.exponential(1.0 / rate)
        nx = int(rng.choice(sides))
        h = int(rng.choice(hh))
        while h > nx // 2:
            h = int(rng.choice(hh))
        nsx = nx // h
        # two levels only while the coarse problem stays small (<= 8 x 8
        # substructures: the coarsest problem is solved directly)
        if nsx >= 16 and nsx % 4 == 0:
            levels, groups = 3, (nsx // 4, nsx // 4)
        elif nsx == 8 and int(rng.integers(0, 2)):
            levels, groups = 3, (2, 2)
        else:
            levels, groups = 2, (1, 1)
        m = int(rng.integers(0, 7))
        nrhs = int(rng.integers(1, max_rhs + 1))
        prob = square_problem(nx, nsx, levels=levels, groups=groups, constraints="adaptive", tau=10.0,
                              kmode="loguniform" if m else "one", kmax_exp=float(m), nrhs=nrhs,
                              seed=int(rng.integers(1 << 30)), name=f"request{r}")
        out.append((t, prob))
    return out


def serving_stream(count: int, *, rate: float = 200.0, seed: int = 5000):
    """The serving workload: Poisson arrivals (mean 200 per second), grid side
    in {128, 256, 512, 1024}, H/h in {8, 16, 32}, two or three levels, k =
    10^U(0, m) with m uniform in 0..6, 1 to 16 right-hand sides, adaptive
    tau = 10 (see request_stream for the level rule)."""
    return request_stream(count, rate=rate, sides=(128, 256, 512, 1024), hh=(8, 16, 32), seed=seed, max_rhs=16)
