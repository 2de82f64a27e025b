"""The seeded input generators: Voronoi partitions and their groups."""

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import synth


def _pieces(part2d, nsub, group):
    q = np.stack([part2d[:-1, :-1], part2d[:-1, 1:], part2d[1:, :-1], part2d[1:, 1:]], 0).reshape(4, -1)
    a, b = [], []
    for i in range(4):
        for j in range(i + 1, 4):
            m = (q[i] != q[j]) & (group[q[i]] == group[q[j]])
            a.append(q[i][m])
            b.append(q[j][m])
    a, b = np.concatenate(a), np.concatenate(b)
    n, lab = connected_components(coo_matrix((np.ones(a.size), (a, b)), shape=(nsub, nsub)), directed=False)
    per = np.zeros(group.max() + 1, int)
    np.add.at(per, group[np.unique(lab, return_index=True)[1]], 1)
    return per


def test_voronoi_groups_are_connected_and_cover_every_region():
    for args in (dict(nx=128, nsub=48, levels=3, ngroups=8, seed=34),
                 dict(nx=256, nsub=400, levels=3, ngroups=36, seed=9, jitter=True)):
        p = synth.voronoi_problem(**args)
        g = p.agglom[0]
        assert g.shape == (p.nsub,) and g.min() == 0
        assert np.all(np.bincount(g) > 0)
        assert np.all(_pieces(p.part.reshape(p.ny, p.nx), p.nsub, g) == 1)
        assert np.array_equal(np.unique(p.part), np.arange(p.nsub))


def test_jittered_seeds_bound_the_region_sizes():
    p = synth.voronoi_problem(256, 256, seed=3, jitter=True)
    sizes = np.bincount(p.part)
    assert sizes.max() <= 2.5 * sizes.mean() and sizes.min() >= 0.25 * sizes.mean()
    q = synth.voronoi_problem(256, 256, seed=3)
    assert np.bincount(q.part).max() > sizes.max()
