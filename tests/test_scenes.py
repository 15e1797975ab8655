"""Input recipes: the stretched-box workload's generator."""
import numpy as np

import hot_scenes as hs


def test_stretched_box_recipe():
    sc = hs.stretched_box(side=6, margin=3, seed=9)
    assert sc.n == 8 * 6 ** 3 and sc.grid_cells == (12, 12, 12)
    assert sc.gravity == (0.0, 0.0, 0.0) and list(sc.bcs) == []
    assert np.all(sc.v == 0.0) and np.all(sc.C == 0.0)
    off = sc.F.copy()
    for a in range(3):
        off[:, a, a] = 0.0
    assert np.all(off == 0.0)  # diagonal deformation gradients
    d = np.stack([sc.F[:, a, a] for a in range(3)], axis=1)
    assert d.min() >= 0.7 and d.max() <= 1.3
    assert np.all(d == d[0])  # one matrix for the whole box
    pp = hs.stretched_box(side=6, margin=3, seed=9, per_particle=True)
    e = np.stack([pp.F[:, a, a] for a in range(3)], axis=1)
    assert e.min() >= 0.7 and e.max() <= 1.3
    # per particle: the mean and variance of U[0.7, 1.3] within sampling error
    assert abs(e.mean() - 1.0) < 0.01 and abs(e.var() - 0.6 ** 2 / 12) < 0.003
    # particles in the box's cells [3, 9)^3, inside the grid
    cell = np.floor(sc.x / sc.dx).astype(int)
    assert cell.min() >= 3 and cell.max() <= 8
    assert sc.tol == 1e-7 and sc.lbfgs_history == 8
    # reproducible from the seed
    assert np.array_equal(hs.stretched_box(side=6, margin=3, seed=9).F, sc.F)
