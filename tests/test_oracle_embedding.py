"""Pins for the oracle's quadratic node embedding (HOT-quadratic).

The paper's alternative embedding applies the quadratic B-spline to the
prolongation too (Sec. 4.2, kernel choice; the HOT-quadratic ablation of
Sec. 7).  These checks rest on properties of that spline rather than on its
formula:
* the per-axis weights form a partition of unity, reproduce linear fields
  (first moment) and have the constant second moment 1 fine spacing^2 that a
  quadratic B-spline of twice the spacing has (3 (h/2)^2 ... = 1 here), with
  three parents for even and two for odd fine coordinates;
* the Galerkin levels built with it are symmetric, their energy is the fine
  level's energy of the prolongated vector, and their stencils grow to 3
  nodes but no further (the paper's bounded growth), against 2 for the
  linear embedding;
* HOT with either embedding converges to the same step (the minimiser of
  Eq. 1 is unique), and the quadratic embedding needs no fewer than about as
  many L-BFGS iterations as the linear one, the paper's ablation finding.
"""
import numpy as np
import pytest

import hot_scenes as hs
import oracle as O


def test_quadratic_weights_moments():
    c = np.arange(2, 200)
    J0, J1, J2, w0, w1, w2 = O.parents_1d_quadratic(c)
    J = np.stack([J0, J1, J2], 1)
    w = np.stack([w0, w1, w2], 1)
    assert np.all(w >= 0.0)
    assert np.allclose(w.sum(1), 1.0, rtol=0, atol=1e-15)
    assert np.allclose((w * (2 * J)).sum(1), c, rtol=0, atol=1e-12)
    assert np.allclose((w * (2 * J - c[:, None]) ** 2).sum(1), 1.0, rtol=0, atol=1e-14)
    nz = (w > 0).sum(1)
    assert np.all(nz[c % 2 == 0] == 3) and np.all(nz[c % 2 == 1] == 2)
    # every parent lies within two fine nodes
    assert np.all(np.abs(2 * J - c[:, None])[w > 0] <= 2)


def test_quadratic_prolongation_reproduces_linear_fields():
    sc = hs.rotating_cube(cells=16, cube=8, seed=3)
    st = O.prepare(sc, O.time_step(sc))
    P, coarse = O.prolongation(st.lev0, "quadratic")
    X = coarse.coords.astype(np.float64)
    x = st.lev0.coords.astype(np.float64)
    assert np.allclose(P @ np.ones(coarse.n), 1.0, atol=1e-14)
    # coarse node K sits at fine node 2K - 2
    for a in range(3):
        assert np.allclose(P @ (2.0 * X[:, a] - 2.0), x[:, a], atol=1e-12)


@pytest.fixture(scope="module")
def quad_hierarchy():
    sc = hs.small_box(cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(9, 9, 9), dx=0.05, seed=31,
                      levels=3, walls=2)
    st = O.prepare(sc, O.time_step(sc))
    H0, nbr0 = O.hessian_slots(st)
    hq = O.build_hierarchy(st, H0, nbr0, 3, embedding="quadratic")
    hl = O.build_hierarchy(st, H0, nbr0, 3)
    return sc, st, hq, hl


def _reach(A, lev):
    C = A.tocoo()
    r, c = C.row // 3, C.col // 3
    return int(np.abs(lev.coords[c] - lev.coords[r]).max())


def test_quadratic_galerkin_levels(quad_hierarchy):
    sc, st, hq, hl = quad_hierarchy
    rng = np.random.Generator(np.random.PCG64(4))
    for m in range(1, 3):
        A, Af, P = hq.A[m], hq.A[m - 1], hq.P[m - 1]
        assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
        u = rng.normal(size=A.shape[0]) * hq.free[m]
        e_c = u @ (A @ u)
        Pu = P @ u
        assert abs(e_c - Pu @ (Af @ Pu)) <= 1e-11 * abs(e_c)
        assert e_c > 0.0
    # stencil reach: quadratic grows to 3 nodes and stays there, linear keeps 2
    assert [_reach(hq.A[m], hq.levels[m]) for m in range(3)] == [2, 3, 3]
    assert [_reach(hl.A[m], hl.levels[m]) for m in range(3)] == [2, 2, 2]


def test_quadratic_vcycle_symmetric(quad_hierarchy):
    sc, st, hq, hl = quad_hierarchy
    n = hq.A[0].shape[0]
    rng = np.random.Generator(np.random.PCG64(5))
    x = rng.normal(size=n) * hq.free[0]
    y = rng.normal(size=n) * hq.free[0]
    # an exact coarsest solve keeps the cycle a fixed linear operator
    Ac = hq.A[-1].toarray()
    coarse = lambda b: np.linalg.solve(Ac, b)
    vx = O.vcycle(hq, x, coarse_solver=coarse)
    vy = O.vcycle(hq, y, coarse_solver=coarse)
    assert abs(y @ vx - x @ vy) <= 1e-9 * abs(y @ vx)


def test_hot_quadratic_converges_to_the_same_step():
    sc = hs.small_box(cells=(10, 10, 10), box_lo=(3, 3, 3), box_hi=(7, 8, 7), dx=0.05, seed=33,
                      levels=3, walls=2, tol=1e-10, E=1e5)
    dt = O.time_step(sc)
    out_l, info_l = O.step(sc, dt=dt)
    out_q, info_q = O.step(sc, dt=dt, embedding="quadratic")
    print(f"HOT {info_l['iters']} iterations, HOT-quadratic {info_q['iters']}")
    assert info_l["converged"] and info_q["converged"]
    scale = np.abs(out_l.v).max()
    assert np.abs(out_q.v - out_l.v).max() <= 1e-6 * scale
    assert np.abs(out_q.x - out_l.x).max() <= 1e-6 * np.abs(out_l.x).max()


def test_quadratic_embedding_rejects_gauss_seidel():
    sc = hs.small_box(levels=2)
    with pytest.raises(ValueError):
        O.step(sc, embedding="quadratic", smoother="sgs")
