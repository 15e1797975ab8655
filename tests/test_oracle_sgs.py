"""Pins for the oracle's coloured symmetric block Gauss-Seidel smoother
(Alg. V-cycle; Sec. 5.3 and Sec. 8 name coloured symmetric Gauss-Seidel).

* The 27-colour classes (grid coordinate mod 3 per axis) never couple two
  distinct nodes at any level, while nodes two apart do couple, so fewer
  residues per axis would not do.
* One smoothing from u0 equals the textbook block Gauss-Seidel pair in the
  colour-major node order, computed with dense library solves:
  (D + L) u' = b - U u0, then (D + U) u1 = b - L u'  (D the 3x3 diagonal
  blocks, L / U the strictly lower / upper block parts).
* Repeated smoothing converges to H^{-1} b (SPD matrix).
* With an exact coarse solve the V-cycle is symmetric positive definite on
  the free DOFs, so it remains a valid L-BFGS initial inverse Hessian.
* HOT with this smoother, driven to a tight tolerance, lands on the dense
  projected-Newton minimiser.
"""
import numpy as np
import pytest

import oracle as O
from test_oracle_solver import _dense_V, _hz, dense_newton, tiny


def _levels_and_colors(seed=81, levels=3):
    sc = tiny(seed, walls=2, cells=(10, 10, 10), box_lo=(2, 2, 2), box_hi=(7, 7, 8))
    st, hz = _hz(sc, 1e-2, levels)
    return st, hz


def test_colors_never_couple_distinct_nodes():
    st, hz = _levels_and_colors()
    for m, (A, lev) in enumerate(zip(hz.A, hz.levels)):
        col = O.node_colors(lev)
        assert col.min() >= 0 and col.max() < O.N_COLORS
        C = A.tocoo()
        bi, bj = C.row // 3, C.col // 3
        nz = (C.data != 0.0) & (bi != bj)
        assert nz.any()
        assert np.all(col[bi[nz]] != col[bj[nz]]), f"level {m}"
        # couplings reach two nodes along an axis: residues mod 2 would clash
        d = np.abs(lev.coords[bi[nz]] - lev.coords[bj[nz]]).max(axis=1)
        assert d.max() == 2


def _block_parts(A, order):
    """Dense D, L, U of A in the node order `order` (3x3 blocks)."""
    dofs = (3 * order[:, None] + np.arange(3)[None, :]).ravel()
    Ad = A.toarray()[np.ix_(dofs, dofs)]
    n = len(order)
    blk = np.arange(3 * n) // 3
    D = np.where(blk[:, None] == blk[None, :], Ad, 0.0)
    L = np.where(blk[:, None] > blk[None, :], Ad, 0.0)
    U = np.where(blk[:, None] < blk[None, :], Ad, 0.0)
    return dofs, D, L, U


@pytest.mark.parametrize("level", [0, 1])
def test_one_smoothing_equals_textbook_block_gauss_seidel(level):
    st, hz = _levels_and_colors(83)
    A, lev = hz.A[level], hz.levels[level]
    col = O.node_colors(lev)
    order = np.lexsort((np.arange(lev.n), col))     # colour-major, then index
    dofs, D, L, U = _block_parts(A, order)
    rng = np.random.Generator(np.random.PCG64(5))
    b = rng.normal(size=3 * lev.n)
    u0 = rng.normal(size=3 * lev.n)
    got = O.sgs(O.sgs_setup(A, lev), b, u0, sweeps=1)
    bp, u0p = b[dofs], u0[dofs]
    half = np.linalg.solve(D + L, bp - U @ u0p)
    ref = np.linalg.solve(D + U, bp - L @ half)
    assert np.abs(got[dofs] - ref).max() < 1e-10 * np.abs(ref).max()


def test_repeated_smoothing_converges_to_solution():
    st, hz = _levels_and_colors(85, levels=2)
    A, lev = hz.A[0], hz.levels[0]
    f = hz.free[0].astype(bool)
    rng = np.random.Generator(np.random.PCG64(6))
    b = rng.normal(size=3 * lev.n) * f
    u = O.sgs(O.sgs_setup(A, lev), b, np.zeros_like(b), sweeps=300)
    x = np.zeros_like(b)
    x[f] = np.linalg.solve(A.toarray()[np.ix_(f, f)], b[f])
    assert np.abs(u - x).max() < 1e-8 * np.abs(x).max()


def test_vcycle_with_sgs_symmetric_positive_definite():
    sc = tiny(87, walls=2, cells=(9, 9, 9), box_lo=(2, 2, 2), box_hi=(6, 6, 7))
    st, hz = _hz(sc, 1e-2, 3)
    Ac = hz.A[-1].toarray()
    N = hz.A[0].shape[0]
    V = np.stack([O.vcycle(hz, e, coarse_solver=lambda b: np.linalg.solve(Ac, b),
                           smoother="sgs") for e in np.eye(N)], 1)
    f = np.repeat(st.free, 3)
    Vf = V[np.ix_(f, f)]
    assert np.abs(Vf - Vf.T).max() < 1e-12 * np.abs(Vf).max()
    assert np.linalg.eigvalsh(0.5 * (Vf + Vf.T)).min() > 0
    assert np.all(V[~f] == 0.0)
    # a different operator from the l1 block-Jacobi cycle
    Vj = _dense_V(hz, smoother="l1jacobi")[np.ix_(f, f)]
    assert np.abs(Vf - Vj).max() > 1e-3 * np.abs(Vj).max()


def test_converged_step_with_sgs_matches_dense_newton():
    sc = tiny(89, model=0, walls=2)
    dt = 1e-2
    st = O.prepare(sc, dt)
    H0, nbr0 = O.hessian_slots(st)
    hz = O.build_hierarchy(st, H0, nbr0, 2)
    dv, info = O.solve(st, hz, tol=1e-12, history=8, max_iters=300, smoother="sgs")
    ref = dense_newton(st)
    a, b = O.g2p(st, dv), O.g2p(st, ref)
    assert np.abs(a.v - b.v).max() < 1e-7 * np.abs(b.v).max()
    assert np.abs(a.x - b.x).max() < 1e-10
    E = info["log"]["E"]
    assert all(y <= x + 1e-13 * abs(x) for x, y in zip(E, E[1:]))
