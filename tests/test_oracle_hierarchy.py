"""Pins for the oracle's grid bookkeeping and Galerkin hierarchy.

* Active-node and block counts of the 16^3-cell rotating cube equal their
  closed forms: a cube of c cells seeded 2x2x2 spans c+3 nodes per axis; two
  nodes share a particle stencil iff they are at most 2 apart on each axis, so
  the block count is (N + 2(N-1) + 2(N-2))^3 with N nodes per axis.  Coarse
  levels embed node 2J, so a span of N fine nodes starting at s has parents
  ceil((s-1)/2) .. floor((s+N)/2).
* Blocks never reach beyond +-2 nodes at any level (Sec. 6 storage bound).
* P reproduces constants and linear fields (linear embedding, Sec. 4.2).
* The composite kernel of level m has support radius 1 + 2^-(m+1) in its own
  units (Fig. kernel width: 3dx -> 2dx).
* H^1 = P~^T H^0 P~ (Eq. buildMultigrid) equals the particle-quadrature
  re-discretisation with composite weight gradients sum_i R_ji grad w_ip
  (Sec. 4.2) plus the embedded mass matrix; checked without Dirichlet nodes.
"""
import numpy as np
import pytest

import hot_scenes as hs
import oracle as O


def span_counts(n_nodes):
    return n_nodes + 2 * (n_nodes - 1) + 2 * (n_nodes - 2)


@pytest.fixture(scope="module")
def cube_hierarchy():
    sc = hs.rotating_cube()
    st = O.prepare(sc, O.time_step(sc))
    lev = st.lev0
    pats = [O.fine_pattern(sc, lev)]
    levels = [lev]
    for _ in range(2):
        P, coarse = O.prolongation(lev)
        pats.append(O.coarse_pattern(lev, pats[-1], P, coarse))
        levels.append(coarse)
        lev = coarse
    return sc, levels, pats


def test_cube_counts_closed_form(cube_hierarchy):
    sc, levels, pats = cube_hierarchy
    # cube cells [8, 24): bases 7..23, nodes 7..25 -> 19 per axis
    start, N = 7, 16 + 3
    expect_nodes, expect_blocks = [], []
    for m in range(3):
        expect_nodes.append(N ** 3)
        expect_blocks.append(span_counts(N) ** 3)
        lo = -((-(start - 1)) // 2)
        hi = (start + N) // 2
        start, N = lo, hi - lo + 1
    assert [l.n for l in levels] == expect_nodes == [6859, 1331, 343]
    assert [int(p.sum()) for p in pats] == expect_blocks == [704969, 117649, 24389]
    for p in pats:
        assert p.any(axis=0).all()          # every one of the 125 offsets occurs


def test_prolongation_reproduces_linear_fields(rng):
    sc = hs.small_box(seed=31, cells=(12, 12, 12), box_lo=(3, 2, 4), box_hi=(9, 7, 8))
    lev = O.active_fine_nodes(sc)
    P, coarse = O.prolongation(lev)
    assert np.abs(P @ np.ones(coarse.n) - 1.0).max() < 1e-15
    for a in range(3):
        assert np.abs(P @ (2.0 * coarse.coords[:, a]) - lev.coords[:, a]).max() < 1e-13
    assert np.all(np.diff(P.indptr) <= 8)
    nnz_col = np.bincount(P.indices, minlength=coarse.n)
    assert nnz_col.max() <= 27


def composite_weights(x, levels_P, lev0, origin, dx):
    """w^m_Jp = sum over the chain of prolongations of w_ip (dense, tiny)."""
    W, G, nodes, _ = O.stencil(x, origin, dx)
    idx = lev0.lookup(O.linear(nodes, lev0.dims))
    dense = np.zeros((x.shape[0], lev0.n))
    np.add.at(dense, (np.repeat(np.arange(x.shape[0]), 27), idx.ravel()), W.ravel())
    out = [dense]
    for P in levels_P:
        out.append(out[-1] @ P.toarray())
    return out


def test_composite_kernel_support_radius():
    # a single dense line of sample points through a fixed grid of nodes
    dx = 1.0
    xs = np.stack([np.linspace(4.02, 27.98, 1200), np.full(1200, 16.3), np.full(1200, 16.3)], -1)
    sc = hs.small_box(seed=1, cells=(40, 40, 40), box_lo=(3, 14, 14), box_hi=(29, 19, 19), dx=dx)
    lev0 = O.active_fine_nodes(sc)
    Ps, lev = [], lev0
    for _ in range(3):
        P, coarse = O.prolongation(lev)
        Ps.append(P)
        lev = coarse
    ws = composite_weights(xs, Ps, lev0, sc.origin, dx)
    levs = [lev0]
    lev = lev0
    for P in Ps:
        _, lev = O.prolongation(lev)
        levs.append(lev)
    for m, (w, L) in enumerate(zip(ws, levs)):
        h = 2.0 ** m
        pos = L.coords[:, 0] * h
        radius = 1.5 if m == 0 else 1.0 + 2.0 ** -(m + 1)
        d = np.abs(xs[:, 0][:, None] - pos[None, :]) / h
        inside = w > 1e-14
        assert d[inside].max() <= radius + 1e-12
        # support is attained: points just inside the radius carry weight
        dyz = np.abs(L.coords[:, 1:] * h - 16.3).max(axis=1) / h
        near = (d > radius - 0.05) & (d < radius - 0.01) & (dyz < radius - 0.05)[None, :]
        assert near.sum() > 0 and np.all(w[near] > 0)


def test_galerkin_equals_composite_particle_quadrature():
    sc = hs.small_box(seed=41, cells=(10, 10, 10), box_lo=(3, 3, 2), box_hi=(7, 6, 7),
                      walls=None, F_spread=0.25, noise=0.2)
    dt = 2e-3
    st = O.prepare(sc, dt)
    H0, nbr0 = O.hessian_slots(st)
    hz = O.build_hierarchy(st, H0, nbr0, 2)
    P = hz.Pnode[0].toarray()
    idx = st.idx
    n1 = hz.levels[1].n
    # composite weight gradients sum_i P_iJ grad w_ip (Sec. 4.2)
    Gc = np.zeros((sc.n, n1, 3))
    for k in range(27):
        Gc += P[idx[:, k]][:, :, None] * st.G[:, k, None, :]
    ac = np.einsum("pba,pjb->pja", sc.F, Gc)
    F0 = O.deformation(st, np.zeros((st.lev0.n, 3)))
    C = O.dPdF(F0, st.model, st.mu, st.lam).reshape(-1, 3, 3, 3, 3)
    H1 = np.einsum("p,pjb,pgbde,pke->jgkd", dt * dt * st.Vp, ac, C, ac).reshape(3 * n1, 3 * n1)
    H1 += np.kron(P.T @ np.diag(st.m) @ P, np.eye(3))
    A1 = hz.A[1].toarray()
    assert np.abs(A1 - H1).max() < 1e-12 * np.abs(H1).max()
    # rigid translations: elastic part vanishes, mass is conserved
    for c in range(3):
        e = np.zeros(3 * n1)
        e[c::3] = 1.0
        assert abs((A1 @ e).sum() - st.m.sum()) < 1e-12 * st.m.sum()


def test_galerkin_with_dirichlet_matches_dense_projection():
    sc = hs.small_box(seed=43, cells=(9, 9, 9), box_lo=(2, 2, 2), box_hi=(7, 6, 6), walls=2)
    st = O.prepare(sc, 5e-3)
    H0, nbr0 = O.hessian_slots(st)
    hz = O.build_hierarchy(st, H0, nbr0, 3)
    assert st.fixed.any() and st.free.any()
    for m in range(2):
        Pd = np.kron(hz.Pnode[m].toarray(), np.eye(3))
        Pt = np.diag(hz.free[m]) @ Pd
        ref = Pt.T @ hz.A[m].toarray() @ Pt
        ref += np.diag((np.diag(ref) == 0.0).astype(float))
        assert np.abs(hz.A[m + 1].toarray() - ref).max() <= 1e-13 * np.abs(ref).max()
    # constrained rows/cols at level 0 are exactly decoupled
    A0 = hz.A[0].toarray()
    fd = np.repeat(st.fixed, 3)
    assert np.all(A0[np.ix_(fd, ~fd)] == 0.0)
