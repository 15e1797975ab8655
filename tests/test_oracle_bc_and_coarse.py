"""Pins for the oracle's boundary conditions, time-step rule, l1 block-Jacobi
smoother and coarsest-level Jacobi-PCG.

* Box walls (Sec. 7 set-ups): the constrained count on a full node lattice is
  (c+1)^3 - (c-1-2t)^3 for c cells and thickness t.
* Grips prescribe a rigid rotation: relative velocities of any two held nodes
  are orthogonal to their separation, speeds equal |omega| times the distance
  to the axis, nodes on the axis are at rest, and the axis direction need not
  be unit length.  The largest prescribed speed reaches the closed-form corner
  bound sqrt(a^2 + b^2)|omega| and no held node exceeds it.
* A moving sphere held at t_end equals the sphere at t = 0 shifted by a whole
  number of cells; later conditions override earlier ones.
* The time-step rule reduces to 1/FPS at rest and to CFL dx / v_max otherwise
  (Sec. 7.1 settings).
* l1 block-Jacobi (the substitute smoother): without coupling it is textbook
  block-Jacobi; for n nodes coupled by c I3 each row's l1 term is (n-1)|c|; and
  on a strongly coupled SPD matrix where plain block-Jacobi diverges,
  2M - A is SPD, so the smoother contracts in the energy norm.
* Jacobi-PCG (Sec. 5.3, coarsest level): after k iterations with no early stop
  its iterate is the energy-norm minimiser over the Krylov space
  span{D^-1 b, (D^-1 A) D^-1 b, ...}, computed here by brute force; on a
  diagonal matrix it is exact after one iteration; it stops at the first
  iterate that meets the relative D^-1-norm rule.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import hot_scenes as hs
import oracle as O


def full_level(cells):
    dims = np.asarray(cells, dtype=np.int64) + 1
    return O.Level(np.arange(int(np.prod(dims)), dtype=np.int64), dims)


def scene_with(bcs, cells=(8, 8, 8), dx=0.1, v=None):
    sc = hs.small_box(cells=cells, dx=dx)
    sc.bcs = list(bcs)
    if v is not None:
        sc.v = np.asarray(v, dtype=np.float64)
    return sc


@pytest.mark.parametrize("cells,th", [((8, 8, 8), 2), ((8, 8, 8), 0), ((10, 10, 10), 3)])
def test_walls_constrained_count_closed_form(cells, th):
    sc = scene_with([hs.bc_walls(th)], cells=cells)
    lev = full_level(cells)
    mask, vbc = O.bc_nodes(sc, lev, 0.0)
    c = cells[0]
    assert mask.sum() == (c + 1) ** 3 - (c - 1 - 2 * th) ** 3
    assert np.all(vbc == 0.0)


def test_grip_is_rigid_rotation():
    # dx = 1/8 keeps node positions, the box and the axis exact in binary
    omega = 2.5
    point = np.array([0.5, 0.375, 0.0])
    sc = scene_with([hs.bc_grip((0.125, 0.125, 0.25), (0.75, 0.625, 0.5), point, (0.0, 0.0, 2.0),
                                omega)], dx=0.125)
    lev = full_level(sc.grid_cells)
    mask, vbc = O.bc_nodes(sc, lev, 0.0)
    x = lev.coords[mask] * sc.dx
    v = vbc[mask]
    assert mask.sum() > 8
    # rigid: (v_i - v_j) . (x_i - x_j) = 0 for every pair
    dv = v[:, None, :] - v[None, :, :]
    dxp = x[:, None, :] - x[None, :, :]
    assert np.max(np.abs(np.sum(dv * dxp, axis=2))) < 1e-12
    # about the z axis through point: speed = omega * radial distance, no axial part
    rad = np.linalg.norm(x[:, :2] - point[:2], axis=1)
    assert np.allclose(np.linalg.norm(v, axis=1), omega * rad, rtol=0, atol=1e-12)
    assert np.all(v[:, 2] == 0.0)
    on_axis = rad < 1e-12
    assert on_axis.any() and np.all(v[on_axis] == 0.0)
    # counter-clockwise seen from +z for omega > 0: v = omega (-(y - py), x - px)
    assert np.allclose(v[:, 0], -omega * (x[:, 1] - point[1]), atol=1e-12)
    assert np.allclose(v[:, 1], omega * (x[:, 0] - point[0]), atol=1e-12)


def test_grip_max_speed_corner_bound():
    omega, a, b = -3.0, 0.375, 0.25
    center = np.array([0.5, 0.5, 0.5])
    lo = center - np.array([a, b, 0.25])
    hi = center + np.array([a, b, 0.25])
    sc = scene_with([hs.bc_grip(lo, hi, center, (0.0, 0.0, 1.0), omega)], dx=0.125)
    smax = O.bc_max_speed(sc)
    assert smax == pytest.approx(abs(omega) * math.hypot(a, b), rel=1e-14)
    mask, vbc = O.bc_nodes(sc, full_level(sc.grid_cells), 0.0)
    speeds = np.linalg.norm(vbc[mask], axis=1)
    assert speeds.max() <= smax * (1 + 1e-12)
    # the box corners sit on lattice nodes here, so the bound is reached
    assert speeds.max() == pytest.approx(smax, rel=1e-12)


def test_sphere_moves_with_its_velocity():
    # centre half-way between nodes and dx = 1/8: squared node distances are
    # exact and none ties with the radius
    dx = 0.125
    vel = np.array([2.0 * dx, -1.0 * dx, 3.0 * dx])  # one time unit = (2, -1, 3) cells
    sc0 = scene_with([hs.bc_sphere((0.4375, 0.5625, 0.3125), 0.3, vel)], cells=(12, 12, 12), dx=dx)
    lev = full_level(sc0.grid_cells)
    m0, v0 = O.bc_nodes(sc0, lev, 0.0)
    m1, v1 = O.bc_nodes(sc0, lev, 1.0)
    assert m0.sum() > 0 and m0.sum() == m1.sum()
    shifted = set(map(tuple, lev.coords[m0] + np.array([2, -1, 3])))
    assert shifted == set(map(tuple, lev.coords[m1]))
    assert np.all(v1[m1] == vel) and np.all(v0[m0] == vel)
    assert np.all(v1[~m1] == 0.0)


def test_later_conditions_override_earlier():
    dx = 0.1
    vel = np.array([0.5, 0.0, 0.0])
    sc = scene_with([hs.bc_walls(2), hs.bc_sphere((0.1, 0.4, 0.4), 0.25, vel)], dx=dx)
    lev = full_level(sc.grid_cells)
    mask, vbc = O.bc_nodes(sc, lev, 0.0)
    walls, _ = O.bc_nodes(scene_with([hs.bc_walls(2)], dx=dx), lev, 0.0)
    ball, _ = O.bc_nodes(scene_with([hs.bc_sphere((0.1, 0.4, 0.4), 0.25, vel)], dx=dx), lev, 0.0)
    both = walls & ball
    assert both.any() and (walls & ~ball).any()
    assert np.array_equal(mask, walls | ball)
    assert np.all(vbc[ball] == vel)
    assert np.all(vbc[walls & ~ball] == 0.0)


def test_time_step_rule():
    sc = scene_with([], v=np.zeros((hs.small_box().n, 3)))
    assert O.time_step(sc) == sc.max_dt
    vel = np.zeros((sc.n, 3))
    vel[7] = (30.0, -40.0, 0.0)  # |v| = 50
    sc.v = vel
    assert O.time_step(sc) == pytest.approx(sc.cfl * sc.dx / 50.0, rel=1e-15)
    # a faster grip sets the step instead of the particles
    sc.bcs = [hs.bc_grip((0.0, 0.0, 0.0), (0.8, 0.8, 0.8), (0.0, 0.0, 0.0), (1.0, 0.0, 0.0), 100.0)]
    assert O.time_step(sc) == pytest.approx(sc.cfl * sc.dx / (100.0 * 0.8 * math.sqrt(2)), rel=1e-14)


def block_matrix(blocks, n):
    """Dense 3n x 3n matrix from a dict {(i, j): 3x3 block}."""
    A = np.zeros((3 * n, 3 * n))
    for (i, j), B in blocks.items():
        A[3 * i:3 * i + 3, 3 * j:3 * j + 3] += B
    return A


def spd_block(rng, scale=1.0):
    G = rng.normal(size=(3, 3))
    return scale * (G @ G.T + 3.0 * np.eye(3))


def test_l1_jacobi_without_coupling_is_block_inverse():
    rng = np.random.default_rng(11)
    n = 5
    blocks = {(i, i): spd_block(rng) for i in range(n)}
    A = block_matrix(blocks, n)
    M = O.l1_block_jacobi_inverse(sp.csr_matrix(A)).toarray()
    assert np.allclose(M, np.linalg.inv(A), rtol=1e-13, atol=1e-15)


def test_l1_term_for_uniform_coupling():
    rng = np.random.default_rng(12)
    n, c = 4, -0.7
    K = spd_block(rng) + 10.0 * np.eye(3)  # off-diagonal entries inside the block too
    blocks = {(i, j): (K if i == j else c * np.eye(3)) for i in range(n) for j in range(n)}
    M = O.l1_block_jacobi_inverse(sp.csr_matrix(block_matrix(blocks, n))).toarray()
    want = np.linalg.inv(K + (n - 1) * abs(c) * np.eye(3))
    for i in range(n):
        assert np.allclose(M[3 * i:3 * i + 3, 3 * i:3 * i + 3], want, rtol=1e-13)
        off = np.delete(M[3 * i:3 * i + 3], np.s_[3 * i:3 * i + 3], axis=1)
        assert np.all(off == 0.0)


def test_l1_jacobi_contracts_where_block_jacobi_diverges():
    rng = np.random.default_rng(13)
    n = 6
    # all nodes strongly coupled: A = J (x) S + I (x) eps I, SPD, off-diagonal
    # blocks as large as the diagonal ones
    S = spd_block(rng)
    blocks = {(i, j): S.copy() for i in range(n) for j in range(n)}
    for i in range(n):
        blocks[(i, i)] = blocks[(i, i)] + 0.05 * np.eye(3)
    A = block_matrix(blocks, n)
    assert np.linalg.eigvalsh(A).min() > 0
    Dinv_plain = np.zeros_like(A)
    for i in range(n):
        Dinv_plain[3 * i:3 * i + 3, 3 * i:3 * i + 3] = np.linalg.inv(A[3 * i:3 * i + 3, 3 * i:3 * i + 3])
    rho_plain = np.abs(np.linalg.eigvals(np.eye(3 * n) - Dinv_plain @ A)).max()
    assert rho_plain > 1.0  # plain block-Jacobi diverges here
    Minv = O.l1_block_jacobi_inverse(sp.csr_matrix(A)).toarray()
    M = np.linalg.inv(Minv)
    assert np.linalg.eigvalsh(M + M.T - A).min() > 0
    rho = np.abs(np.linalg.eigvals(np.eye(3 * n) - Minv @ A)).max()
    assert rho < 1.0


def random_spd(rng, m, cond=1e2):
    Q, _ = np.linalg.qr(rng.normal(size=(m, m)))
    ev = np.geomspace(1.0, cond, m)
    D = rng.uniform(0.5, 5.0, size=m)  # badly scaled rows: the Jacobi preconditioner matters
    A = (Q * ev) @ Q.T
    return D[:, None] * A * D[None, :]


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_pcg_iterate_minimises_energy_error_over_krylov_space(k):
    rng = np.random.default_rng(20 + k)
    m = 18
    A = random_spd(rng, m)
    b = rng.normal(size=m)
    d = np.diag(A).copy()
    log = []
    x = O.coarse_pcg(sp.csr_matrix(A), d, b, rel=0.0, max_iter=k, log=log)
    assert log == [k]
    # brute force: an orthonormal basis of the Krylov space of D^-1 A and
    # D^-1 b (each new direction orthogonalised twice), then the Galerkin
    # solve on it, which is the energy-norm minimiser
    Q = np.empty((m, k))
    vec = b / d
    for j in range(k):
        for _ in range(2):
            vec = vec - Q[:, :j] @ (Q[:, :j].T @ vec)
        Q[:, j] = vec / np.linalg.norm(vec)
        vec = (A @ Q[:, j]) / d
    y = np.linalg.solve(Q.T @ A @ Q, Q.T @ b)
    want = Q @ y
    assert np.allclose(x, want, rtol=1e-8, atol=1e-10 * np.abs(want).max())


def test_pcg_diagonal_matrix_exact_in_one_iteration():
    rng = np.random.default_rng(30)
    d = rng.uniform(0.1, 10.0, size=12)
    b = rng.normal(size=12)
    log = []
    x = O.coarse_pcg(sp.diags(d).tocsr(), d, b, rel=1e-14, log=log)
    assert log == [1]
    assert np.allclose(x, b / d, rtol=1e-14)


def test_pcg_stops_at_first_iterate_meeting_the_rule():
    rng = np.random.default_rng(31)
    m = 24
    A = random_spd(rng, m, cond=1e3)
    b = rng.normal(size=m)
    d = np.diag(A).copy()
    As = sp.csr_matrix(A)

    def dnorm(r):
        return math.sqrt(float(r @ (r / d)))

    for rel in (0.5, 1e-3, 1e-6):
        log = []
        x = O.coarse_pcg(As, d, b, rel=rel, log=log)
        it = log[0]
        assert dnorm(b - A @ x) <= rel * dnorm(b) * (1 + 1e-9)
        if it > 1:
            xp = O.coarse_pcg(As, d, b, rel=0.0, max_iter=it - 1)
            assert dnorm(b - A @ xp) > rel * dnorm(b)
    # a tight solve is the exact solution
    x = O.coarse_pcg(As, d, b, rel=1e-12)
    want = np.linalg.solve(A, b)
    assert np.allclose(x, want, rtol=1e-6, atol=1e-9 * np.abs(want).max())
