"""Pins for the oracle's quadratic B-spline kernel and APIC transfers.

Closed forms: partition of unity, vanishing first moment, second moment
dx^2/4 I, sum of gradients 0 and sum x_i grad w^T = I (quadratic B-spline,
Sec. 6).  Invariants: P2G/G2P conserve mass, linear and angular momentum
(APIC, Sec. 3.1), and reproduce affine velocity fields exactly.
"""
import math

import numpy as np
import pytest

import hot_scenes as hs
import oracle as O


def _random_points(rng, n=400, dx=0.07):
    origin = np.array([0.1, -0.2, 0.3])
    x = origin + rng.uniform(3.0, 9.0, size=(n, 3)) * dx
    return x, origin, dx


def test_bspline_closed_forms(rng):
    x, o, dx = _random_points(rng)
    W, G, nodes, xip = O.stencil(x, o, dx)
    xi = o + nodes * dx
    assert np.allclose(W.sum(1), 1.0, atol=1e-14)
    assert np.abs(np.einsum("pk,pka->pa", W, xip)).max() < 1e-14
    M2 = np.einsum("pk,pka,pkb->pab", W, xip, xip)
    assert np.abs(M2 - dx * dx / 4.0 * np.eye(3)).max() < 1e-15
    assert np.abs(G.sum(1)).max() < 1e-12
    I = np.einsum("pka,pkb->pab", xi, G)
    assert np.abs(I - np.eye(3)).max() < 1e-12
    # f in [1/2, 3/2) and weights non-negative
    _, w, _, f = O.bspline(x, o, dx)
    assert f.min() >= 0.5 and f.max() < 1.5 and w.min() >= 0.0


def test_bspline_gradient_is_derivative(rng):
    x, o, dx = _random_points(rng, n=50)
    h = 1e-7 * dx
    W, G, nodes, _ = O.stencil(x, o, dx)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        Wp, _, nodes_p, _ = O.stencil(x + e, o, dx)
        Wm, _, nodes_m, _ = O.stencil(x - e, o, dx)
        same = np.all(nodes_p == nodes, axis=(1, 2)) & np.all(nodes_m == nodes, axis=(1, 2))
        fd = (Wp - Wm) / (2 * h)
        # grad w_ip is the derivative with respect to the particle position
        assert np.abs(fd[same] - G[same][:, :, a]).max() < 1e-6 / dx


def test_binning_keys_and_stable_order():
    sc = hs.small_box(seed=3)
    keys, perm = O.bin_particles(sc)
    k = keys[perm]
    assert np.all(np.diff(k) >= 0)
    # ties keep input order
    same = np.diff(k) == 0
    assert np.all(np.diff(perm)[same] > 0)


def _prep(sc):
    return O.prepare(sc, 1e-3, 0.0)


def test_p2g_conserves_mass_momentum_angular_momentum():
    sc = hs.small_box(seed=11, gravity=(0, 0, 0), walls=None, noise=0.3, F_spread=0.1)
    st = _prep(sc)
    assert abs(st.m.sum() - st.mp.sum()) < 1e-13 * st.mp.sum()
    P_grid = (st.m[:, None] * st.vn).sum(0)
    P_part = (st.mp[:, None] * sc.v).sum(0)
    assert np.abs(P_grid - P_part).max() < 1e-13 * np.abs(P_part).max() + 1e-15
    xi = np.asarray(sc.origin) + st.lev0.coords * sc.dx
    L_grid = np.cross(xi, st.m[:, None] * st.vn).sum(0)
    # APIC: L = sum_p m_p (x_p x v_p + dx^2/4 eps_abg C_gb)
    epsC = np.stack([sc.C[:, 2, 1] - sc.C[:, 1, 2], sc.C[:, 0, 2] - sc.C[:, 2, 0],
                     sc.C[:, 1, 0] - sc.C[:, 0, 1]], -1)
    L_part = (st.mp[:, None] * (np.cross(sc.x, sc.v) + sc.dx ** 2 / 4.0 * epsC)).sum(0)
    assert np.abs(L_grid - L_part).max() < 1e-12 * np.abs(L_part).max()


def test_p2g_reproduces_affine_field():
    omega = np.array([0.4, -1.1, 0.7])
    sc = hs.small_box(seed=5, omega=tuple(omega), noise=0.0, walls=None)
    c = (np.array([2, 2, 2]) + np.array([5, 6, 5])) / 2.0 * sc.dx
    st = _prep(sc)
    xi = np.asarray(sc.origin) + st.lev0.coords * sc.dx
    exact = np.cross(omega, xi - c)
    assert np.abs(st.vn - exact).max() < 1e-13


def test_g2p_conserves_momentum_and_angular_momentum():
    sc = hs.small_box(seed=19, gravity=(0, 0, 0), walls=None, noise=0.3)
    st = _prep(sc)
    rng = np.random.Generator(np.random.PCG64(2))
    dv = rng.normal(size=st.vstar.shape) * 0.1
    out = O.g2p(st, dv)
    vgrid = st.vstar + dv
    P_grid = (st.m[:, None] * vgrid).sum(0)
    P_part = (st.mp[:, None] * out.v).sum(0)
    assert np.abs(P_grid - P_part).max() < 1e-13 * np.abs(P_grid).max()
    xi = np.asarray(sc.origin) + st.lev0.coords * sc.dx
    L_grid = np.cross(xi, st.m[:, None] * vgrid).sum(0)
    C = out.C
    epsC = np.stack([C[:, 2, 1] - C[:, 1, 2], C[:, 0, 2] - C[:, 2, 0], C[:, 1, 0] - C[:, 0, 1]], -1)
    L_part = (st.mp[:, None] * (np.cross(sc.x, out.v) + sc.dx ** 2 / 4.0 * epsC)).sum(0)
    assert np.abs(L_grid - L_part).max() < 1e-12 * np.abs(L_grid).max()


def test_deformation_update_matches_velocity_gradient_of_affine_field():
    # an affine grid velocity v_i = A x_i gives F^{n+1} = (I + dt A) F^n
    sc = hs.small_box(seed=23, walls=None, F_spread=0.2)
    st = _prep(sc)
    A = np.array([[0.1, -0.3, 0.2], [0.05, 0.0, -0.1], [0.3, 0.2, -0.2]])
    xi = np.asarray(sc.origin) + st.lev0.coords * sc.dx
    dv = xi @ A.T - st.vstar
    F = O.deformation(st, dv)
    assert np.abs(F - (np.eye(3) + st.dt * A) @ sc.F).max() < 1e-13


def test_massless_stencil_node():
    """A particle exactly where a weight vanishes (fractional position 1/2)
    reaches a node with zero weight and zero gradient.  If no other particle
    reaches that node it carries no mass: the transfer leaves it at v* = 0
    and xi = 0 instead of 0/0, mass and momentum sums still equal the
    particles', and the CN norm and the whole step stay finite."""
    sc = hs.small_box(seed=23, cells=(10, 10, 10), box_lo=(4, 4, 4), box_hi=(5, 5, 5),
                      walls=None, noise=0.0, levels=2)
    for f in ("x", "v", "F", "C", "vol0", "mat_id"):
        setattr(sc, f, np.ascontiguousarray(getattr(sc, f)[:1]))
    sc.x[0] = (np.array([4.5, 4.5, 4.5]) + np.array([0.25, 0.0, 0.5])) * sc.dx
    sc.F[0] = np.diag([1.1, 0.95, 1.05])
    t = (sc.x[0] - np.asarray(sc.origin)) / sc.dx
    frac = t - np.floor(t - 0.5)
    assert np.any(frac == 0.5)          # the set-up really sits on the plane
    st = _prep(sc)
    massless = st.m == 0.0
    assert massless.sum() == 9           # the 3x3 far layer of that axis
    assert np.all(st.vstar[massless] == 0.0) and np.all(st.xi[massless] == 0.0)
    assert np.all(np.isfinite(st.vstar)) and np.all(np.isfinite(st.xi))
    assert abs(st.m.sum() - st.mp.sum()) < 1e-13 * st.mp.sum()
    P_grid = (st.m[:, None] * st.vn).sum(0)
    assert np.abs(P_grid - st.mp[0] * sc.v[0]).max() < 1e-13 * (np.abs(sc.v[0]).max() * st.mp[0] + 1e-300)
    assert math.isfinite(O.cn_norm(st, np.zeros_like(st.vstar)))
    out, info = O.step(sc, dt=1e-3)
    assert info["converged"] and np.all(np.isfinite(out.x)) and np.all(np.isfinite(out.F))
