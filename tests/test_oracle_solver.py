"""Pins for the oracle's incremental potential, Hessian, V-cycle, L-BFGS,
line search, characteristic norm, plasticity and the converged step.

* g is the central finite difference of E (Eq. 1); the unprojected Hessian is
  the finite difference of g; the projected one is symmetric positive
  definite; translation invariance gives sum_i (g_i - m_i dv_i) = 0.
* With an exact coarse solve the V-cycle is linear, symmetric and positive
  definite on the free DOFs (Sec. 5.1); with many smoothing sweeps it
  approaches H^{-1} (the l1 smoother converges on SPD matrices).
* The two-loop recursion equals the dense BFGS inverse update started from
  the V-cycle matrix.
* HOT converged to a tight tolerance reaches the minimiser found by a dense
  projected Newton method with Cholesky solves (brute force on tiny grids).
* Accepted iterates decrease E; step lengths are powers of two.
* For one material the node-wise CN is a uniform scaling (Sec. 5.2).
* Von Mises return: unchanged below yield, on the yield surface after,
  volume kept, idempotent.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import hot_scenes as hs
import oracle as O


def tiny(seed, model=0, walls=None, **kw):
    base = dict(seed=seed, cells=(8, 8, 8), box_lo=(2, 3, 2), box_hi=(5, 6, 6), model=model,
                walls=walls, F_spread=0.15, noise=0.3, E=2e4, nu=0.32)
    base.update(kw)
    return hs.small_box(**base)


@pytest.mark.parametrize("model", [0, 1])
def test_gradient_is_energy_derivative(model):
    sc = tiny(51, model=model, walls=2)
    st = O.prepare(sc, 4e-3)
    rng = np.random.Generator(np.random.PCG64(9))
    dv = rng.normal(size=(st.lev0.n, 3)) * 0.05 * st.free[:, None]
    g = O.gradient(st, dv)
    h = 1e-6
    free = np.nonzero(st.free)[0][:12]
    for i in free:
        for c in range(3):
            e = np.zeros_like(dv)
            e[i, c] = h
            fd = (O.energy(st, dv + e) - O.energy(st, dv - e)) / (2 * h)
            assert abs(fd - g[i, c]) < 1e-6 * (abs(g).max() + 1e-12)
    assert np.all(g[st.fixed] == 0.0)


def test_momentum_balance_of_gradient():
    sc = tiny(53, walls=None, gravity=(0, 0, 0))
    st = O.prepare(sc, 4e-3)
    rng = np.random.Generator(np.random.PCG64(10))
    dv = rng.normal(size=(st.lev0.n, 3)) * 0.05
    g = O.gradient(st, dv)
    resid = (g - st.m[:, None] * dv).sum(0)
    assert np.abs(resid).max() < 1e-12 * np.abs(g).max()


@pytest.mark.parametrize("model", [0, 1])
def test_hessian_is_gradient_derivative(model):
    sc = tiny(55, model=model, walls=2)
    st = O.prepare(sc, 4e-3)
    n = st.lev0.n
    H, nbr = O.hessian_slots(st, project=False)
    A = O.slots_to_csr(H, nbr, n).toarray()
    h = 1e-6
    free = np.nonzero(st.free)[0][:8]
    for i in free:
        for c in range(3):
            e = np.zeros((n, 3))
            e[i, c] = h
            col = ((O.gradient(st, e) - O.gradient(st, -e)) / (2 * h)).ravel()
            fdofs = np.repeat(st.free, 3)
            assert np.abs(col[fdofs] - A[fdofs, 3 * i + c]).max() < 1e-6 * np.abs(A).max()


def test_projected_hessian_spd_and_symmetric():
    sc = tiny(57, walls=2, F_spread=0.4)
    st = O.prepare(sc, 1e-2)
    H, nbr = O.hessian_slots(st)
    A = O.slots_to_csr(H, nbr, st.lev0.n).toarray()
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0


def _hz(sc, dt, levels):
    st = O.prepare(sc, dt)
    H0, nbr0 = O.hessian_slots(st)
    return st, O.build_hierarchy(st, H0, nbr0, levels)


def _dense_V(hz, sweeps=1, smoother="l1jacobi"):
    Ac = hz.A[-1].toarray()
    solve = lambda b: np.linalg.solve(Ac, b)
    N = hz.A[0].shape[0]
    return np.stack([O.vcycle(hz, e, sweeps=sweeps, coarse_solver=solve, smoother=smoother)
                     for e in np.eye(N)], 1)


@pytest.mark.parametrize("smoother", O.SMOOTHERS)
def test_vcycle_symmetric_positive_definite_with_exact_coarse_solve(smoother):
    sc = tiny(59, walls=2, cells=(9, 9, 9), box_lo=(2, 2, 2), box_hi=(6, 6, 7))
    st, hz = _hz(sc, 1e-2, 3)
    V = _dense_V(hz, smoother=smoother)
    f = np.repeat(st.free, 3)
    Vf = V[np.ix_(f, f)]
    assert np.abs(Vf - Vf.T).max() < 1e-12 * np.abs(Vf).max()
    assert np.linalg.eigvalsh(0.5 * (Vf + Vf.T)).min() > 0
    assert np.all(V[~f] == 0.0)


@pytest.mark.parametrize("smoother,sweeps", [("sgs", 100), ("l1jacobi", 400)])
def test_vcycle_many_sweeps_approaches_inverse(smoother, sweeps):
    sc = tiny(61, walls=2)
    st, hz = _hz(sc, 1e-3, 2)
    V = _dense_V(hz, sweeps=sweeps, smoother=smoother)
    f = np.repeat(st.free, 3)
    A = hz.A[0].toarray()[np.ix_(f, f)]
    assert np.abs(V[np.ix_(f, f)] @ A - np.eye(f.sum())).max() < 1e-6


def test_two_loop_equals_dense_bfgs_inverse_update():
    sc = tiny(63, walls=2)
    st, hz = _hz(sc, 1e-2, 2)
    Ac = hz.A[-1].toarray()
    Vfun = lambda q: O.vcycle(hz, q.ravel(), coarse_solver=lambda b: np.linalg.solve(Ac, b)).reshape(q.shape)
    V = _dense_V(hz)
    rng = np.random.Generator(np.random.PCG64(4))
    n = st.lev0.n
    f = np.repeat(st.free, 3).astype(float)
    hist = []
    Hk = V.copy()
    A0 = hz.A[0].toarray()
    for _ in range(5):
        s = rng.normal(size=3 * n) * f
        y = A0 @ s + 0.1 * s
        rho = 1.0 / (y @ s)
        hist.append((s.reshape(n, 3), y.reshape(n, 3), rho))
        I = np.eye(3 * n)
        Hk = (I - rho * np.outer(s, y)) @ Hk @ (I - rho * np.outer(y, s)) + rho * np.outer(s, s)
    g = (rng.normal(size=3 * n) * f).reshape(n, 3)
    d = O.two_loop(hist, g, Vfun)
    assert np.abs(d.ravel() + Hk @ g.ravel()).max() < 1e-11 * np.abs(d).max()


def dense_newton(st, tol=1e-14, iters=60):
    """Projected Newton with dense Cholesky solves and Armijo backtracking."""
    n = st.lev0.n
    f = np.repeat(st.free, 3)
    dv = np.zeros((n, 3))
    E = O.energy(st, dv)
    for _ in range(iters):
        g = O.gradient(st, dv).ravel()
        if np.linalg.norm(g) <= tol * max(1.0, np.abs(st.m).max()):
            break
        H, nbr = O.hessian_slots(st, dv=dv)
        A = O.slots_to_csr(H, nbr, n).toarray()[np.ix_(f, f)]
        p = np.zeros(3 * n)
        p[f] = -sla.cho_solve(sla.cho_factor(A), g[f])
        a = 1.0
        for _ in range(40):
            Et = O.energy(st, dv + a * p.reshape(n, 3))
            if Et <= E + 1e-4 * a * (g @ p):
                break
            a *= 0.5
        dv = dv + a * p.reshape(n, 3)
        E = Et
    return dv


@pytest.mark.parametrize("model,walls,mats", [(0, None, 1), (1, 2, 1), (0, 2, 3)])
def test_converged_step_matches_dense_newton(model, walls, mats):
    """HOT driven to a tight tolerance lands on the dense Newton minimiser.

    The comparison is made on what the step outputs (particle velocities and
    positions after G2P).  Nodal dv at boundary nodes carrying ~1e-6 of the
    typical mass is poorly determined by the energy, and the FP64 energy
    differences in the Armijo test stop decreasing near a 1e-8 relative
    velocity error, so the bound is 1e-7 on velocities, 1e-8 on F and
    1e-10 m on positions."""
    sc = tiny(65 + model, model=model, walls=walls, n_mats=mats)
    dt = 1e-2
    st = O.prepare(sc, dt)
    H0, nbr0 = O.hessian_slots(st)
    hz = O.build_hierarchy(st, H0, nbr0, 2)
    # the l1 block-Jacobi cycle; the Gauss-Seidel cycle has its own pin
    dv, info = O.solve(st, hz, tol=1e-12, history=8, max_iters=300)
    ref = dense_newton(st)
    a, b = O.g2p(st, dv), O.g2p(st, ref)
    assert np.abs(a.v - b.v).max() < 1e-7 * np.abs(b.v).max()
    assert np.abs(a.x - b.x).max() < 1e-10
    assert np.abs(a.F - b.F).max() < 1e-8
    E = info["log"]["E"]
    assert all(y <= x + 1e-13 * abs(x) for x, y in zip(E, E[1:]))   # round-off in the total
    # only the final search may fail (energy differences at round-off level)
    assert all(h >= 0 for h in info["log"]["alpha_halvings"][:-1])
    assert info["iters"] > 5


def test_cn_uniform_scaling_single_material():
    sc = tiny(71, walls=2)
    st = O.prepare(sc, 3e-3)
    g = O.gradient(st, np.zeros((st.lev0.n, 3)))
    xi = O.cn_xi(st.mu[0], st.lam[0])
    assert np.allclose(st.xi, xi, rtol=1e-13)
    ref = np.linalg.norm(g) / (24.0 * sc.dx ** 2 * xi * st.dt)
    assert abs(O.cn_norm(st, g) - ref) < 1e-12 * ref


def test_cfg_style_step_converges_monotonically():
    sc = hs.small_box(seed=73, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(9, 8, 9), walls=2,
                      levels=3, n_mats=2)
    out, info = O.step(sc)
    assert info["converged"]
    E = info["log"]["E"]
    assert all(b <= a for a, b in zip(E, E[1:]))
    assert info["log"]["cn"][-1] <= sc.tol * math.sqrt(info["n_nodes"])


def test_von_mises_return_mapping():
    rng = np.random.Generator(np.random.PCG64(77))
    n = 300
    mu = np.full(n, 4e6)
    ys = np.full(n, 1e5)
    U = np.linalg.qr(rng.normal(size=(n, 3, 3)))[0]
    Vm = np.linalg.qr(rng.normal(size=(n, 3, 3)))[0]
    s = np.exp(rng.normal(size=(n, 3)) * 0.03)
    F = U @ (s[:, :, None] * np.swapaxes(Vm, 1, 2))
    Fp = O.von_mises(F, mu, ys)
    S = np.linalg.svd(Fp, compute_uv=False)
    eps = np.log(S)
    dev = eps - eps.mean(1, keepdims=True)
    lim = math.sqrt(2.0 / 3.0) * 1e5
    assert np.all(2 * mu * np.linalg.norm(dev, axis=1) <= lim * (1 + 1e-12))
    assert np.allclose(np.linalg.det(Fp), np.linalg.det(F), rtol=1e-12)
    eps0 = np.log(np.linalg.svd(F, compute_uv=False))
    below = 2 * mu * np.linalg.norm(eps0 - eps0.mean(1, keepdims=True), axis=1) <= lim
    assert below.sum() > 0 and (~below).sum() > 0
    assert np.array_equal(Fp[below], F[below])
    assert np.abs(O.von_mises(Fp, mu, ys) - Fp).max() < 1e-12
    assert np.array_equal(O.von_mises(F, mu, np.zeros(n)), F)


def test_snow_clamp():
    """Snow-type plastic flow: singular values of F clamped into [lo, hi]
    (Sec. 7, table of material parameters: [0.99, 1.001])."""
    rng = np.random.Generator(np.random.PCG64(79))
    n = 400
    U = np.linalg.qr(rng.normal(size=(n, 3, 3)))[0]
    V = np.linalg.qr(rng.normal(size=(n, 3, 3)))[0]
    U *= np.sign(np.linalg.det(U))[:, None, None]
    V *= np.sign(np.linalg.det(V))[:, None, None]
    s = np.exp(rng.normal(size=(n, 3)) * 0.01)
    F = U @ (s[:, :, None] * np.swapaxes(V, 1, 2))
    clamp = np.tile([0.99, 1.001], (n, 1))
    Fc = O.snow_clamp(F, clamp)
    # plain positive-singular-value reconstruction (det F > 0 here)
    Ur, Sr, Vtr = np.linalg.svd(F)
    ref = Ur @ (np.clip(Sr, 0.99, 1.001)[:, :, None] * Vtr)
    assert np.abs(Fc - ref).max() < 1e-13
    Sc = np.linalg.svd(Fc, compute_uv=False)
    assert Sc.min() >= 0.99 - 1e-13 and Sc.max() <= 1.001 + 1e-13
    inside = np.all((s >= 0.99) & (s <= 1.001), axis=1)
    assert inside.sum() > 0 and (~inside).sum() > 0
    assert np.abs(Fc[inside] - F[inside]).max() < 1e-14
    assert np.abs(O.snow_clamp(Fc, clamp) - Fc).max() < 1e-14
    # rotation equivariance, and no effect where no clamp is set
    R = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    R *= np.sign(np.linalg.det(R))
    assert np.abs(O.snow_clamp(R @ F, clamp) - R @ Fc).max() < 1e-13
    assert np.array_equal(O.snow_clamp(F, np.zeros((n, 2))), F)


# ---- gravity (applied to the grid velocity before the solve, v* = v + dt g)

def test_gravity_free_fall_of_unstressed_translating_body():
    """A body at rest shape (F = I) translating uniformly, with no walls,
    stays unstressed: the grid velocity field is uniform, so no deformation
    arises, dv = 0 is the minimiser, and grid-to-particle transfer returns
    every particle's velocity plus dt g exactly (up to rounding), with the
    positions advanced by dt times that velocity."""
    g = np.array([0.7, -9.8, 1.3])
    sc = hs.small_box(seed=61, cells=(10, 10, 10), box_lo=(3, 3, 3), box_hi=(7, 6, 7),
                      walls=None, omega=(0.0, 0.0, 0.0), noise=0.0, gravity=tuple(g), E=5e4)
    v0 = np.array([0.4, 0.1, -0.25])
    sc.v[:] = v0
    dt = 5e-3
    out, info = O.step(sc, dt=dt)
    assert info["converged"]
    assert np.abs(out.v - (v0 + dt * g)).max() <= 1e-13
    assert np.abs(out.x - (sc.x + dt * out.v)).max() <= 1e-15
    assert np.abs(out.F - np.eye(3)).max() <= 1e-13


@pytest.mark.parametrize("model", [0, 1])
def test_gravity_momentum_balance_of_converged_step(model):
    """Internal forces sum to zero (translation invariance), so without walls
    the particles' total momentum grows by exactly dt M g over one converged
    step, whatever the stress state; the residual left by the CN tolerance
    bounds the mismatch."""
    g = np.array([0.0, -9.8, 2.0])
    sc = tiny(63, model=model, walls=None, gravity=tuple(g))
    sc.tol = 1e-11
    dens = np.array([m["density"] for m in sc.materials])
    mp = dens[sc.mat_id] * sc.vol0
    dt = 4e-3
    out, info = O.step(sc, dt=dt)
    assert info["converged"]
    dp = mp @ out.v - mp @ sc.v
    want = dt * mp.sum() * g
    assert np.abs(dp - want).max() <= 1e-9 * np.abs(want).max()
