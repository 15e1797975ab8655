"""Pins for the oracle's Newton-Krylov baselines (Alg. 1): PN-PCG (diagonal
preconditioner) and PN-MGPCG (one V-cycle of the Galerkin hierarchy rebuilt
from each Newton iteration's Hessian).

* preconditioned CG reaches the dense solution of A x = b; it stops at the
  first iterate that meets its relative energy-norm rule (brute force over
  the iteration cap); with the identity preconditioner its k-th iterate is
  the A-norm minimiser over the k-th Krylov space (dense least squares);
* the adaptive tolerance k = min(1/2, sqrt(max(sqrt(r0^T M r0), tau))) in
  closed form at chosen values (Sec. 5.3);
* both Newton solvers driven to a tight tolerance land on the dense
  projected-Newton minimiser, as HOT does;
* the Newton step's linear solve is exact when the tolerance rule asks for
  it: with k forced tiny, one PN iteration from dv = 0 equals the dense
  projected Newton direction.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import hot_scenes as hs
import oracle as O
from test_oracle_solver import dense_newton, tiny


def spd(n, seed, cond=1e3):
    rng = np.random.Generator(np.random.PCG64(seed))
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.exp(rng.uniform(0.0, math.log(cond), size=n))
    return sp.csr_matrix((Q * ev) @ Q.T), rng


def test_precond_cg_reaches_the_dense_solution():
    A, rng = spd(40, 1)
    b = rng.normal(size=40)
    d = A.diagonal()
    x = O.precond_cg(A, lambda r: r / d, b, 1e-14, 1000)
    xs = np.linalg.solve(A.toarray(), b)
    assert np.abs(x - xs).max() <= 1e-9 * np.abs(xs).max()


@pytest.mark.parametrize("rel", [0.5, 0.1, 1e-3])
def test_precond_cg_stops_at_the_first_iterate_meeting_its_rule(rel):
    A, rng = spd(30, 2)
    b = rng.normal(size=30)
    d = A.diagonal()
    M = lambda r: r / d
    log = []
    O.precond_cg(A, M, b, rel, 1000, log=log)
    stop = rel * math.sqrt(b @ M(b))
    first = None
    for j in range(1, 200):
        x = O.precond_cg(A, M, b, 0.0, j)
        r = b - A @ x
        if math.sqrt(r @ M(r)) <= stop:
            first = j
            break
    # the truncated runs recompute the residual directly from A x
    assert first is not None and log[0] == first


def test_cg_iterates_minimise_the_energy_norm_over_krylov_spaces():
    A, rng = spd(25, 3, cond=50.0)
    Ad = A.toarray()
    b = rng.normal(size=25)
    xs = np.linalg.solve(Ad, b)
    L = np.linalg.cholesky(Ad)
    for k in (1, 3, 6):
        x = O.precond_cg(A, lambda r: r, b, 0.0, k)
        K = np.stack([np.linalg.matrix_power(Ad, j) @ b for j in range(k)], axis=1)
        Qk, _ = np.linalg.qr(K)
        # minimise ||L^T (Q c - xs)||_2 over c
        c, *_ = np.linalg.lstsq(L.T @ Qk, L.T @ xs, rcond=None)
        assert np.abs(x - Qk @ c).max() <= 1e-8 * np.abs(xs).max()


def test_inexact_tolerance_closed_form():
    assert O.inexact_tolerance(1e-4, 1e-6) == pytest.approx(0.1, rel=1e-14)
    assert O.inexact_tolerance(1.0, 1e-6) == 0.5
    assert O.inexact_tolerance(0.0, 1e-6) == pytest.approx(1e-3, rel=1e-14)
    assert O.inexact_tolerance(1e-16, 1e-6) == pytest.approx(1e-3, rel=1e-14)


@pytest.mark.parametrize("precond,model,walls", [("jacobi", 0, None), ("mg", 1, 2), ("mg", 0, 2)])
def test_newton_krylov_converged_step_matches_dense_newton(precond, model, walls):
    sc = tiny(71 + model, model=model, walls=walls)
    st = O.prepare(sc, 1e-2)
    dv, info = O.solve_pn(st, 1e-12, 2, precond, max_iters=200)
    assert info["converged"]
    ref = dense_newton(st)
    a, b = O.g2p(st, dv), O.g2p(st, ref)
    assert np.abs(a.v - b.v).max() < 1e-7 * np.abs(b.v).max()
    assert np.abs(a.x - b.x).max() < 1e-10


def test_exact_linear_solve_gives_the_newton_direction(monkeypatch):
    sc = tiny(75, model=0, walls=2)
    st = O.prepare(sc, 1e-2)
    n = st.lev0.n
    monkeypatch.setattr(O.hot_oracle, "inexact_tolerance", lambda r0Mr0, tau: 1e-15)
    dv, info = O.solve_pn(st, 0.0, 1, "jacobi", max_iters=1)
    assert info["log"]["alpha_halvings"] == [0]
    f = np.repeat(st.free, 3)
    H, nbr = O.hessian_slots(st)
    A = O.slots_to_csr(H, nbr, n).toarray()[np.ix_(f, f)]
    g = O.gradient(st, np.zeros((n, 3))).ravel()
    p = np.zeros(3 * n)
    p[f] = -sla.cho_solve(sla.cho_factor(A), g[f])
    assert np.abs(dv.ravel() - p).max() <= 1e-9 * np.abs(p).max()
