"""Pins for the oracle's elasticity: SVD, energy density, stress, stress
derivative and its positive-definite projection.

Pinned against: the LAPACK singular values; zero energy and stress under
rigid rotation; rotation invariance; central finite differences of psi and
of P; the linear-elasticity tensor at F = I; PSD-ness of the projection and
its identity on already-PSD tensors; the characteristic-norm stiffness
closed form (Sec. 5.2).
"""
import numpy as np
import pytest

import oracle as O


def rotations(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    a, b, c, d = q.T
    return np.stack([
        np.stack([a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)], -1),
        np.stack([2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)], -1),
        np.stack([2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d], -1),
    ], axis=1)


def random_F(rng, n, spread=0.3):
    U = rotations(rng, n)
    V = rotations(rng, n)
    s = rng.uniform(1 - spread, 1 + spread, size=(n, 3))
    return U @ (s[:, :, None] * np.swapaxes(V, 1, 2))


MODELS = [(0, "fcr"), (1, "nh")]


def params(n, model):
    E, nu = 3e4, 0.35
    mu, lam = O.lame(np.full(n, E), np.full(n, nu))
    return np.full(n, model, dtype=np.int32), mu, lam


def test_svd_signed(rng):
    F = random_F(rng, 200, 0.5)
    F[:50] = F[:50] @ np.diag([1.0, 1.0, -1.0])     # inverted
    U, S, V = O.svd_signed(F)
    assert np.abs(U @ (S[:, :, None] * np.swapaxes(V, 1, 2)) - F).max() < 1e-14
    assert np.allclose(np.linalg.det(U), 1.0) and np.allclose(np.linalg.det(V), 1.0)
    ref = np.linalg.svd(F, compute_uv=False)
    assert np.abs(np.abs(S) - ref).max() < 1e-14
    assert np.all(S[:, :2] > 0)
    assert np.all((S[:, 2] < 0) == (np.linalg.det(F) < 0))


@pytest.mark.parametrize("model,_", MODELS)
def test_rigid_rotation_zero_energy_and_stress(rng, model, _):
    R = rotations(rng, 100)
    m, mu, lam = params(100, model)
    assert np.abs(O.psi(R, m, mu, lam)).max() < 1e-9
    assert np.abs(O.piola(R, m, mu, lam)).max() < 1e-9 * mu[0]


@pytest.mark.parametrize("model,_", MODELS)
def test_rotation_invariance(rng, model, _):
    F = random_F(rng, 100)
    Q = rotations(rng, 100)
    m, mu, lam = params(100, model)
    a, b = O.psi(F, m, mu, lam), O.psi(Q @ F, m, mu, lam)
    assert np.abs(a - b).max() < 1e-10 * np.abs(a).max()


@pytest.mark.parametrize("model,_", MODELS)
def test_piola_is_energy_derivative(rng, model, _):
    F = random_F(rng, 40)
    m, mu, lam = params(40, model)
    P = O.piola(F, m, mu, lam)
    h = 1e-6
    fd = np.zeros_like(F)
    for a in range(3):
        for b in range(3):
            E = np.zeros((3, 3))
            E[a, b] = h
            fd[:, a, b] = (O.psi(F + E, m, mu, lam) - O.psi(F - E, m, mu, lam)) / (2 * h)
    assert np.abs(fd - P).max() < 1e-7 * np.abs(P).max()


@pytest.mark.parametrize("model,_", MODELS)
def test_stress_derivative_matches_fd_of_piola(rng, model, _):
    F = random_F(rng, 30, 0.4)
    F[:5] = F[:5] @ np.diag([1.0, 1.0, 1.0])
    m, mu, lam = params(30, model)
    C = O.dPdF(F, m, mu, lam, project=False)
    h = 1e-6
    fd = np.zeros((30, 9, 9))
    for d in range(3):
        for e in range(3):
            E = np.zeros((3, 3))
            E[d, e] = h
            dP = (O.piola(F + E, m, mu, lam) - O.piola(F - E, m, mu, lam)) / (2 * h)
            fd[:, :, 3 * d + e] = dP.reshape(30, 9)
    assert np.abs(fd - C).max() < 1e-6 * np.abs(C).max()
    assert np.abs(C - np.swapaxes(C, 1, 2)).max() < 1e-9 * np.abs(C).max()


@pytest.mark.parametrize("model,_", MODELS)
def test_stress_derivative_at_identity_is_linear_elasticity(model, _):
    m, mu, lam = params(1, model)
    C = O.dPdF(np.eye(3)[None], m, mu, lam, project=True)[0]
    ref = np.zeros((3, 3, 3, 3))
    d = np.eye(3)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    ref[i, j, k, l] = mu[0] * (d[i, k] * d[j, l] + d[i, l] * d[j, k]) + lam[0] * d[i, j] * d[k, l]
    assert np.abs(C - ref.reshape(9, 9)).max() < 1e-10 * mu[0]


@pytest.mark.parametrize("model,_", MODELS)
def test_projection_is_psd_and_identity_on_psd(rng, model, _):
    F = random_F(rng, 200, 0.6)
    m, mu, lam = params(200, model)
    Cp = O.dPdF(F, m, mu, lam, project=True)
    Cu = O.dPdF(F, m, mu, lam, project=False)
    ev_p = np.linalg.eigvalsh(Cp)
    scale = np.abs(ev_p).max(axis=1)
    assert np.all(ev_p.min(axis=1) >= -1e-12 * scale)
    ev_u = np.linalg.eigvalsh(Cu)
    psd = ev_u.min(axis=1) >= 0
    assert psd.sum() > 0 and (~psd).sum() > 0
    assert np.abs(Cp[psd] - Cu[psd]).max() < 1e-10 * scale.max()
    # projection = nearest PSD matrix: eigen-clamp of the unprojected tensor
    w, Q = np.linalg.eigh(Cu)
    ref = Q @ (np.maximum(w, 0)[:, :, None] * np.swapaxes(Q, 1, 2))
    assert np.abs(ref - Cp).max() < 1e-9 * scale.max()


def test_cn_stiffness_closed_form():
    mu, lam = O.lame(np.array([1e5, 1e8]), np.array([0.3, 0.45]))
    # Frobenius norm of the diagonal-space block at sigma = (1,1,1)
    for model in (0, 1):
        A, _, _, _ = O.diag_space(np.ones((2, 3)), np.full(2, model), mu, lam)
        assert np.allclose(np.linalg.norm(A, axis=(1, 2)), O.cn_xi(mu, lam), rtol=1e-14)


# ---- Lame parameters, pinned by elasticity relations that do not restate
# the conversion: the bulk modulus and the inverse conversions, and the
# small-strain response of both energy densities to a uniaxial stress state.

LAME_CASES = [(1e4, 0.2), (1e5, 0.3), (3e6, 0.4), (1e8, 0.45), (2e5, -0.3)]


@pytest.mark.parametrize("E,nu", LAME_CASES)
def test_lame_against_moduli_relations(E, nu):
    mu, lam = (float(a) for a in O.lame(E, nu))
    # bulk modulus: lambda + 2 mu / 3 = E / (3 (1 - 2 nu))
    assert abs((lam + 2.0 * mu / 3.0) - E / (3.0 * (1.0 - 2.0 * nu))) <= 1e-13 * E / (1 - 2 * nu)
    # the inverse relations give back E and nu
    assert abs(mu * (3.0 * lam + 2.0 * mu) / (lam + mu) - E) <= 1e-13 * E
    assert abs(lam / (2.0 * (lam + mu)) - nu) <= 1e-13
    # P-wave modulus lambda + 2 mu = E (1 - nu) / ((1 + nu)(1 - 2 nu))
    assert abs((lam + 2.0 * mu) - E * (1 - nu) / ((1 + nu) * (1 - 2 * nu))) <= 1e-13 * E * 10


@pytest.mark.parametrize("model,_", MODELS)
@pytest.mark.parametrize("E,nu", LAME_CASES[:4])
def test_uniaxial_stress_gives_youngs_modulus_and_poisson_ratio(model, _, E, nu):
    """A bar stretched by a small strain e along x and contracted by nu e
    across carries, to first order, stress E e along x and no stress across
    (the definition of E and nu).  Both energy densities reduce to linear
    elasticity at small strain, so their P (through O.lame) must show it."""
    e = 1e-7
    F = np.diag([1.0 + e, 1.0 - nu * e, 1.0 - nu * e])[None]
    mu, lam = O.lame(np.array([E]), np.array([nu]))
    P = O.piola(F, np.array([model], dtype=np.int32), mu, lam)[0]
    assert abs(P[0, 0] - E * e) <= 1e-5 * E * e
    assert abs(P[1, 1]) <= 1e-5 * E * e and abs(P[2, 2]) <= 1e-5 * E * e
    assert np.abs(P - np.diag(np.diag(P))).max() <= 1e-9 * E * e
