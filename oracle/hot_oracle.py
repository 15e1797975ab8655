"""HOT implicit MPM step, CPU FP64 oracle (test infrastructure only).

Every function cites the passage of the paper (arXiv 1911.07913) it follows.
Where the paper is silent the reading used is stated in the docstring; the
same readings are listed in the repository design notes.

Nothing here is blocked, fused or reordered for speed: per-particle
quantities are computed with vectorised numpy over particles, scatters use
``np.bincount``, sparse products use scipy, SVD/eigen/inverse use LAPACK
(library primitives).  Parity status of each function: pinned by the
``-m "not gpu"`` tests in ``tests/test_oracle_*.py`` (B-spline identities,
material finite differences and closed forms, pattern counts in closed form,
Galerkin vs dense products and vs the composite-kernel re-discretisation,
the quadratic embedding's weight moments and Galerkin energy identity,
V-cycle symmetry and exactness, two-loop vs dense BFGS, converged step vs a
dense projected-Newton minimiser, boundary conditions and the time-step rule
in closed form, l1 block-Jacobi special cases and contraction, coarsest PCG
vs the brute-force Krylov minimiser).  Whole-trajectory values are parity
unpinned beyond these pieces: the paper prints no worked example.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

# --------------------------------------------------------------------------
# Material parameters
# --------------------------------------------------------------------------


def lame(E, nu):
    """Lame parameters from Young's modulus and Poisson ratio (standard)."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def particle_materials(scene):
    """Per-particle (model, mu, lambda, density, yield) arrays (the snow
    clamp interval comes from ``particle_snow_clamp``)."""
    mats = scene.materials
    mid = scene.mat_id
    model = np.array([m["model"] for m in mats], dtype=np.int32)[mid]
    E = np.array([m["E"] for m in mats])[mid]
    nu = np.array([m["nu"] for m in mats])[mid]
    rho = np.array([m["density"] for m in mats])[mid]
    ys = np.array([m["yield_stress"] for m in mats])[mid]
    mu, lam = lame(E, nu)
    return model, mu, lam, rho, ys


def particle_snow_clamp(scene):
    """Per-particle snow clamp interval [lo, hi] ((0, 0): none)."""
    c = np.array([m.get("snow_clamp", (0.0, 0.0)) for m in scene.materials], dtype=np.float64)
    return c[scene.mat_id]


def cn_xi(mu, lam):
    """Per-particle stiffness scale of the characteristic norm (Sec. 5.2).

    The stress derivative in diagonal space at the undeformed state is
    2*mu*I + lambda*1 1^T for both elastic models; its Frobenius norm is used.
    """
    return np.sqrt(3.0 * (2.0 * mu + lam) ** 2 + 6.0 * lam ** 2)


# --------------------------------------------------------------------------
# Quadratic B-spline transfer kernel (Sec. 6, "Sparse matrix storage")
# --------------------------------------------------------------------------

OFFS = np.array([[kx, ky, kz] for kz in range(3) for ky in range(3) for kx in range(3)],
                dtype=np.int64)  # 27 stencil offsets, x fastest


def bspline(x, origin, dx):
    """Base node, per-axis weights and weight derivatives.

    Nodes sit at origin + i*dx.  base = floor((x - o)/dx - 1/2); f = (x-o)/dx -
    base lies in [1/2, 3/2).  Returns base (n,3) int64, w (n,3,3) and dw
    (n,3,3) indexed [particle, axis, offset 0..2].
    """
    t = (x - np.asarray(origin)) / dx
    base = np.floor(t - 0.5).astype(np.int64)
    f = t - base
    w = np.stack([0.5 * (1.5 - f) ** 2, 0.75 - (f - 1.0) ** 2, 0.5 * (f - 0.5) ** 2], axis=-1)
    dw = np.stack([(f - 1.5) / dx, -2.0 * (f - 1.0) / dx, (f - 0.5) / dx], axis=-1)
    return base, w, dw, f


def stencil(x, origin, dx):
    """Weights w_ip (n,27), gradients grad w_ip (n,27,3), node coords (n,27,3)
    and node-minus-particle offsets x_i - x_p (n,27,3) over the 27 nodes."""
    base, w, dw, f = bspline(x, origin, dx)
    kx, ky, kz = OFFS[:, 0], OFFS[:, 1], OFFS[:, 2]
    wx, wy, wz = w[:, 0, kx], w[:, 1, ky], w[:, 2, kz]
    dwx, dwy, dwz = dw[:, 0, kx], dw[:, 1, ky], dw[:, 2, kz]
    W = wx * wy * wz
    G = np.stack([dwx * wy * wz, wx * dwy * wz, wx * wy * dwz], axis=-1)
    nodes = base[:, None, :] + OFFS[None, :, :]
    xip = (OFFS[None, :, :] - f[:, None, :]) * dx
    return W, G, nodes, xip


# --------------------------------------------------------------------------
# Grid bookkeeping: active nodes and sparsity (Sec. 3.1, Sec. 4.2, Sec. 6)
# --------------------------------------------------------------------------


def node_dims(scene):
    return np.array(scene.grid_cells, dtype=np.int64) + 1


def linear(coords, dims):
    coords = np.asarray(coords, dtype=np.int64)
    return coords[..., 0] + dims[0] * (coords[..., 1] + dims[1] * coords[..., 2])


def unlinear(lin, dims):
    lin = np.asarray(lin, dtype=np.int64)
    return np.stack([lin % dims[0], (lin // dims[0]) % dims[1], lin // (dims[0] * dims[1])], -1)


def bin_particles(scene):
    """Binning key = linear index of the base node; stable sort (Sec. 3.1: the
    active grid is found by traversing particles).  Returns keys and the
    stable permutation (ties keep input order)."""
    base, _, _, _ = bspline(scene.x, scene.origin, scene.dx)
    keys = linear(base, node_dims(scene))
    perm = np.argsort(keys, kind="stable")
    return keys, perm


SLOT_OFFS = np.array([[dx, dy, dz] for dz in range(-2, 3) for dy in range(-2, 3)
                      for dx in range(-2, 3)], dtype=np.int64)  # 125 offsets, x fastest


def slot_of(delta):
    d = np.asarray(delta) + 2
    return d[..., 0] + 5 * d[..., 1] + 25 * d[..., 2]


class Level:
    """One level of the hierarchy: node coordinates, pattern, matrix."""

    def __init__(self, lin, dims):
        self.lin = np.asarray(lin, dtype=np.int64)          # sorted linear indices
        self.dims = np.asarray(dims, dtype=np.int64)
        self.coords = unlinear(self.lin, self.dims)
        self.n = len(self.lin)
        self.index = {}  # built lazily

    def lookup(self, lin):
        """Map linear indices to compact indices (-1 if inactive)."""
        lin = np.asarray(lin, dtype=np.int64)
        pos = np.searchsorted(self.lin, lin)
        pos = np.minimum(pos, self.n - 1)
        ok = self.lin[pos] == lin
        return np.where(ok, pos, -1)


def active_fine_nodes(scene):
    """Active fine nodes = union over particles of base + {0,1,2}^3, sorted by
    linear index (the changing sparse grid, Sec. 3.1)."""
    base, _, _, _ = bspline(scene.x, scene.origin, scene.dx)
    dims = node_dims(scene)
    nodes = base[:, None, :] + OFFS[None, :, :]
    lin = np.unique(linear(nodes, dims).ravel())
    return Level(lin, dims)


def fine_pattern(scene, lev):
    """Symbolic level-0 pattern (n, 125) bool: block (i, j) present iff some
    particle's 27-node stencil holds both i and j (Sec. 6: at most 5^d blocks
    per row)."""
    base, _, _, _ = bspline(scene.x, scene.origin, scene.dx)
    nodes = base[:, None, :] + OFFS[None, :, :]
    idx = lev.lookup(linear(nodes, lev.dims))                 # (np, 27)
    kl_slot = slot_of(OFFS[None, :, :] - OFFS[:, None, :])    # [k, l] -> slot of l - k
    flat = (idx[:, :, None] * 125 + kl_slot[None, :, :]).ravel()
    cnt = np.bincount(flat, minlength=lev.n * 125)
    return (cnt > 0).reshape(lev.n, 125)


def parents_1d(c):
    """Linear node embedding along one axis (Sec. 4.2: linear kernel).

    Coarse node J sits at fine node 2J.  An even fine coordinate embeds in one
    coarse node with weight 1, an odd one in its two neighbours with 1/2."""
    c = np.asarray(c, dtype=np.int64)
    even = (c % 2) == 0
    J0 = np.where(even, c // 2, (c - 1) // 2)
    J1 = np.where(even, c // 2, (c + 1) // 2)
    w0 = np.where(even, 1.0, 0.5)
    w1 = np.where(even, 0.0, 0.5)
    return J0, J1, w0, w1


def quad_bspline(t):
    """Quadratic B-spline N(t) of unit spacing, support |t| < 3/2."""
    a = np.abs(np.asarray(t, dtype=np.float64))
    return np.where(a <= 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def parents_1d_quadratic(c):
    """Quadratic node embedding along one axis, the alternative kernel of
    Sec. 4.2 (HOT-quadratic in Sec. 7): coarse node J sits at fine node 2J and
    weighs fine node c by the quadratic B-spline of the coarse spacing,
    N((c - 2J) / 2).  The parents are J = floor(c/2) - 1 .. floor(c/2) + 1;
    returns (J0, J1, J2, w0, w1, w2) (a weight is 0 where 2J is 3 or more
    fine nodes away)."""
    c = np.asarray(c, dtype=np.int64)
    h = c // 2
    Js = [h - 1, h, h + 1]
    ws = [quad_bspline((c - 2 * J) / 2.0) for J in Js]
    return (*Js, *ws)


def coarse_dims(dims, embedding="linear"):
    d = np.asarray(dims, dtype=np.int64)
    return d // 2 + 1 if embedding == "linear" else (d + 2) // 2 + 2


def prolongation(fine: Level, embedding="linear"):
    """Prolongation P (node level, n_fine x n_coarse) and the coarse level.

    P = R^T with R = (d x^0 / d x^1)^T (Sec. 4.1); entries are products of the
    per-axis embedding weights.  Linear (HOT, Sec. 4.2): 1 and 1/2, so 3^d
    nonzeros per coarse column (Sec. 6).  Quadratic (HOT-quadratic): the
    coarse quadratic B-spline at the fine nodes, 3/4, 1/2 and 1/8, 5^d
    nonzeros per coarse column; its coarse node K sits at fine node 2K - 2
    (the coarse grid keeps one node of margin below the fine one, so that
    nodes at the lower edge of every level keep all their parents)."""
    cd = coarse_dims(fine.dims, embedding)
    rows, cols, vals = [], [], []
    if embedding == "linear":
        per_axis = [parents_1d(fine.coords[:, a]) for a in range(3)]
        npar = 2
    elif embedding == "quadratic":
        per_axis = [parents_1d_quadratic(fine.coords[:, a] + 2) for a in range(3)]
        npar = 3
    else:
        raise ValueError(f"unknown embedding {embedding!r}")
    for sx in range(npar):
        for sy in range(npar):
            for sz in range(npar):
                J = np.stack([per_axis[0][sx], per_axis[1][sy], per_axis[2][sz]], -1)
                w = (per_axis[0][npar + sx] * per_axis[1][npar + sy] *
                     per_axis[2][npar + sz])
                keep = w > 0
                if np.any(keep):
                    Jk = J[keep]
                    if np.any(Jk < 0) or np.any(Jk >= cd[None, :]):
                        raise ValueError("a coarse parent falls outside the coarse grid")
                rows.append(np.nonzero(keep)[0])
                cols.append(linear(J[keep], cd))
                vals.append(w[keep])
    rows = np.concatenate(rows)
    clin = np.concatenate(cols)
    vals = np.concatenate(vals)
    coarse = Level(np.unique(clin), cd)
    P = sp.csr_matrix((vals, (rows, coarse.lookup(clin))), shape=(fine.n, coarse.n))
    return P, coarse


def coarse_pattern(fine: Level, fine_pat, P, coarse: Level):
    """Symbolic coarse pattern = structure of R * pattern * P (Sec. 4.1)."""
    r, s = np.nonzero(fine_pat)
    c = fine.lookup(linear(fine.coords[r] + SLOT_OFFS[s], fine.dims))
    A = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(fine.n, fine.n))
    S = sp.csr_matrix((np.ones(P.nnz), P.indices, P.indptr), shape=P.shape)
    C = (S.T @ A @ S).tocoo()
    delta = coarse.coords[C.col] - coarse.coords[C.row]
    assert np.all(np.abs(delta) <= 2), "coarse stencil exceeds 5^3 blocks"
    pat = np.zeros((coarse.n, 125), dtype=bool)
    pat[C.row, slot_of(delta)] = True
    return pat


# --------------------------------------------------------------------------
# Boundary conditions (Sec. 4.1: Dirichlet conditions resolved by projection)
# --------------------------------------------------------------------------


def bc_nodes(scene, lev: Level, t_end):
    """Constrained-node mask and prescribed velocities at the end of the step.

    Walls hold nodes within ``thickness`` of the grid boundary at rest; grips
    prescribe a rigid rotation about their axis inside their box; a sphere
    prescribes its velocity inside its position at t_end.  Later conditions in
    the list override earlier ones."""
    xi = np.asarray(scene.origin) + lev.coords * scene.dx
    cells = np.asarray(scene.grid_cells)
    mask = np.zeros(lev.n, dtype=bool)
    vbc = np.zeros((lev.n, 3))
    for bc in scene.bcs:
        p = np.asarray(bc["p"], dtype=np.float64)
        if bc["kind"] == 0:
            th = int(p[0])
            sel = np.any((lev.coords <= th) | (lev.coords >= cells - th), axis=1)
            mask |= sel
            vbc[sel] = 0.0
        elif bc["kind"] == 1:
            sel = np.all((xi >= p[0:3]) & (xi <= p[3:6]), axis=1)
            a = p[9:12] / np.linalg.norm(p[9:12])
            mask |= sel
            vbc[sel] = p[12] * np.cross(a, xi[sel] - p[6:9])
        elif bc["kind"] == 2:
            c = p[0:3] + p[4:7] * t_end
            sel = np.sum((xi - c) ** 2, axis=1) <= p[3] ** 2
            mask |= sel
            vbc[sel] = p[4:7]
        else:
            raise ValueError("unknown boundary condition kind")
    return mask, vbc


def bc_max_speed(scene):
    """Largest speed any boundary condition can prescribe (for the time-step
    rule): grip corners' distance from the axis times |omega|; sphere speed."""
    s = 0.0
    for bc in scene.bcs:
        p = np.asarray(bc["p"], dtype=np.float64)
        if bc["kind"] == 1:
            a = p[9:12] / np.linalg.norm(p[9:12])
            corners = np.array([[p[3 * bx], p[3 * by + 1], p[3 * bz + 2]]
                                for bx in range(2) for by in range(2) for bz in range(2)])
            r = np.linalg.norm(np.cross(a, corners - p[6:9]), axis=1).max()
            s = max(s, abs(p[12]) * r)
        elif bc["kind"] == 2:
            s = max(s, float(np.linalg.norm(p[4:7])))
    return s


# --------------------------------------------------------------------------
# Elasticity: energy density, first Piola stress, projected stress derivative
# (fixed-corotated per Sec. 7.1; Neo-Hookean for the multi-bar workload)
# --------------------------------------------------------------------------


def svd_signed(F):
    """SVD with U, V proper rotations; a negative determinant moves into the
    last (smallest) singular value (LAPACK routine)."""
    U, S, Vt = np.linalg.svd(F)
    V = np.swapaxes(Vt, -1, -2).copy()
    U = U.copy()
    S = S.copy()
    dU = np.linalg.det(U) < 0
    dV = np.linalg.det(V) < 0
    U[dU, :, 2] *= -1.0
    S[dU, 2] *= -1.0
    V[dV, :, 2] *= -1.0
    S[dV, 2] *= -1.0
    return U, S, V


def cofactor(F):
    """cof(F) = det(F) F^{-T}, written with column cross products."""
    c0, c1, c2 = F[..., :, 0], F[..., :, 1], F[..., :, 2]
    return np.stack([np.cross(c1, c2), np.cross(c2, c0), np.cross(c0, c1)], axis=-1)


def psi(F, model, mu, lam):
    """Energy density.  FCR: mu ||F - R||^2 + lambda/2 (J-1)^2 with R the
    rotation of the polar decomposition.  NH: mu/2 (tr F^T F - 3) - mu ln J +
    lambda/2 (ln J)^2, +inf for J <= 0."""
    U, S, V = svd_signed(F)
    R = U @ np.swapaxes(V, -1, -2)
    J = np.linalg.det(F)
    fcr = mu * np.sum((F - R) ** 2, axis=(-1, -2)) + 0.5 * lam * (J - 1.0) ** 2
    with np.errstate(invalid="ignore", divide="ignore"):
        lnJ = np.log(np.where(J > 0, J, 1.0))
        nh = 0.5 * mu * (np.sum(F * F, axis=(-1, -2)) - 3.0) - mu * lnJ + 0.5 * lam * lnJ ** 2
    nh = np.where(J > 0, nh, np.inf)
    return np.where(model == 0, fcr, nh)


def piola(F, model, mu, lam):
    """First Piola-Kirchhoff stress P = d psi / d F."""
    U, S, V = svd_signed(F)
    R = U @ np.swapaxes(V, -1, -2)
    J = np.linalg.det(F)
    cof = cofactor(F)
    m = mu[:, None, None]
    l = lam[:, None, None]
    fcr = 2.0 * m * (F - R) + l * (J - 1.0)[:, None, None] * cof
    with np.errstate(invalid="ignore", divide="ignore"):
        FinvT = cof / J[:, None, None]
        lnJ = np.log(np.where(J > 0, J, 1.0))[:, None, None]
    nh = m * (F - FinvT) + l * lnJ * FinvT
    return np.where((model == 0)[:, None, None], fcr, nh)


def diag_space(S, model, mu, lam):
    """Diagonal-space Hessian A = d^2 psi_hat / d sigma^2 (n,3,3) and, for the
    pairs (0,1), (0,2), (1,2), the eigenvalues of the 2x2 blocks on the
    symmetric and antisymmetric off-diagonal directions (n,3) each.  Closed
    forms without (sigma_i - sigma_j) divisions."""
    s = S
    J = s[:, 0] * s[:, 1] * s[:, 2]
    pairs = [(0, 1, 2), (0, 2, 1), (1, 2, 0)]
    n = s.shape[0]
    A = np.zeros((n, 3, 3))
    lam_sym = np.zeros((n, 3))
    lam_anti = np.zeros((n, 3))
    fcr = model == 0
    lnJ = np.log(np.where(J > 0, J, 1.0))
    for i in range(3):
        j, k = [a for a in range(3) if a != i]
        other = s[:, j] * s[:, k]
        A_fcr = 2.0 * mu + lam * other ** 2
        A_nh = mu + (mu + lam * (1.0 - lnJ)) / s[:, i] ** 2
        A[:, i, i] = np.where(fcr, A_fcr, A_nh)
    for q, (i, j, k) in enumerate(pairs):
        Aij_fcr = lam * s[:, k] * (2.0 * J - 1.0)
        Aij_nh = lam / (s[:, i] * s[:, j])
        A[:, i, j] = A[:, j, i] = np.where(fcr, Aij_fcr, Aij_nh)
        ssum = s[:, i] + s[:, j]
        ssum = np.where(np.abs(ssum) < 1e-12, np.where(ssum < 0, -1e-12, 1e-12), ssum)
        sym_fcr = 2.0 * mu - lam * (J - 1.0) * s[:, k]
        anti_fcr = 2.0 * mu - 4.0 * mu / ssum + lam * (J - 1.0) * s[:, k]
        t = (mu - lam * lnJ) / (s[:, i] * s[:, j])
        lam_sym[:, q] = np.where(fcr, sym_fcr, mu + t)
        lam_anti[:, q] = np.where(fcr, anti_fcr, mu - t)
    return A, lam_sym, lam_anti, pairs


def dPdF(F, model, mu, lam, project=True):
    """Stress derivative C[3g+b, 3d+e] = dP_gb / dF_de (n,9,9).

    Built from its eigensystem in the SVD frame; with ``project`` every
    negative eigenvalue is clamped to zero (positive-definite fix, cited in
    Sec. 2 and Alg. HOT's projectHessian)."""
    U, S, V = svd_signed(F)
    A, ls, la, pairs = diag_space(S, model, mu, lam)
    ev, Q = np.linalg.eigh(A)
    if project:
        ev = np.maximum(ev, 0.0)
        ls = np.maximum(ls, 0.0)
        la = np.maximum(la, 0.0)
    n = F.shape[0]
    C = np.zeros((n, 9, 9))
    Vt = np.swapaxes(V, -1, -2)
    for k in range(3):
        D = U @ (Q[:, :, k][:, :, None] * Vt)           # U diag(q_k) V^T
        d = D.reshape(n, 9)
        C += ev[:, k, None, None] * d[:, :, None] * d[:, None, :]
    r2 = 1.0 / math.sqrt(2.0)
    for q, (i, j, _) in enumerate(pairs):
        Eij = np.zeros((3, 3))
        Eij[i, j] = 1.0
        Eji = Eij.T
        for lamq, M in ((ls[:, q], (Eij + Eji) * r2), (la[:, q], (Eij - Eji) * r2)):
            D = U @ M @ Vt
            d = D.reshape(n, 9)
            C += lamq[:, None, None] * d[:, :, None] * d[:, None, :]
    return C


# --------------------------------------------------------------------------
# The implicit step
# --------------------------------------------------------------------------


class StepState:
    """Per-step quantities shared by the energy, gradient and Hessian."""
    pass


def prepare(scene, dt, t=0.0):
    """Binning, active grid, P2G with APIC and the CN field, gravity and
    boundary conditions (Sec. 3.1 P2G; Sec. 5.2 CN transfer).

    Gravity is applied to the grid velocity before the solve (v* = v + dt g)
    so that the incremental potential of Eq. 1 is written about v*; boundary
    velocities are written into v* so the initial iterate dv = 0 is feasible.
    """
    st = StepState()
    st.scene, st.dt, st.t = scene, dt, t
    st.model, st.mu, st.lam, rho, st.yield_stress = particle_materials(scene)
    st.mp = rho * scene.vol0
    st.Vp = scene.vol0
    st.lev0 = active_fine_nodes(scene)
    W, G, nodes, xip = stencil(scene.x, scene.origin, scene.dx)
    st.W, st.G, st.xip = W, G, xip
    st.idx = st.lev0.lookup(linear(nodes, st.lev0.dims))         # (np, 27)
    n = st.lev0.n
    mw = W * st.mp[:, None]
    st.m = np.bincount(st.idx.ravel(), weights=mw.ravel(), minlength=n)
    # APIC momentum: m_p (v_p + C_p (x_i - x_p))
    vapic = scene.v[:, None, :] + np.einsum("pab,pkb->pka", scene.C, xip)
    mom = np.stack([np.bincount(st.idx.ravel(), weights=(mw * vapic[:, :, a]).ravel(),
                                minlength=n) for a in range(3)], -1)
    xi_p = cn_xi(st.mu, st.lam)
    # A stencil node can receive no mass at all when every particle reaching
    # it sits where its weight vanishes (fractional position exactly 1/2 on
    # an axis): it carries no momentum equation, gets v* = 0 and xi = 0, and
    # its exactly zero Hessian diagonal constrains it (reading: nodes without
    # mass are outside the grid equations of the transfer, Sec. 3.1).
    has_m = st.m > 0.0
    m_safe = np.where(has_m, st.m, 1.0)
    xi_sum = np.bincount(st.idx.ravel(), weights=(mw * xi_p[:, None]).ravel(), minlength=n)
    st.xi = np.where(has_m, xi_sum / m_safe, 0.0)
    st.vn = np.where(has_m[:, None], mom / m_safe[:, None], 0.0)
    st.vstar = np.where(has_m[:, None], st.vn + dt * np.asarray(scene.gravity)[None, :], 0.0)
    st.fixed, vbc = bc_nodes(scene, st.lev0, t + dt)
    st.vstar[st.fixed] = vbc[st.fixed]
    st.free = ~st.fixed
    # a_ip = F_p^n^T grad w_ip (updated-Lagrangian derivative, Sec. 4.1 forces)
    st.a = np.einsum("pba,pkb->pka", scene.F, G)
    return st


def deformation(st, dv):
    """F_p(dv) = (I + dt sum_i (v*_i + dv_i) grad w_ip^T) F_p^n (Sec. 3.1)."""
    vel = (st.vstar + dv)[st.idx]                             # (np, 27, 3)
    gradv = np.einsum("pka,pkb->pab", vel, st.G)
    return (np.eye(3)[None] + st.dt * gradv) @ st.scene.F


def particle_psi(st, dv):
    return psi(deformation(st, dv), st.model, st.mu, st.lam)


def energy_terms(st, dv):
    """Per-particle V_p psi_p and per-node 1/2 m_i |dv_i|^2 of Eq. 1."""
    return st.Vp * particle_psi(st, dv), 0.5 * st.m * np.sum(dv * dv, axis=1)


def energy(st, dv):
    """Incremental potential E(dv), Eq. 1."""
    ep, en = energy_terms(st, dv)
    return float(np.sum(ep) + np.sum(en))


def gradient(st, dv):
    """g_i = m_i dv_i + dt sum_p V_p P_p F_p^n^T grad w_ip, projected onto the
    free DOFs (Sec. 4.1 nodal forces; Eq. 1)."""
    F = deformation(st, dv)
    P = piola(F, st.model, st.mu, st.lam) * st.Vp[:, None, None]
    contrib = np.einsum("pgb,pkb->pkg", P, st.a) * st.dt
    n = st.lev0.n
    g = st.m[:, None] * dv + np.stack(
        [np.bincount(st.idx.ravel(), weights=contrib[:, :, c].ravel(), minlength=n)
         for c in range(3)], -1)
    g[st.fixed] = 0.0
    return g


def hessian_slots(st, project=True, chunk=2048, dv=None):
    """Level-0 system matrix in 125-slot block form (n, 125, 3, 3).

    H_ij = m_i delta_ij I + dt^2 sum_p V_p a_ip^T C_p a_jp with C_p the
    (projected) stress derivative at dv = 0 (Alg. HOT initialisation:
    projectHessian at dv^1 = 0; other points only for tests).  Then Dirichlet projection: rows and columns
    of constrained nodes are zeroed and their diagonal set to m_i I."""
    n = st.lev0.n
    F0 = deformation(st, np.zeros((n, 3)) if dv is None else dv)
    kl_slot = slot_of(OFFS[None, :, :] - OFFS[:, None, :])     # [k, l]
    out = np.zeros((n * 125, 9))
    for s0 in range(0, st.scene.n, chunk):
        sl = slice(s0, s0 + chunk)
        C = dPdF(F0[sl], st.model[sl], st.mu[sl], st.lam[sl], project=project)
        C4 = C.reshape(-1, 3, 3, 3, 3)
        a = st.a[sl]
        Z = np.einsum("pkb,pgbde->pkgde", a, C4)
        blk = np.einsum("pkgde,ple->pklgd", Z, a)
        blk *= (st.dt ** 2 * st.Vp[sl])[:, None, None, None, None]
        flat = (st.idx[sl][:, :, None] * 125 + kl_slot[None, :, :]).ravel()
        blk = blk.reshape(-1, 9)
        for c in range(9):
            out[:, c] += np.bincount(flat, weights=blk[:, c], minlength=n * 125)
    H = out.reshape(n, 125, 3, 3)
    H[:, 62] += st.m[:, None, None] * np.eye(3)[None]
    # Dirichlet projection of rows and columns (Sec. 4.1)
    nbr = st.lev0.lookup(linear(st.lev0.coords[:, None, :] + SLOT_OFFS[None], st.lev0.dims))
    fixed_nbr = np.where(nbr >= 0, st.fixed[np.maximum(nbr, 0)], False)
    H[st.fixed] = 0.0
    H[fixed_nbr] = 0.0
    H[st.fixed, 62] = st.m[st.fixed, None, None] * np.eye(3)[None]
    return H, nbr


def slots_to_csr(H, nbr, n):
    """Expand a 125-slot block matrix to a scipy CSR over 3n DOFs."""
    r, s = np.nonzero(nbr >= 0)
    c = nbr[r, s]
    blk = H[r, s]                                              # (nnzb, 3, 3)
    rows = (3 * r[:, None, None] + np.arange(3)[None, :, None]) + 0 * np.arange(3)[None, None, :]
    cols = (3 * c[:, None, None] + np.arange(3)[None, None, :]) + 0 * np.arange(3)[None, :, None]
    return sp.csr_matrix((blk.ravel(), (rows.ravel(), cols.ravel())), shape=(3 * n, 3 * n))


def csr_to_slots(A, lev: Level):
    """Block-slot view (n, 125, 3, 3) of a CSR matrix over 3n DOFs."""
    C = A.tocoo()
    bi, bj = C.row // 3, C.col // 3
    delta = lev.coords[bj] - lev.coords[bi]
    assert np.all(np.abs(delta) <= 2)
    H = np.zeros((lev.n, 125, 3, 3))
    np.add.at(H, (bi, slot_of(delta), C.row % 3, C.col % 3), C.data)
    return H


class Hierarchy:
    """Levels, Galerkin matrices, prolongations and smoother blocks."""
    pass


def build_hierarchy(st, H0_slots, nbr0, levels, project_pattern=True, embedding="linear"):
    """Galerkin hierarchy H^{m+1} = P~^T H^m P~ (Eq. buildMultigrid, Sec. 4.1)
    with P~ = Pi P: rows of constrained fine DOFs are removed before the
    product so Dirichlet conditions hold at every level.  A coarse DOF whose
    diagonal comes out exactly zero has no free fine DOF below it; it is
    constrained at its level (diagonal set to 1).  embedding: "linear" (HOT)
    or "quadratic" (HOT-quadratic, whose coarse stencils reach 3 nodes, so
    no 125-slot patterns are formed)."""
    if embedding != "linear":
        project_pattern = False
    hz = Hierarchy()
    lev = st.lev0
    hz.levels = [lev]
    hz.A = [slots_to_csr(H0_slots, nbr0, lev.n)]
    free_dof = np.repeat(st.free, 3).astype(np.float64)
    d0 = hz.A[0].diagonal()
    zero0 = (d0 == 0.0)
    if np.any(zero0):
        hz.A[0] = hz.A[0] + sp.diags(zero0.astype(np.float64))
        free_dof = free_dof * (~zero0)
    hz.free = [free_dof]
    hz.P = []
    hz.Pnode = []
    hz.patterns = [fine_pattern(st.scene, lev)] if project_pattern else [None]
    for m in range(levels - 1):
        Pn, coarse = prolongation(lev, embedding)
        Pd = sp.kron(Pn, sp.identity(3), format="csr")
        Pt = sp.diags(hz.free[m]) @ Pd
        Ac = (Pt.T @ hz.A[m] @ Pt).tocsr()
        d = Ac.diagonal()
        zero = d == 0.0
        Ac = Ac + sp.diags(zero.astype(np.float64))
        hz.free.append((~zero).astype(np.float64))
        hz.P.append(Pt.tocsr())
        hz.Pnode.append(Pn)
        if project_pattern:
            hz.patterns.append(coarse_pattern(lev, hz.patterns[-1], Pn, coarse))
        hz.A.append(Ac.tocsr())
        hz.levels.append(coarse)
        lev = coarse
    hz.Dinv = [l1_block_jacobi_inverse(A) for A in hz.A]
    hz.diag = [A.diagonal() for A in hz.A]
    return hz


def l1_block_jacobi_inverse(A):
    """Inverse of the l1 block-Jacobi smoother matrix (as a block-diagonal CSR).

    D~_i = H_ii + diag_g( sum_{j != i} sum_d |(H_ij)_gd| ): the 3x3 diagonal
    block plus, on its diagonal, the l1 sums of the row outside the block.
    (The paper smooths with colored symmetric Gauss-Seidel; block-Jacobi with
    this l1 augmentation is the substitute used here: it needs no weight and
    converges for SPD matrices.)"""
    n = A.shape[0] // 3
    C = A.tocoo()
    bi, bj = C.row // 3, C.col // 3
    off = bi != bj
    l1 = np.bincount(C.row[off], weights=np.abs(C.data[off]), minlength=3 * n)
    D = np.zeros((n, 3, 3))
    on = ~off
    np.add.at(D, (bi[on], C.row[on] % 3, C.col[on] % 3), C.data[on])
    D[:, np.arange(3), np.arange(3)] += l1.reshape(n, 3)
    Dinv = np.linalg.inv(D)
    rows = (3 * np.arange(n)[:, None, None] + np.arange(3)[None, :, None]).repeat(3, 2)
    cols = (3 * np.arange(n)[:, None, None] + np.arange(3)[None, None, :]).repeat(3, 1)
    return sp.csr_matrix((Dinv.ravel(), (rows.ravel(), cols.ravel())), shape=A.shape)


SMOOTHERS = ("l1jacobi", "sgs")
N_COLORS = 27


def node_colors(lev):
    """Colour of every node of a level for the coloured Gauss-Seidel smoother
    (Alg. V-cycle; Sec. 5.3 names coloured symmetric Gauss-Seidel, Sec. 8
    parallelises it by colouring): (x mod 3) + 3 (y mod 3) + 9 (z mod 3) of
    the node's grid coordinate.  A block row couples nodes at most 2 apart
    per axis (125 slots), so two distinct nodes of one colour are never
    coupled and a colour's nodes can all be updated at once."""
    c = np.mod(lev.coords, 3)
    return c[:, 0] + 3 * c[:, 1] + 9 * c[:, 2]


def sgs_setup(A, lev):
    """Per colour: its nodes, their DOF rows, the off-diagonal-block part of
    those rows of A and the inverses of their 3x3 diagonal blocks."""
    n = lev.n
    C = A.tocoo()
    bi, bj = C.row // 3, C.col // 3
    on = bi == bj
    D = np.zeros((n, 3, 3))
    np.add.at(D, (bi[on], C.row[on] % 3, C.col[on] % 3), C.data[on])
    Aoff = sp.csr_matrix((C.data[~on], (C.row[~on], C.col[~on])), shape=A.shape)
    col = node_colors(lev)
    out = []
    for c in range(N_COLORS):
        nodes = np.nonzero(col == c)[0]
        dofs = (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()
        out.append((nodes, dofs, Aoff[dofs], np.linalg.inv(D[nodes])))
    return out


def sgs(setup, b, u, sweeps=1):
    """Symmetric block Gauss-Seidel smoothing (Alg. V-cycle): a forward pass
    over the colours 0..26, then a backward pass 26..0.  Within a colour every
    node i takes u_i = H_ii^{-1} (b_i - sum_{j != i} H_ij u_j) with the
    current u (the colour's nodes do not see each other)."""
    u = u.copy()
    for _ in range(sweeps):
        for order in (range(N_COLORS), range(N_COLORS - 1, -1, -1)):
            for c in order:
                nodes, dofs, Aoff_c, Dinv_c = setup[c]
                if len(nodes) == 0:
                    continue
                r = (b[dofs] - Aoff_c @ u).reshape(-1, 3)
                u[dofs] = np.einsum("kab,kb->ka", Dinv_c, r).ravel()
    return u


def sgs_data(hz):
    """The coloured Gauss-Seidel set-up of every smoothed level (cached)."""
    if getattr(hz, "sgs", None) is None:
        hz.sgs = [sgs_setup(hz.A[m], hz.levels[m]) for m in range(len(hz.A) - 1)]
    return hz.sgs


def coarse_pcg(A, diag, b, rel=0.5, max_iter=500, log=None):
    """Jacobi-preconditioned CG on the coarsest level (Alg. V-cycle), from
    x0 = 0, stopped once sqrt(r^T D^{-1} r) <= rel * sqrt(b^T D^{-1} b) with D
    the diagonal of the level matrix (Sec. 5.3, inexact coarse solve)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = r / diag
    rz = float(r @ z)
    stop = rel * math.sqrt(max(rz, 0.0))
    it = 0
    if rz > 0.0:
        p = z.copy()
        while it < max_iter:
            q = A @ p
            alpha = rz / float(p @ q)
            x += alpha * p
            r -= alpha * q
            z = r / diag
            rz_new = float(r @ z)
            it += 1
            if math.sqrt(max(rz_new, 0.0)) <= stop:
                break
            beta = rz_new / rz
            rz = rz_new
            p = z + beta * p
    if log is not None:
        log.append(it)
    return x


def vcycle(hz, b, sweeps=1, coarse_solver=None, log=None, smoother="l1jacobi"):
    """Multigrid V-cycle (Alg. V-cycle) with l1 block-Jacobi smoothing, or with
    the paper's coloured symmetric block Gauss-Seidel (smoother="sgs").

    Down: u^m = smooth(0, b^m); b^{m+1} = P~^T (b^m - H^m u^m).  Coarsest: PCG
    to relative 1/2.  Up: u^m += P~ u^{m+1}; u^m = smooth(u^m, b^m)."""
    assert smoother in SMOOTHERS
    M = len(hz.A)
    us, bs = [None] * M, [None] * M
    bs[0] = b * hz.free[0]
    gs = sgs_data(hz) if smoother == "sgs" else None
    for m in range(M - 1):
        u = np.zeros_like(bs[m])
        if gs is not None:
            u = sgs(gs[m], bs[m], u, sweeps)
        else:
            for _ in range(sweeps):
                u = u + hz.Dinv[m] @ (bs[m] - hz.A[m] @ u)
        us[m] = u
        bs[m + 1] = hz.P[m].T @ (bs[m] - hz.A[m] @ u)
    if coarse_solver is None:
        us[M - 1] = coarse_pcg(hz.A[M - 1], hz.diag[M - 1], bs[M - 1], log=log)
    else:
        us[M - 1] = coarse_solver(bs[M - 1])
    us[M - 1] = us[M - 1] * hz.free[M - 1]
    for m in range(M - 2, -1, -1):
        u = us[m] + hz.P[m] @ us[m + 1]
        if gs is not None:
            u = sgs(gs[m], bs[m], u, sweeps)
        else:
            for _ in range(sweeps):
                u = u + hz.Dinv[m] @ (bs[m] - hz.A[m] @ u)
        us[m] = u * hz.free[m]
    return us[0]


def cn_norm(st, g):
    """||g_hat||_2 with g_hat_i = g_i / (24 dx^2 xi_i dt) (Eq. nodewiseCN),
    over the nodes that carry mass (xi_i > 0; see prepare)."""
    live = st.xi > 0.0
    scale = 24.0 * st.scene.dx ** 2 * st.xi[live] * st.dt
    return float(math.sqrt(np.sum((g[live] / scale[:, None]) ** 2)))


def two_loop(hist, g, apply_H0):
    """L-BFGS two-loop recursion with the V-cycle as initial inverse Hessian
    (Alg. HOT).  ``hist`` is a list of (s, y, rho), oldest first."""
    q = -g
    alphas = []
    for s, y, rho in reversed(hist):
        al = rho * float(np.sum(s * q))
        q = q - al * y
        alphas.append(al)
    alphas.reverse()
    r = apply_H0(q)
    for (s, y, rho), al in zip(hist, alphas):
        beta = rho * float(np.sum(y * r))
        r = r + (al - beta) * s
    return r


def solve(st, hz, tol, history, max_iters=500, sweeps=1, c1=1e-4, max_halvings=30,
          smoother="l1jacobi"):
    """HOT quasi-Newton solve (Alg. HOT).

    dv^1 = 0; while the CN-scaled gradient norm exceeds eps*sqrt(n): two-loop
    direction with the V-cycle as H0, backtracking line search from alpha = 1
    (Armijo, c1 = 1e-4, halving, at most 30 halvings; the energy change is
    summed as per-particle and per-node differences), secant pair stored when
    y^T s > 1e-12 |y||s|.  A non-descent direction clears the history and
    retries with the bare V-cycle, then with -D~^{-1} g."""
    n = st.lev0.n
    dv = np.zeros((n, 3))
    g = gradient(st, dv)
    ep, en = energy_terms(st, dv)
    hist = []
    log = dict(cn=[], alpha_halvings=[], skipped=[], cg=[], fallback=[], E=[])
    thresh = tol * math.sqrt(n)
    cn = cn_norm(st, g)
    log["cn"].append(cn)
    log["E"].append(float(np.sum(ep) + np.sum(en)))
    it = 0
    converged = cn <= thresh
    while not converged and it < max_iters:
        cg_log = []
        V = lambda q: vcycle(hz, q.ravel(), sweeps=sweeps, log=cg_log,
                             smoother=smoother).reshape(n, 3)
        p = two_loop(hist, g, V)
        fb = 0
        if float(np.sum(p * g)) >= 0.0:
            hist = []
            p = V(-g)
            fb = 1
            if float(np.sum(p * g)) >= 0.0:
                p = -(hz.Dinv[0] @ g.ravel()).reshape(n, 3)
                fb = 2
        gp = float(np.sum(g * p))
        alpha = 1.0
        accepted = False
        halvings = 0
        for halvings in range(max_halvings + 1):
            dv_t = dv + alpha * p
            ep_t, en_t = energy_terms(st, dv_t)
            dE = float(np.sum(ep_t - ep) + np.sum(en_t - en))
            if np.isfinite(dE) and dE <= c1 * alpha * gp:
                accepted = True
                break
            alpha *= 0.5
        log["alpha_halvings"].append(halvings if accepted else -1)
        log["cg"].append(cg_log)
        log["fallback"].append(fb)
        if not accepted:
            break
        g_new = gradient(st, dv_t)
        s = dv_t - dv
        y = g_new - g
        ys = float(np.sum(y * s))
        skip = not (ys > 1e-12 * math.sqrt(float(np.sum(y * y)) * float(np.sum(s * s))))
        if not skip:
            hist.append((s, y, 1.0 / ys))
            if len(hist) > history:
                hist.pop(0)
        log["skipped"].append(int(skip))
        dv, g, ep, en = dv_t, g_new, ep_t, en_t
        it += 1
        cn = cn_norm(st, g)
        log["cn"].append(cn)
        log["E"].append(float(np.sum(ep) + np.sum(en)))
        converged = cn <= thresh
    return dv, dict(iters=it, converged=bool(converged), log=log, n_nodes=n)


def precond_cg(A, apply_M, b, rel, max_iter, log=None):
    """Preconditioned conjugate gradients from x0 = 0 for A x = b, stopped at
    the first iterate with sqrt(r^T M r) <= rel * sqrt(b^T M b), where M is
    the preconditioner's inverse as applied by ``apply_M`` (the inexact linear
    solve of Sec. 5.3, in the preconditioner's energy norm), or after
    max_iter iterations.  With apply_M = r / diag(A) this is the arithmetic
    of ``coarse_pcg``."""
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_M(r)
    rz = float(r @ z)
    stop = rel * math.sqrt(max(rz, 0.0))
    it = 0
    if rz > 0.0:
        p = z.copy()
        while it < max_iter:
            q = A @ p
            alpha = rz / float(p @ q)
            x += alpha * p
            r -= alpha * q
            z = apply_M(r)
            rz_new = float(r @ z)
            it += 1
            if math.sqrt(max(rz_new, 0.0)) <= stop:
                break
            beta = rz_new / rz
            rz = rz_new
            p = z + beta * p
    if log is not None:
        log.append(it)
    return x


def inexact_tolerance(r0Mr0, tau):
    """Relative tolerance of a Newton step's linear solve (Sec. 5.3, adaptive
    inexactness): k = min(1/2, sqrt(max(sqrt(r0^T M r0), tau))), with M the
    preconditioner (its energy norm scales the residual by the local
    stiffness) and tau the floor; the reading used is tau = the CN
    tolerance eps."""
    return min(0.5, math.sqrt(max(math.sqrt(max(r0Mr0, 0.0)), tau)))


def solve_pn(st, tol, levels, precond="jacobi", max_iters=500, cg_max_iter=10000, sweeps=1,
             c1=1e-4, max_halvings=30, smoother="l1jacobi"):
    """Projected Newton with inexact preconditioned CG (Alg. 1, the inexact
    Newton-Krylov baseline; PN-PCG with precond="jacobi", PN-MGPCG with
    precond="mg", Sec. 5.1 and Sec. 7).

    dv^1 = 0; while the CN-scaled gradient norm exceeds eps*sqrt(n): the
    projected Hessian at dv^i (Teran et al. 2005 projection, Dirichlet
    projection), its linear system H p = -g solved by CG from 0 to the
    adaptive relative tolerance k (preconditioner: the scalar diagonal, or
    one V-cycle of the Galerkin hierarchy rebuilt from this Hessian), then
    the same backtracking line search as HOT."""
    n = st.lev0.n
    dv = np.zeros((n, 3))
    g = gradient(st, dv)
    ep, en = energy_terms(st, dv)
    log = dict(cn=[], alpha_halvings=[], cg=[], k=[], E=[])
    thresh = tol * math.sqrt(n)
    cn = cn_norm(st, g)
    log["cn"].append(cn)
    log["E"].append(float(np.sum(ep) + np.sum(en)))
    it = 0
    converged = cn <= thresh
    while not converged and it < max_iters:
        H, nbr = hessian_slots(st, dv=dv)
        hz = build_hierarchy(st, H, nbr, levels if precond == "mg" else 1, project_pattern=False)
        b = -g.ravel() * hz.free[0]
        if precond == "mg":
            apply_M = lambda r: vcycle(hz, r, sweeps=sweeps, smoother=smoother)
        else:
            apply_M = lambda r: r / hz.diag[0]
        k = inexact_tolerance(float(b @ apply_M(b)), tol)
        cg_log = []
        p = precond_cg(hz.A[0], apply_M, b, k, cg_max_iter, log=cg_log).reshape(n, 3)
        gp = float(np.sum(g * p))
        alpha = 1.0
        accepted = False
        halvings = 0
        for halvings in range(max_halvings + 1):
            dv_t = dv + alpha * p
            ep_t, en_t = energy_terms(st, dv_t)
            dE = float(np.sum(ep_t - ep) + np.sum(en_t - en))
            if np.isfinite(dE) and dE <= c1 * alpha * gp:
                accepted = True
                break
            alpha *= 0.5
        log["alpha_halvings"].append(halvings if accepted else -1)
        log["cg"].append(cg_log[0])
        log["k"].append(k)
        if not accepted:
            break
        dv, ep, en = dv_t, ep_t, en_t
        g = gradient(st, dv)
        it += 1
        cn = cn_norm(st, g)
        log["cn"].append(cn)
        log["E"].append(float(np.sum(ep) + np.sum(en)))
        converged = cn <= thresh
    return dv, dict(iters=it, converged=bool(converged), log=log, n_nodes=n)


def von_mises(F, mu, ys):
    """Von Mises return mapping on the Hencky strain, applied once per step
    after the solve (lagged plasticity, Sec. 2 and Sec. 8).  Deviatoric log
    strain is scaled back onto 2 mu |eps_dev| = sqrt(2/3) sigma_y; volume is
    kept.  Particles with yield stress 0 are elastic."""
    out = F.copy()
    sel = ys > 0
    if not np.any(sel):
        return out
    U, S, V = svd_signed(F[sel])
    eps = np.log(np.abs(S))
    sign = np.sign(S)
    dev = eps - eps.mean(axis=1, keepdims=True)
    nd = np.linalg.norm(dev, axis=1)
    lim = math.sqrt(2.0 / 3.0) * ys[sel] / (2.0 * mu[sel])
    yielded = nd > lim
    scale = np.where(yielded, lim / np.where(nd > 0, nd, 1.0), 1.0)
    eps_new = eps.mean(axis=1, keepdims=True) + dev * scale[:, None]
    Snew = sign * np.exp(eps_new)
    Fn = U @ (Snew[:, :, None] * np.swapaxes(V, -1, -2))
    sub = out[sel]
    sub[yielded] = Fn[yielded]
    out[sel] = sub
    return out


def snow_clamp(F, clamp):
    """Snow-type plastic flow (Sec. 7, table of material parameters, after
    Stomakhin et al. 2013): after the step the singular values of F are
    clamped into [lo, hi]; the rest of the deformation is plastic and
    forgotten (no hardening).  Uses the signed SVD; rows with hi = 0 are
    untouched."""
    out = F.copy()
    sel = clamp[:, 1] > 0
    if not np.any(sel):
        return out
    U, S, V = svd_signed(F[sel])
    Sc = np.clip(S, clamp[sel, 0:1], clamp[sel, 1:2])
    out[sel] = U @ (Sc[:, :, None] * np.swapaxes(V, -1, -2))
    return out


def time_step(scene):
    """dt = min(1/FPS, CFL * dx / v_max) (Sec. 7.1 simulation settings);
    v_max includes prescribed boundary speeds."""
    vmax = max(float(np.max(np.linalg.norm(scene.v, axis=1))) if scene.n else 0.0,
               bc_max_speed(scene))
    if vmax <= 0.0:
        return scene.max_dt
    return min(scene.max_dt, scene.cfl * scene.dx / vmax)


def g2p(st, dv):
    """Grid-to-particle APIC transfer, deformation update and advection
    (Sec. 3.1): v_p = sum w v_i; C_p = 4/dx^2 sum w v_i (x_i - x_p)^T;
    F^{n+1} = (I + dt sum v_i grad w^T) F^n; lagged plasticity (von Mises or
    the snow clamp); x += dt v_p."""
    sc = st.scene
    vnew = st.vstar + dv
    vel = vnew[st.idx]
    vp = np.einsum("pk,pka->pa", st.W, vel)
    Cp = (4.0 / sc.dx ** 2) * np.einsum("pk,pka,pkb->pab", st.W, vel, st.xip)
    gradv = np.einsum("pka,pkb->pab", vel, st.G)
    F = (np.eye(3)[None] + st.dt * gradv) @ sc.F
    F = von_mises(F, st.mu, st.yield_stress)
    F = snow_clamp(F, particle_snow_clamp(sc))
    out = sc.copy()
    out.x = sc.x + st.dt * vp
    out.v = vp
    out.C = Cp
    out.F = F
    return out


def step(scene, dt=None, t=0.0, levels=None, history=None, tol=None, max_iters=None,
         sweeps=None, return_internals=False, smoother="l1jacobi", solver="hot",
         embedding="linear"):
    """One implicit MPM step: P2G, the solve for dv, G2P (Sec. 3.1).  solver:
    "hot" (Alg. HOT), "pn-pcg" or "pn-mgpcg" (Alg. 1 with the diagonal or the
    multigrid preconditioner).  embedding "quadratic" builds HOT's hierarchy
    with the quadratic node embedding (HOT-quadratic, Sec. 7; l1 block-Jacobi
    smoothing only: the colouring of the Gauss-Seidel smoother assumes
    stencils of +-2 nodes)."""
    if embedding != "linear" and smoother != "l1jacobi":
        raise ValueError("the quadratic embedding is built with l1 block-Jacobi smoothing only")
    if dt is None or dt <= 0:
        dt = time_step(scene)
    levels = scene.mg_levels if levels is None else levels
    history = scene.lbfgs_history if history is None else history
    tol = scene.tol if tol is None else tol
    max_iters = scene.max_iters if max_iters is None else max_iters
    sweeps = getattr(scene, "smoother_sweeps", 1) if sweeps is None else sweeps
    st = prepare(scene, dt, t)
    if solver != "hot":
        assert solver in ("pn-pcg", "pn-mgpcg")
        dv, info = solve_pn(st, tol, levels, "mg" if solver == "pn-mgpcg" else "jacobi",
                            max_iters=max_iters, sweeps=sweeps, smoother=smoother)
        out = g2p(st, dv)
        info["dt"] = dt
        if return_internals:
            return out, info, dict(st=st, dv=dv)
        return out, info
    H0, nbr0 = hessian_slots(st)
    hz = build_hierarchy(st, H0, nbr0, levels, embedding=embedding)
    dv, info = solve(st, hz, tol, history, max_iters=max_iters, sweeps=sweeps,
                     smoother=smoother)
    out = g2p(st, dv)
    info["dt"] = dt
    if return_internals:
        return out, info, dict(st=st, hz=hz, H0=H0, nbr0=nbr0, dv=dv)
    return out, info
