"""Seeded synthetic scene generators for the implicit MPM step.

This module only *generates inputs*: particle lattices, initial velocity
fields, material tables and boundary-condition descriptors.  It performs none
of the method's arithmetic (no transfers, no energies, no solves), so both the
CPU oracle and the HIP path can consume the same scenes without sharing any
solver code.

Conventions (shared input format):
  * Grid nodes sit at ``origin + i*dx`` for i = 0..grid_cells (per axis).
  * Particles are seeded 2x2x2 per cell at sub-positions 1/4 and 3/4 of the
    cell, cells enumerated x fastest, then the 8 sub-positions x fastest.
    Each coordinate gets a jitter drawn from U(-0.25, 0.25) * dx/2.
  * ``F`` and ``C`` are (n, 3, 3) row-major; ``C`` is the APIC affine velocity
    matrix (velocity gradient for an affine field).
  * Materials: model 0 = fixed-corotated, 1 = Neo-Hookean; SI units.
  * Boundary conditions (all sticky, i.e. every velocity component prescribed):
      kind 0 (box walls): p[0] = thickness in cells; nodes whose index is
              <= p[0] or >= grid_cells - p[0] on any axis are held at rest.
      kind 1 (grip): p[0:3] box min, p[3:6] box max (world), p[6:9] a point on
              the rotation axis, p[9:12] axis direction, p[12] angular speed
              (rad/s).  Nodes inside the box move with w * (a x (x - c)).
      kind 2 (sphere): p[0:3] centre at t = 0, p[3] radius, p[4:7] velocity.
              Nodes inside the moving sphere at the end of the step get the
              sphere's velocity.

Random streams: numpy PCG64 with an explicit seed per scene; the jitter array
is drawn before the velocity-noise array.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

FCR = 0
NEOHOOKEAN = 1

BC_BOX_WALLS = 0
BC_GRIP = 1
BC_SPHERE = 2


@dataclasses.dataclass
class Scene:
    name: str
    dx: float
    grid_cells: tuple
    origin: tuple
    gravity: tuple
    x: np.ndarray            # (n, 3) float64
    v: np.ndarray            # (n, 3) float64
    F: np.ndarray            # (n, 3, 3) float64
    C: np.ndarray            # (n, 3, 3) float64
    vol0: np.ndarray         # (n,) float64
    mat_id: np.ndarray       # (n,) int32
    materials: List[dict]
    bcs: List[dict]
    cfl: float = 0.6
    max_dt: float = 1.0 / 24.0
    tol: float = 1e-6
    lbfgs_history: int = 8
    mg_levels: int = 3
    max_iters: int = 500
    n_steps: int = 1
    smoother_sweeps: int = 1  # smoothing sweeps per level and direction

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def copy(self) -> "Scene":
        out = dataclasses.replace(self)
        for f in ("x", "v", "F", "C", "vol0", "mat_id"):
            setattr(out, f, getattr(self, f).copy())
        out.materials = [dict(m) for m in self.materials]
        out.bcs = [dict(kind=b["kind"], p=np.array(b["p"], dtype=np.float64)) for b in self.bcs]
        return out


def material(model: int, E: float, nu: float, density: float, yield_stress: float = 0.0,
             snow_clamp=(0.0, 0.0)) -> dict:
    return dict(model=int(model), E=float(E), nu=float(nu), density=float(density),
                yield_stress=float(yield_stress),
                snow_clamp=(float(snow_clamp[0]), float(snow_clamp[1])))


def bc_walls(thickness: int) -> dict:
    p = np.zeros(16)
    p[0] = thickness
    return dict(kind=BC_BOX_WALLS, p=p)


def bc_grip(box_min, box_max, axis_point, axis_dir, omega) -> dict:
    p = np.zeros(16)
    p[0:3] = box_min
    p[3:6] = box_max
    p[6:9] = axis_point
    p[9:12] = axis_dir
    p[12] = omega
    return dict(kind=BC_GRIP, p=p)


def bc_sphere(center, radius, velocity) -> dict:
    p = np.zeros(16)
    p[0:3] = center
    p[3] = radius
    p[4:7] = velocity
    return dict(kind=BC_SPHERE, p=p)


def lattice(cell_lo, cell_hi, dx, origin, jitter):
    """Positions of a 2x2x2-per-cell lattice over cells [lo, hi) per axis.

    ``jitter`` is an (n, 3) array of offsets already scaled to metres.
    """
    lo = np.asarray(cell_lo, dtype=np.int64)
    hi = np.asarray(cell_hi, dtype=np.int64)
    cz, cy, cx = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]),
                             np.arange(lo[0], hi[0]), indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(np.float64)
    sz, sy, sx = np.meshgrid([0.25, 0.75], [0.25, 0.75], [0.25, 0.75], indexing="ij")
    subs = np.stack([sx.ravel(), sy.ravel(), sz.ravel()], axis=1)
    pos = (cells[:, None, :] + subs[None, :, :]).reshape(-1, 3)
    return np.asarray(origin, dtype=np.float64) + pos * dx + jitter


def lattice_count(cell_lo, cell_hi) -> int:
    d = np.asarray(cell_hi) - np.asarray(cell_lo)
    return int(np.prod(d)) * 8


def skew(w):
    w = np.asarray(w, dtype=np.float64)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def _assemble(name, dx, cells, origin, gravity, blocks, materials, bcs, seed, noise_sigma,
              **params) -> Scene:
    """blocks: list of (cell_lo, cell_hi, mat_id, omega_vec, center) seeded in order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_tot = sum(lattice_count(b[0], b[1]) for b in blocks)
    jitter = rng.uniform(-0.25, 0.25, size=(n_tot, 3)) * (dx / 2.0)
    noise = rng.normal(0.0, 1.0, size=(n_tot, 3)) * noise_sigma
    xs, vs, Cs, mids = [], [], [], []
    off = 0
    for lo, hi, mid, omega, center in blocks:
        nb = lattice_count(lo, hi)
        x = lattice(lo, hi, dx, origin, jitter[off:off + nb])
        W = skew(omega)
        v = (x - np.asarray(center)) @ W.T + noise[off:off + nb]
        xs.append(x)
        vs.append(v)
        Cs.append(np.broadcast_to(W, (nb, 3, 3)))
        mids.append(np.full(nb, mid, dtype=np.int32))
        off += nb
    x = np.concatenate(xs)
    n = x.shape[0]
    return Scene(name=name, dx=float(dx), grid_cells=tuple(int(c) for c in cells),
                 origin=tuple(float(o) for o in origin), gravity=tuple(float(g) for g in gravity),
                 x=x, v=np.concatenate(vs), F=np.broadcast_to(np.eye(3), (n, 3, 3)).copy(),
                 C=np.concatenate(Cs).copy(), vol0=np.full(n, dx ** 3 / 8.0),
                 mat_id=np.concatenate(mids), materials=materials, bcs=bcs, **params)


def rotating_cube(cells=32, cube=16, seed=0) -> Scene:
    """FCR cube spinning at 1 rad/s about +z, resting inside sticky walls.

    32^3 grid with dx = 1/32 and a centred 16^3-cell cube gives 32768 particles.
    """
    dx = 1.0 / cells
    lo = (cells - cube) // 2
    center = np.full(3, (lo + cube / 2.0) * dx)
    return _assemble(
        f"rotating_cube_{cells}_{cube}", dx, (cells,) * 3, (0.0, 0.0, 0.0), (0.0, -9.8, 0.0),
        [((lo,) * 3, (lo + cube,) * 3, 0, (0.0, 0.0, 1.0), center)],
        [material(FCR, 1e5, 0.3, 1000.0)], [bc_walls(2)], seed, 0.05,
        tol=1e-6, lbfgs_history=5, mg_levels=3, n_steps=1)


def twisting_bars(side=16, seed=1000, length=192, n_steps=20, sweeps=5) -> Scene:
    """Four parallel Neo-Hookean bars twisted by opposite grips at +-2 rad/s.

    Grid 256x64x64 with dx = 1/64; bars run along x over cells [32, 32+length)
    with a side x side cross-section, laid out 2x2 in y-z.  side=12 gives
    884736 particles and side=16 gives 1572864.  E per bar in {1e5..1e8} Pa.
    Solver settings: 5 levels, L-BFGS window 8, CN tolerance 1e-6, and
    ``sweeps`` l1 block-Jacobi sweeps per level and direction.
    """
    dx = 1.0 / 64.0
    cells = (256, 64, 64)
    starts = {12: (14, 38), 16: (12, 36)}.get(side)
    if starts is None:
        starts = (32 - side - 4, 36)
    x0, x1 = 32, 32 + length
    blocks, mats, bcs = [], [], [bc_walls(2)]
    k = 0
    for z0 in starts:
        for y0 in starts:
            lo, hi = (x0, y0, z0), (x1, y0 + side, z0 + side)
            blocks.append((lo, hi, k, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0)))
            mats.append(material(NEOHOOKEAN, 10.0 ** (5 + k), 0.4, 1000.0))
            axis_pt = np.array([0.0, (y0 + side / 2.0) * dx, (z0 + side / 2.0) * dx])
            ylo, yhi = (y0 - 2) * dx, (y0 + side + 2) * dx
            zlo, zhi = (z0 - 2) * dx, (z0 + side + 2) * dx
            bcs.append(bc_grip(((x0 - 2) * dx, ylo, zlo), ((x0 + 8) * dx, yhi, zhi),
                               axis_pt, (1.0, 0.0, 0.0), +2.0))
            bcs.append(bc_grip(((x1 - 8) * dx, ylo, zlo), ((x1 + 2) * dx, yhi, zhi),
                               axis_pt, (1.0, 0.0, 0.0), -2.0))
            k += 1
    return _assemble(f"twisting_bars_{side}", dx, cells, (0.0, 0.0, 0.0), (0.0, -9.8, 0.0),
                     blocks, mats, bcs, seed, 0.0, tol=1e-6, lbfgs_history=8, mg_levels=5,
                     n_steps=n_steps, smoother_sweeps=sweeps)


def sphere_slab(seed=3000, n=192, slab=(160, 40, 160), y0=24, radius=0.1, speed=3.0,
                levels=4, n_steps=30) -> Scene:
    """Elastoplastic FCR slab (von Mises, yield 1e5 Pa) struck by a rigid sphere.

    192^3 grid, dx = 1/192, slab of 160x40x160 cells (8.19M particles), sphere of
    radius 0.1 m starting one cell above the slab top and moving down at 3 m/s.
    """
    dx = 1.0 / n
    xlo = (n - slab[0]) // 2
    zlo = (n - slab[2]) // 2
    lo, hi = (xlo, y0, zlo), (xlo + slab[0], y0 + slab[1], zlo + slab[2])
    cy = (y0 + slab[1] + 1) * dx + radius
    bcs = [bc_walls(2), bc_sphere((0.5 * n * dx, cy, 0.5 * n * dx), radius, (0.0, -speed, 0.0))]
    return _assemble(f"sphere_slab_{n}", dx, (n,) * 3, (0.0, 0.0, 0.0), (0.0, -9.8, 0.0),
                     [(lo, hi, 0, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))],
                     [material(FCR, 1e7, 0.3, 2000.0, yield_stress=1e5)], bcs, seed, 0.0,
                     tol=1e-6, lbfgs_history=8, mg_levels=levels, n_steps=n_steps)


def stiffness_bar(E_mid=1e5, side=8, length=96, seed=5000, E_end=1e5, levels=3,
                  n_steps=10) -> Scene:
    """A three-material bar twisted by opposite grips at +-2 rad/s: the two
    end thirds keep E = E_end and the middle third has E = E_mid (the paper's
    varying-stiffness experiment raises it from 1e5 to 1e10 Pa).  FCR,
    nu = 0.3, density 1000; dx = 1/64, grid of (length + 16) x 32 x 32 cells,
    bar along x from cell 8, centred in y and z, gravity on, sticky walls
    two cells thick."""
    dx = 1.0 / 64.0
    cells = (length + 16, 32, 32)
    x0, x1 = 8, 8 + length
    y0 = z0 = (32 - side) // 2
    t1, t2 = x0 + length // 3, x0 + 2 * length // 3
    blocks = [((x0, y0, z0), (t1, y0 + side, z0 + side), 0, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
              ((t1, y0, z0), (t2, y0 + side, z0 + side), 1, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
              ((t2, y0, z0), (x1, y0 + side, z0 + side), 2, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))]
    mats = [material(FCR, E_end, 0.3, 1000.0), material(FCR, E_mid, 0.3, 1000.0),
            material(FCR, E_end, 0.3, 1000.0)]
    axis_pt = np.array([0.0, (y0 + side / 2.0) * dx, (z0 + side / 2.0) * dx])
    ylo, yhi = (y0 - 2) * dx, (y0 + side + 2) * dx
    zlo, zhi = (z0 - 2) * dx, (z0 + side + 2) * dx
    bcs = [bc_walls(2),
           bc_grip(((x0 - 2) * dx, ylo, zlo), ((x0 + 4) * dx, yhi, zhi), axis_pt, (1.0, 0.0, 0.0),
                   +2.0),
           bc_grip(((x1 - 4) * dx, ylo, zlo), ((x1 + 2) * dx, yhi, zhi), axis_pt, (1.0, 0.0, 0.0),
                   -2.0)]
    return _assemble(f"stiffness_bar_{E_mid:g}", dx, cells, (0.0, 0.0, 0.0), (0.0, -9.8, 0.0),
                     blocks, mats, bcs, seed, 0.0, tol=1e-6, lbfgs_history=8, mg_levels=levels,
                     n_steps=n_steps)


def serving_scene(index: int, seed_base=4000, n_min=4096, n_max=262144, dx=0.01) -> Scene:
    """One request of the serving stream: a random spinning FCR box.

    Particle count log-uniform in [n_min, n_max], box aspect log-uniform in
    [1/2, 2] per axis, grid twice the bounding box plus a wall margin,
    E log-uniform in [1e4, 1e8] Pa, nu ~ U(0.2, 0.45), |omega| ~ U(0.5, 2).
    """
    rng = np.random.Generator(np.random.PCG64(seed_base + index))
    n_target = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
    aspect = np.exp(rng.uniform(math.log(0.5), math.log(2.0), size=3))
    n_cells = n_target / 8.0
    scale = (n_cells / np.prod(aspect)) ** (1.0 / 3.0)
    dims = np.maximum(2, np.round(aspect * scale)).astype(int)
    E = math.exp(rng.uniform(math.log(1e4), math.log(1e8)))
    nu = rng.uniform(0.2, 0.45)
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    omega = axis * rng.uniform(0.5, 2.0)
    cells = tuple(int(2 * d + 8) for d in dims)
    lo = tuple((c - d) // 2 for c, d in zip(cells, dims))
    hi = tuple(l + d for l, d in zip(lo, dims))
    center = (np.array(lo) + dims / 2.0) * dx
    sc = _assemble(f"serve_{index}", dx, cells, (0.0, 0.0, 0.0), (0.0, -9.8, 0.0),
                   [(lo, hi, 0, tuple(omega), center)],
                   [material(FCR, E, nu, 1000.0)], [bc_walls(2)],
                   int(rng.integers(0, 2 ** 31 - 1)), 0.05,
                   tol=1e-6, lbfgs_history=8, mg_levels=3, n_steps=10)
    return sc


def small_box(cells=(8, 8, 8), box_lo=(2, 2, 2), box_hi=(5, 6, 5), dx=0.1, seed=7,
              model=FCR, E=1e4, nu=0.3, density=1000.0, omega=(0.3, -0.2, 0.5),
              noise=0.05, F_spread=0.0, walls=None, gravity=(0.0, -9.8, 0.0),
              n_mats=1, levels=2, history=5, tol=1e-6, extra_bcs=()) -> Scene:
    """Small box for unit tests.  ``F_spread`` > 0 draws diagonal-plus-rotation
    initial deformation gradients with singular values in [1-s, 1+s] (the
    stretched-box set-up); ``n_mats`` > 1 splits the box into materials whose
    Young's modulus grows by 10x per material along x."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = np.array(box_lo), np.array(box_hi)
    center = (lo + hi) / 2.0 * dx
    sc = _assemble(f"small_box_{seed}", dx, tuple(cells), (0.0, 0.0, 0.0), gravity,
                   [(tuple(lo), tuple(hi), 0, omega, center)],
                   [material(model, E * 10.0 ** k, nu, density) for k in range(n_mats)],
                   ([] if walls is None else [bc_walls(walls)]) + list(extra_bcs),
                   int(rng.integers(0, 2 ** 31 - 1)), noise,
                   tol=tol, lbfgs_history=history, mg_levels=levels, n_steps=1)
    if n_mats > 1:
        xs = (sc.x[:, 0] - lo[0] * dx) / ((hi[0] - lo[0]) * dx)
        sc.mat_id = np.minimum((xs * n_mats).astype(np.int32), n_mats - 1)
    if F_spread > 0:
        n = sc.n
        diag = rng.uniform(1.0 - F_spread, 1.0 + F_spread, size=(n, 3))
        q = rng.normal(size=(n, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        a, b, c, d = q.T
        R = np.stack([
            np.stack([a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)], -1),
            np.stack([2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)], -1),
            np.stack([2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d], -1),
        ], axis=1)
        sc.F = R * diag[:, None, :]
    return sc


def stretched_box(side=32, margin=8, seed=6000, E=1e5, levels=3, tol=1e-7, history=8,
                  per_particle=False) -> Scene:
    """The stretched-box convergence workload (Sec. 8): a soft FCR box at rest
    whose deformation gradient starts as a diagonal matrix with entries drawn
    uniformly from [0.7, 1.3] -- one matrix for the whole box, or with
    ``per_particle`` one per particle.  No gravity and no boundary conditions,
    so the first step is the box relaxing from that state.  dx = 1/64, a
    side^3-cell box (8 particles per cell) centred in a (side + 2 margin)^3
    grid; nu = 0.3, density 1000; L-BFGS window 8 and CN tolerance 1e-7 (the
    paper's defaults)."""
    dx = 1.0 / 64.0
    n = side + 2 * margin
    center = np.full(3, (margin + side / 2.0) * dx)
    sc = _assemble(f"stretched_box_{side}", dx, (n,) * 3, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0),
                   [((margin,) * 3, (margin + side,) * 3, 0, (0.0, 0.0, 0.0), center)],
                   [material(FCR, E, 0.3, 1000.0)], [], seed, 0.0,
                   tol=tol, lbfgs_history=history, mg_levels=levels, n_steps=1)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    d = rng.uniform(0.7, 1.3, size=(sc.n if per_particle else 1, 3))
    F = np.zeros((sc.n, 3, 3))
    for a in range(3):
        F[:, a, a] = d[:, a]
    sc.F = F
    return sc


CONFIGS = {
    "rotating_cube": rotating_cube,
    "stiffness_bar": stiffness_bar,
    "twisting_bars": twisting_bars,
    "sphere_slab": sphere_slab,
    "stretched_box": stretched_box,
}
