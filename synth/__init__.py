"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds workload *descriptions* and seeded random numbers only.  It
contains none of the solver's arithmetic: mesh refinement, balancing,
coarsening, degrees of freedom, constraints, operators and transfers are
implemented separately (and independently) in ``oracle/`` and in the HIP
library.  Both sides read the same descriptors defined here.

Mesh descriptors
----------------
A mesh is a coarse ``n0^3`` grid of cubes on ``[lo, hi]^3``, refined
``n_global`` times uniformly and then once per entry of ``steps``.  Each step
refines every active cell for which the step's predicate holds and then closes
the mesh so that two leaves that touch (share at least a point) differ by at
most one level (the one-irregularity closure of the paper's test meshes,
Section 4 "Examples").  Predicate kinds (the paper's octant and shell
criteria, plus the ball and sphere criteria of the benchmark workloads):

* ``ALL``          every cell.
* ``BALL``         params (x0, y0, z0, r): the cell centre c has
                   (cx-x0)^2 + (cy-y0)^2 + (cz-z0)^2 <= r^2.
* ``BOX_LE``       params (a, b, c): cx <= a and cy <= b and cz <= c
                   (the paper's octant [-1,0]^3 with a=b=c=0).
* ``BAND``         params (x0, y0, z0, r1, r2): r1^2 <= |c - x0|^2 <= r2^2
                   (the paper's shell bands).
* ``SPHERE_CUT``   params (x0, y0, z0, ra, rb): the closed cell box
                   intersects the sphere |x - x0| = ra or (if rb > 0) the
                   sphere |x - x0| = rb, i.e. dmin <= r <= dmax with dmin,
                   dmax the smallest and largest distance from x0 to the box.

Canonical node codes and the hash input
---------------------------------------
``dof_hash`` turns an exact integer identification of a node position (three
64-bit codes, one per axis, computed independently by each side) into a
pseudo-random value in [-1, 1).  It uses the published SplitMix64 finaliser
(Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014) and serves as the vector input of operator parity tests at any
mesh size: both sides can evaluate it at any node without exchanging vectors.
"""
from __future__ import annotations

import numpy as np

# predicate kinds (same integers as the C ABI's MFMG_PRED_* values)
ALL, BALL, BOX_LE, BAND, SPHERE_CUT = 0, 1, 2, 3, 4
KIND_NAMES = {ALL: "all", BALL: "ball", BOX_LE: "box_le", BAND: "band",
              SPHERE_CUT: "sphere_cut"}

# maximum refinement depth encoded in node codes (finest lattice = level 20)
CODE_MAX_LEVEL = 20


# Diffusion-coefficient descriptors (kinds as the library's coef_kind): the
# constant, a ball inclusion, a checkerboard.  Parameters only, no arithmetic.
COEF_CONST, COEF_BALL, COEF_CHECKER = 0, 1, 2


def coef_desc(kind, params):
    return {"kind": int(kind), "params": [float(p) for p in params]}


# a high-contrast inclusion: c = 1000 in the ball of radius 0.3 about
# (0.5, 0.5, 0.5), 1 elsewhere
COEF_INCLUSION = coef_desc(COEF_BALL, (0.5, 0.5, 0.5, 0.3, 1000.0, 1.0))
# a high-contrast checkerboard of 0.25-cubes (c = 1 and 1000), aligned with the
# coarse grids of the benchmark meshes
COEF_CHECKER_1000 = coef_desc(COEF_CHECKER, (1.0, 1000.0, 0.25, 0.0))

# Cell-geometry descriptors (kinds as the library's geom_kind): the coarse-grid
# vertices moved by an affine map (kind 1, parameters of an upper-triangular
# matrix) or by an interior bump that keeps the boundary (kind 2, amplitude
# and direction).  Parameters only, no arithmetic.
GEOM_NONE, GEOM_AFFINE, GEOM_BUMP = 0, 1, 2


def geom_desc(kind, params):
    return {"kind": int(kind), "params": [float(p) for p in params]}


GEOM_SHEAR = geom_desc(GEOM_AFFINE, (1.3, 0.4, -0.2, 0.9, 0.3, 1.1))
GEOM_BUMP8 = geom_desc(GEOM_BUMP, (0.08, 1.0, -0.7, 0.5))


def mesh_desc(name, n0, lo, hi, n_global, steps):
    return {"name": name, "n0": int(n0), "lo": float(lo), "hi": float(hi),
            "n_global": int(n_global),
            "steps": [(int(k), tuple(float(p) for p in params)) for k, params in steps]}


def ball_mesh(name, n0, n_global, n_steps, r=0.5, centre=(0.0, 0.0, 0.0), lo=0.0, hi=1.0):
    return mesh_desc(name, n0, lo, hi, n_global,
                     [(BALL, (*centre, r))] * n_steps)


# -- workloads -----------------------------------------------------------------
# Poisson on the unit cube, refinement towards the corner at the origin.
# 4^3 coarse cubes, one uniform refinement, two ball steps: 2808 cells, Q2.
CFG1 = ball_mesh("cube4_g1_ball2", 4, 1, 2)
# Literal reading without the uniform step: 386 cells (brute-force sized).
CFG1_TINY = ball_mesh("cube4_ball2", 4, 0, 2)
# 16^3 coarse cubes, four ball steps: 1,068,726 cells, Q4 (about 68M DoFs).
CFG2 = ball_mesh("cube16_ball4", 16, 0, 4)
# [-1,1]^3, 12^3 coarse cubes, one uniform step, three steps refining cells cut
# by the spheres of radius 0.3 and 0.7 about the centre; Q6 -> Q3 -> Q1.
CFG4 = mesh_desc("cube12_g1_spheres3", 12, -1.0, 1.0, 1,
                 [(SPHERE_CUT, (0.0, 0.0, 0.0, 0.3, 0.7))] * 3)
# The learned coarse correction where the coarse level matters: 6^3 coarse
# cubes (the Q2 coarse problem has 1,331 DoFs), two uniform steps and one
# ball step; three levels, so the coarse correction carries the smooth error
# that the smoothers of the two finer levels leave.
CFG5_GAIN = ball_mesh("cube6_g2_ball1", 6, 2, 1)


def octant_mesh(L):
    """Paper's ``octant`` case: [-1,1]^3, refine cells in [-1,0]^3, L times."""
    return mesh_desc(f"octant{L}", 1, -1.0, 1.0, 0, [(BOX_LE, (0.0, 0.0, 0.0))] * L)


def shell_mesh(L):
    """Paper's ``shell`` case: L-3 uniform steps then three band steps."""
    return mesh_desc(f"shell{L}", 1, -1.0, 1.0, L - 3,
                     [(BAND, (0.0, 0.0, 0.0, 0.0, 0.55)),
                      (BAND, (0.0, 0.0, 0.0, 0.3, 0.43)),
                      (BAND, (0.0, 0.0, 0.0, 0.335, 0.39))])


# the paper's two test shapes at about 17M Q4 DoFs, and a uniform mesh of
# that size built the same way from one cell (hanging-node overhead)
OCTANT7 = octant_mesh(7)
SHELL8 = shell_mesh(8)
UNIFORM64 = mesh_desc("uniform64", 1, -1.0, 1.0, 6, [])


def small_mesh(name="tiny2", n0=2, n_global=0, n_steps=2, r=0.6, lo=0.0, hi=1.0):
    """Very small hanging-node meshes for brute-force checks."""
    return ball_mesh(name, n0, n_global, n_steps, r=r, lo=lo, hi=hi)


# -- seeded numbers -------------------------------------------------------------
_M64 = (1 << 64) - 1


def _splitmix64_np(z):
    z = (z + np.uint64(0x9E3779B97F4A7C15))
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def dof_hash(codes, seed=12292):
    """Value in [-1, 1) for each node from its three exact integer codes.

    ``codes``: int64 array of shape (n, 3).  Returns float64 array (n,).
    """
    codes = np.asarray(codes, dtype=np.int64)
    with np.errstate(over="ignore"):
        h = _splitmix64_np(np.full(codes.shape[0], seed, dtype=np.uint64))
        for d in range(3):
            h = _splitmix64_np(h ^ codes[:, d].astype(np.uint64))
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 / 9007199254740992.0) - 1.0


def uniform_vector(n, seed=12292, dtype=np.float64):
    """U(-1, 1) vector from numpy's PCG64 with the given seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=n).astype(dtype)


def gaussian_rhs(seed, n_terms, w_lo, w_hi, amplitude="one", lo=0.0, hi=1.0):
    """Parameters of f(x) = sum_m a_m exp(-|x - c_m|^2 / (2 w_m^2)).

    Centres uniform in [lo, hi]^3, widths uniform in [w_lo, w_hi], amplitudes 1
    (``amplitude="one"``) or N(0, 1) (``"normal"``).  Returns an (n_terms, 5)
    float64 array of rows (cx, cy, cz, w, a).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(lo, hi, size=(n_terms, 3))
    w = rng.uniform(w_lo, w_hi, size=n_terms)
    a = np.ones(n_terms) if amplitude == "one" else rng.standard_normal(n_terms)
    return np.column_stack([c, w, a])


def gaussian_rhs_batch(n_rhs, n_terms=4, w_lo=0.05, w_hi=0.2, lo=-1.0, hi=1.0, seed0=1000):
    """The batch of right-hand sides of the p-multigrid workload (seed 1000+i)."""
    return [gaussian_rhs(seed0 + i, n_terms, w_lo, w_hi, "one", lo, hi) for i in range(n_rhs)]


def gaussian_rhs_training(j, seed0=2000, lo=0.0, hi=1.0):
    """Right-hand side j of the learned-correction data set: 1-6 terms,
    widths in [0.05, 0.3], amplitudes N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed0 + j))
    n_terms = int(rng.integers(1, 7))
    return gaussian_rhs(seed0 + j + 7_000_000, n_terms, 0.05, 0.3, "normal", lo, hi)
