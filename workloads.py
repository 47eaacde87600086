"""Seeded synthetic inputs for the equivalent-charge FMM.

This module is the only code shared by the oracle side (tests, CPU baseline)
and the GPU side (tests, bench).  It draws positions and charges and holds the
workload table; it holds none of the method's arithmetic.

The paper's own experiments use random +-1 charges scattered in a unit cube
(Sec. 3.1, Table 1: N = 23040, 8x8x8 finest cells, order 3..7).  The larger
workloads below keep that shape (uniform cube, neutral charges) at the sizes
the hot path is measured on, plus a clustered set and a water-like periodic
box.  Everything is generated with ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FREE, FREE_CONTINUOUS, PERIODIC, PERIODIC_CONTINUOUS = 0, 1, 2, 3
FP64, FP32, FP32_BF16FAR = 0, 1, 2

BOUNDARY_NAMES = {FREE: "free", FREE_CONTINUOUS: "free-continuous",
                  PERIODIC: "periodic", PERIODIC_CONTINUOUS: "periodic-continuous"}
PRECISION_NAMES = {FP64: "f64", FP32: "f32", FP32_BF16FAR: "f32+bf16far"}


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int            # number of charges
    levels: int       # finest level l_f
    order: int        # points per axis (the paper's n)
    boundary: int
    precision: int
    seed: int
    kind: str         # generator: uniform_alt / uniform_meansub / uniform_pm / clustered / water / paper_t1


# The five measured workloads (uniform, clustered, water-like) and the
# paper's Table 1 workload.
WORKLOADS = {
    "c1": Workload("c1-uniform4096-l3-n4-free-f64", 4096, 3, 4, FREE, FP64, 1, "uniform_alt"),
    "c2": Workload("c2-uniform262144-l5-n4-free-f32", 262144, 5, 4, FREE, FP32, 2, "uniform_meansub"),
    "c3": Workload("c3-uniform2097152-l6-n5-periodic-continuous-f32", 2097152, 6, 5,
                   PERIODIC_CONTINUOUS, FP32, 3, "uniform_pm"),
    "c4": Workload("c4-clustered1048576-l6-n6-free-continuous-f32", 1048576, 6, 6,
                   FREE_CONTINUOUS, FP32, 4, "clustered"),
    "c5": Workload("c5-water3145728-l7-n4-periodic-continuous-f32", 3 * 4 * 64 ** 3, 7, 4,
                   PERIODIC_CONTINUOUS, FP32, 5, "water"),
    "t1": Workload("paper-table1-uniform23040-l3", 23040, 3, 4, FREE, FP64, 11, "uniform_pm"),
}


def uniform_positions(rng, n):
    return rng.random((n, 3))


def alternating_charges(n):
    q = np.ones(n)
    q[1::2] = -1.0
    return q


def meansub_charges(rng, n):
    q = rng.uniform(-1.0, 1.0, n)
    return q - q.mean()


def pm_charges(rng, n):
    """Half +1, half -1 in random order (net neutral); n even."""
    q = np.concatenate([np.ones(n // 2), -np.ones(n - n // 2)])
    return rng.permutation(q)


def clustered_positions(rng, n, centres=64, sigma=0.02):
    cen = rng.random((centres, 3))
    lab = rng.integers(0, centres, n)
    pos = cen[lab] + sigma * rng.standard_normal((n, 3))
    return np.clip(pos, 0.0, np.nextafter(1.0, 0.0))


# Water-like box: rigid 3-site molecules, O-H 0.09572 nm and H-O-H 104.52
# degrees, at the number density of liquid water (one molecule per
# (0.3104 nm)^3); the box side is scaled to 1.  The oxygens sit on a jittered
# face-centred cubic lattice of m^3 cells (4 m^3 molecules, 2^20 for m = 64).
WATER_Q = (-0.834, 0.417, 0.417)
WATER_SPACING_NM = 0.3104
WATER_ROH_NM = 0.09572
WATER_THETA_DEG = 104.52
FCC_BASIS = ((0.0, 0.0, 0.0), (0.5, 0.5, 0.0), (0.5, 0.0, 0.5), (0.0, 0.5, 0.5))


def water_positions(rng, m):
    """4*m**3 molecules on a jittered FCC lattice of m**3 cells, uniform random
    orientations (unit quaternions); returns [3*4*m**3, 3] in [0,1) and charges."""
    nmol = 4 * m ** 3
    box_nm = WATER_SPACING_NM * nmol ** (1.0 / 3.0)
    r_oh = WATER_ROH_NM / box_nm
    g = np.arange(m)
    cx, cy, cz = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(float)
    o = (cells[:, None, :] + np.array(FCC_BASIS)[None, :, :] + 0.25).reshape(-1, 3) / m
    o = o + rng.uniform(-0.05 / m, 0.05 / m, o.shape)
    nm = o.shape[0]
    # uniform random rotations from unit quaternions (Shoemake's method)
    u1, u2, u3 = rng.random((3, nm))
    qa = np.sqrt(1 - u1) * np.sin(2 * np.pi * u2)
    qb = np.sqrt(1 - u1) * np.cos(2 * np.pi * u2)
    qc = np.sqrt(u1) * np.sin(2 * np.pi * u3)
    qd = np.sqrt(u1) * np.cos(2 * np.pi * u3)
    w, x, y, z = qd, qa, qb, qc
    rot = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], 1)  # [nm, 3, 3]
    half = math.radians(WATER_THETA_DEG) / 2
    h1 = np.array([math.sin(half), math.cos(half), 0.0]) * r_oh
    h2 = np.array([-math.sin(half), math.cos(half), 0.0]) * r_oh
    p1 = o + rot @ h1
    p2 = o + rot @ h2
    pos = np.stack([o, p1, p2], axis=1).reshape(-1, 3)
    pos = np.mod(pos, 1.0)
    pos[pos >= 1.0] = 0.0
    q = np.tile(np.array(WATER_Q), nm)
    return pos, q


def water_step(rng, pos, sigma=1e-4):
    """One step of the perturbation sequence: every charge moves by
    N(0, sigma) per axis and is wrapped back into [0, 1)."""
    p = np.mod(pos + sigma * rng.standard_normal(pos.shape), 1.0)
    p[p >= 1.0] = 0.0
    return p


def make_inputs(kind, n, seed):
    """Positions [n,3] (float64, in [0,1)^3) and charges [n] (float64)."""
    rng = np.random.default_rng(seed)
    if kind == "uniform_alt":
        return uniform_positions(rng, n), alternating_charges(n)
    if kind == "uniform_meansub":
        pos = uniform_positions(rng, n)
        return pos, meansub_charges(rng, n)
    if kind == "uniform_pm":
        pos = uniform_positions(rng, n)
        return pos, pm_charges(rng, n)
    if kind == "clustered":
        pos = clustered_positions(rng, n)
        return pos, meansub_charges(rng, n)
    if kind == "water":
        m = round((n // 12) ** (1.0 / 3.0))
        if 12 * m ** 3 != n:
            raise ValueError("water workload needs n = 12*m**3 (FCC cells of 4 molecules)")
        return water_positions(rng, m)
    raise ValueError(f"unknown generator {kind!r}")


def workload_inputs(key):
    w = WORKLOADS[key]
    pos, q = make_inputs(w.kind, w.n, w.seed)
    return w, pos, q


def small_variant(key, n, levels, seed_offset=100):
    """Same generator and mode as workload `key`, at a size the oracle finishes
    in seconds (used by the parity tests)."""
    w = WORKLOADS[key]
    kind = w.kind
    if kind == "water":
        m = max(2, round((n // 12) ** (1.0 / 3.0)))
        n = 12 * m ** 3
    pos, q = make_inputs(kind, n, w.seed + seed_offset)
    return dataclasses.replace(w, n=n, levels=levels, name=w.name + f"-small{n}-l{levels}"), pos, q
