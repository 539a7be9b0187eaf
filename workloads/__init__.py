"""Seeded synthetic inputs shaped like the paper's electrolyte workloads.

This module only draws positions and charges (NumPy PCG64, fixed seeds) and
describes the five benchmark systems.  It holds none of the method's
arithmetic, so both the oracle and the GPU harness can take their inputs
from it without sharing any part of the computation.

Workload shapes follow the paper's test systems (Sec. 4.1: monovalent and
2:1 primitive electrolytes at ~10 % volume fraction; Sec. 4.3: ions confined
between two dielectric walls; Sec. 5: sizes from 1e2 to 1e6 particles).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    """One system plus the method parameters it is run with."""
    name: str
    geometry: int                 # 0 = fully periodic (HSMA3D), 1 = slab (HSMA2D)
    box: Tuple[float, float, float]
    n: int
    seed: int
    p: int
    F: int
    K: int
    lam: float
    charges: str = "pm1"          # "pm1": +1/-1 halves; "2to1": +2 x n/3, -1 x 2n/3
    min_spacing: float = 0.0      # random sequential addition spacing (0 = none)
    z_range: Optional[Tuple[float, float]] = None  # slab: z drawn uniform in this range
    M: int = 0                    # slab: image layers per side
    gamma_up: float = 0.0
    gamma_low: float = 0.0
    nz: int = 0                   # slab: interface grid points per dimension
    Fw: int = 0                   # lattice generator for the surface rule (0 = auto)
    surface_rule: int = 0
    precision: int = 1            # 0 = fp64, 1 = fp32 compensated
    near_rule: int = 0            # 0 = cell/layer stencil, 1 = images inside the sphere only, 2 = stencil by treecode


# The five systems.  Box lower corner is the origin; slab walls sit at z=0
# and z=Lz.
C1 = Workload("c1_hsma3d_n100_fp64", 0, (10.0, 10.0, 10.0), 100, 1,
              p=6, F=200, K=100, lam=1.5, precision=0)
C2 = Workload("c2_hsma3d_n50000_fp32c", 0, (60.0, 60.0, 60.0), 50_000, 2,
              p=10, F=800, K=400, lam=1.5, min_spacing=0.5)
C3 = Workload("c3_hsma2d_n20000_slab", 1, (40.0, 40.0, 20.0), 20_000, 3,
              p=10, F=800, K=400, lam=1.6, z_range=(0.5, 19.5), M=10,
              gamma_up=-0.94, gamma_low=-0.94, nz=80)
C5 = Workload("c5_hsma3d_n999999_2to1", 0, (200.0, 200.0, 200.0), 999_999, 5,
              p=12, F=1152, K=800, lam=1.5, charges="2to1")

CONFIGS = {w.name: w for w in (C1, C2, C3, C5)}


def serving_systems(count: int = 256, n_lo: int = 500, n_hi: int = 20_000,
                    density: float = 0.05, seed0: int = 1000):
    """The serving mix: `count` independent cubic systems, N uniform in
    [n_lo, n_hi] rounded to even, side L = (N/density)^(1/3), +/-1 charges,
    p=8, F=512, K=162, lambda=1.5, seeds seed0+i."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed0 + i))
        n = int(rng.integers(n_lo, n_hi + 1))
        n -= n % 2
        L = (n / density) ** (1.0 / 3.0)
        out.append(Workload(f"serve_{i:03d}", 0, (L, L, L), n, seed0 + i,
                            p=8, F=512, K=162, lam=1.5))
    return out


def _charges(w: Workload, rng) -> np.ndarray:
    if w.charges == "pm1":
        if w.n % 2:
            raise ValueError("+/-1 systems need an even particle count")
        q = np.concatenate([np.ones(w.n // 2), -np.ones(w.n // 2)])
    elif w.charges == "2to1":
        if w.n % 3:
            raise ValueError("2:1 systems need a particle count divisible by 3")
        q = np.concatenate([np.full(w.n // 3, 2.0), np.full(2 * w.n // 3, -1.0)])
    else:
        raise ValueError(w.charges)
    rng.shuffle(q)
    return q


def _rsa(n: int, box, spacing: float, rng) -> np.ndarray:
    """Random sequential addition in a periodic box with a minimum
    (minimum-image) spacing, using a cell list."""
    box = np.asarray(box, dtype=np.float64)
    ncell = np.maximum((box // spacing).astype(int), 1)
    csize = box / ncell
    cells = {}
    pos = np.empty((n, 3))
    placed = 0
    s2 = spacing * spacing
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    while placed < n:
        cand = rng.random((4096, 3)) * box
        for x in cand:
            ci = (x // csize).astype(int) % ncell
            ok = True
            for o in offs:
                key = tuple((ci + o) % ncell)
                for j in cells.get(key, ()):
                    d = x - pos[j]
                    d -= box * np.round(d / box)
                    if d @ d < s2:
                        ok = False
                        break
                if not ok:
                    break
            if ok:
                pos[placed] = x
                cells.setdefault(tuple(ci), []).append(placed)
                placed += 1
                if placed == n:
                    break
    return pos


def make_system(w: Workload):
    """Positions (n,3), charges (n,), box_lo (3,), box_len (3,) for `w`."""
    rng = np.random.Generator(np.random.PCG64(w.seed))
    box = np.asarray(w.box, dtype=np.float64)
    if w.min_spacing > 0:
        pos = _rsa(w.n, box, w.min_spacing, rng)
    else:
        pos = rng.random((w.n, 3)) * box
    if w.z_range is not None:
        lo, hi = w.z_range
        pos[:, 2] = lo + (hi - lo) * rng.random(w.n)
    q = _charges(w, rng)
    return pos, q, np.zeros(3), box


def small_system(n: int, box, seed: int, geometry: int = 0, z_margin: float = 0.5,
                 charges: str = "pm1"):
    """A small random neutral system for tests (uniform positions)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    box = np.asarray(box, dtype=np.float64)
    pos = rng.random((n, 3)) * box
    if geometry == 1:
        pos[:, 2] = z_margin + (box[2] - 2 * z_margin) * rng.random(n)
    w = Workload("small", geometry, tuple(box), n, seed, p=0, F=0, K=0, lam=0.0,
                 charges=charges)
    q = _charges(w, rng)
    return pos, q, np.zeros(3), box
