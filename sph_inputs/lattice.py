"""Seeded cubic-lattice inputs (geometric placement on a rectangular lattice, section
"Setting up Neutron Stars": rectangle / hcp / fcc / random placement)."""
from __future__ import annotations

import math

import numpy as np


def cubic_lattice(n_side: int, L: float = 1.0):
    """Particles at ((i, j, k) + 1/2) * L / n_side, ordered with i fastest."""
    dx = L / n_side
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * dx
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return x.ravel().copy(), y.ravel().copy(), z.ravel().copy(), dx


def gaussian_velocities(n: int, sigma: float, seed: int):
    """i.i.d. N(0, sigma^2) per component (numpy PCG64), equal-mass mean removed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(0.0, sigma, size=(3, n))
    v -= v.mean(axis=1, keepdims=True)
    return v[0].copy(), v[1].copy(), v[2].copy()


def random_box(n: int, L: float, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.uniform(0.0, L, size=(3, n))
    return p[0].copy(), p[1].copy(), p[2].copy()


def cfl_dt(h, c_long, vmax, C=0.3):
    """Fixed step C * min_a h_a / (c_L,a + |v_a|) (Courant condition; the paper gives none)."""
    return float(C * np.min(np.asarray(h) / (np.asarray(c_long) + np.asarray(vmax))))
