"""Seeded set-up of a neutron star for relaxation (section "Setting up Neutron Stars").

The paper's recipe, which this module prepares the inputs for:
  1. particles on concentric spherical shells, each an icosahedral grid (a subdivided
     icosahedron, 10 f^2 + 2 points), shell radii following the TOV density profile;
  2. a random perturbation of the positions (to avoid lattice artefacts);
  3. relaxation in an external effective potential built from the desired density profile:
     with P = K rho^Gamma, equilibrium of dv/dt = -grad P / rho + g_eff needs
     g_eff = -grad phi_eff = K Gamma rho^(Gamma - 2) grad rho, phi_eff = -K Gamma rho^(Gamma-1)/(Gamma-1),
     plus potential walls that confine the particles; Gamma close to 1 (1.01 here) makes the
     sound speed almost uniform, sqrt(Gamma K rho^(Gamma - 1)), so relaxation time steps are not
     set by the stiff centre;
  4. a modification step that assigns the real EoS's u for the profile density rho(r), after
     which the star is evolved (and perturbed) in the fixed background.
Steps 3 and 4 run through the particle loop itself (external potential, walls and drag in the
force pass; the modification step as its own call); this module only builds the tables and the
initial arrays.  The relaxation works on the computational density D0 = rho psi^6 of the static
star, the density the SPH sum recovers, so that the relaxed particles follow the star in its
isotropic coordinates.  Every random draw uses numpy PCG64 with the stated seed.
"""
from __future__ import annotations

import math

import numpy as np

from .star import _random_rotation
from .tov import Background


def icosphere(f: int) -> np.ndarray:
    """The 10 f^2 + 2 vertices of an icosahedron whose edges are divided into f segments,
    projected onto the unit sphere (f >= 1)."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t],
                  [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    pts = {}
    for a, b, c in F:
        A, B, C = V[a], V[b], V[c]
        for i in range(f + 1):
            for j in range(f + 1 - i):
                # integer barycentric key shared by faces that meet at an edge or corner
                wa, wb, wc = f - i - j, i, j
                key = tuple(sorted(((a, wa), (b, wb), (c, wc)), key=lambda q: q[0]))
                key = tuple((v, w) for v, w in key if w > 0)
                if key not in pts:
                    p = (wa * A + wb * B + wc * C) / f
                    pts[key] = p / np.linalg.norm(p)
    P = np.array(list(pts.values()))
    assert P.shape[0] == 10 * f * f + 2, (P.shape, f)
    return P


def icosahedral_star(bg: Background, N: int, seed: int, perturb: float = 0.1):
    """Particles on concentric icosahedral shells following the static star's computational
    density D0(rbar), each shell randomly rotated, then displaced by a seeded Gaussian of
    `perturb` times the local spacing per component.  The shell counts 10 f^2 + 2 fix the
    particle number near N; returns (x, y, z, m) with m = M_b / (particles placed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Mb = bg.mc[-1]
    m0 = Mb / N

    def mc_of(r):
        return float(np.interp(r, bg.rbar, bg.mc))

    def r_of_mc(q):
        return float(np.interp(q, bg.mc, bg.rbar))

    def ell(r):
        D = float(np.interp(r, bg.rbar, bg.D0))
        return (m0 / max(D, 1e-300)) ** (1.0 / 3.0)

    shells = []          # (radius, count)
    placed = 0
    # the centre holds one particle
    shells.append((0.0, 1))
    placed = 1
    while True:
        r_in = r_of_mc(placed * m0)
        rem = N - placed
        if rem <= 0:
            break
        r_mid = min(r_in + 0.5 * ell(r_in), bg.Rbar)
        f = max(1, int(round(math.sqrt(max(4.0 * math.pi * r_mid**2 / ell(r_mid) ** 2 - 2.0, 0.0) / 10.0))))
        cnt = 10 * f * f + 2
        if rem < cnt:
            # the last layer: the icosahedral grid whose count is nearest to what is left
            f = max(1, int(round(math.sqrt(max(rem - 2, 0) / 10.0))))
            cnt = 10 * f * f + 2
            shells.append((r_of_mc(min(placed + 0.5 * cnt, N) * m0), cnt))
            placed += cnt
            break
        shells.append((r_of_mc((placed + 0.5 * cnt) * m0), cnt))
        placed += cnt
    m = Mb / placed
    pts = [np.zeros((1, 3))]
    for r, cnt in shells[1:]:
        f = int(round(math.sqrt((cnt - 2) / 10.0)))
        P = icosphere(f) @ _random_rotation(rng).T
        pts.append(P * r)
    X = np.concatenate(pts)
    rr = np.linalg.norm(X, axis=1)
    loc = np.array([(m / max(float(np.interp(r, bg.rbar, bg.D0)), 1e-300)) ** (1.0 / 3.0) for r in rr])
    X = X + rng.normal(size=X.shape) * (perturb * loc)[:, None]
    return X[:, 0].copy(), X[:, 1].copy(), X[:, 2].copy(), m


def phi_eff_table(rbar: np.ndarray, D: np.ndarray, K: float, Gamma: float, floor_frac: float = 1e-3):
    """Radial acceleration g(rbar_i) = K Gamma D^(Gamma - 2) dD/drbar (outward positive) of the
    effective potential phi_eff = -K Gamma D^(Gamma - 1) / (Gamma - 1) that holds the density
    profile D(rbar) in equilibrium with P = K D^Gamma; rbar must be uniform.  The density is
    floored at floor_frac of its maximum, where the profile ends at the surface."""
    D = np.maximum(np.asarray(D, np.float64), floor_frac * float(np.max(D)))
    phi = -K * Gamma * D ** (Gamma - 1.0) / (Gamma - 1.0)
    g = -np.gradient(phi, rbar)
    return np.ascontiguousarray(g)
