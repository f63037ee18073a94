"""Seeded particle placement for a static TOV star in isotropic coordinates.

The paper places neutron-star particles on concentric spherical shells whose radial
distribution follows the TOV density profile (section "Setting up Neutron Stars").  Here
each shell holds the baryon mass of a layer one local particle spacing thick,
ell = (m / D0)^(1/3) with D0 = rho psi^6 the static computational density, and its
particles sit on a Fibonacci sphere with a random rotation and a small tangential jitter.
Velocity perturbations follow the paper's oscillation tests (section "Spherically
symmetric and static neutron star tests"): a radial profile for l = 0 and
A sin(pi rbar/Rbar) d_theta P_l(cos theta) along e_theta for l > 0.
"""
from __future__ import annotations

import math

import numpy as np

from .tov import KM, Background, areal_radius

GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _fibonacci_sphere(k: int):
    i = np.arange(k, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / k
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * GOLDEN_ANGLE
    return np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=1)


def place_star(bg: Background, N: int, seed: int, jitter: float = 0.05):
    """Return (x, y, z, shell_radius, m) of N equal-mass particles; m = M_b / N."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Mb = bg.mc[-1]
    m = Mb / N

    def mc_of(r):
        return float(np.interp(r, bg.rbar, bg.mc))

    def ell(r):
        D = float(np.interp(r, bg.rbar, bg.D0))
        return (m / max(D, 1e-300)) ** (1.0 / 3.0)

    edges = [0.0]
    # central cell: a sphere holding one particle mass
    r1 = (3.0 * m / (4.0 * math.pi * bg.D0[0])) ** (1.0 / 3.0)
    edges.append(min(r1, bg.Rbar))
    while edges[-1] < bg.Rbar:
        r_in = edges[-1]
        r_out = r_in + ell(r_in)
        for _ in range(3):
            r_out = r_in + ell(min(0.5 * (r_in + r_out), bg.Rbar))
        if r_out >= bg.Rbar or Mb - mc_of(r_out) < 1.5 * m:
            r_out = bg.Rbar
        edges.append(r_out)
    edges = np.asarray(edges)
    cum = np.rint(np.array([mc_of(r) for r in edges]) / m).astype(np.int64)
    cum[-1] = N
    cum = np.maximum.accumulate(cum)
    counts = np.diff(cum)
    # a last shell holding under a tenth of the particles of the one below (a tenuous envelope)
    # is merged into it: its few particles would otherwise need supports spanning the star
    while len(counts) > 2 and 0 < counts[-1] < 0.1 * counts[-2]:
        counts = np.append(counts[:-2], counts[-2] + counts[-1])
        edges = np.append(edges[:-2], edges[-1])
    pts, radii = [], []
    for k, cnt in enumerate(counts):
        if cnt <= 0:
            continue
        target = 0.5 * (mc_of(edges[k]) + mc_of(edges[k + 1]))
        rk = float(np.interp(target, bg.mc, bg.rbar))
        if cnt == 1 and k == 0:
            pts.append(np.zeros((1, 3)))
            radii.append(np.zeros(1))
            continue
        p = _fibonacci_sphere(int(cnt)) @ _random_rotation(rng).T
        if jitter > 0:
            t = rng.normal(scale=jitter * ell(rk) / max(rk, 1e-300), size=p.shape)
            t -= (t * p).sum(axis=1, keepdims=True) * p       # tangential only
            p = p + t
            p /= np.linalg.norm(p, axis=1, keepdims=True)
        pts.append(p * rk)
        radii.append(np.full(int(cnt), rk))
    P = np.concatenate(pts)
    rr = np.concatenate(radii)
    assert P.shape[0] == N, (P.shape, N)
    return P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy(), rr, m


def profile_at(bg: Background, rbar):
    """Static profile (rho, P, u, D0) at isotropic radius rbar (zero outside the star)."""
    rbar = np.asarray(rbar, dtype=np.float64)
    f = lambda arr: np.interp(rbar, bg.rbar, arr, right=0.0)
    return f(bg.rho), f(bg.P), f(bg.u), f(bg.D0)


def crust_mask(bg: Background, rbar, depth_km: float = 1.0):
    """Solid crust = areal radius within depth_km of the surface."""
    return areal_radius(bg, rbar) > bg.R - depth_km * KM


def radial_perturbation(x, y, z, A, Rbar):
    """xdot = A sin(pi rbar / Rbar) n (l = 0, n = 1 member of the paper's family)."""
    r = np.sqrt(x * x + y * y + z * z)
    s = A * np.sin(np.pi * np.minimum(r, Rbar) / Rbar)
    with np.errstate(invalid="ignore", divide="ignore"):
        f = np.where(r > 0, s / np.where(r > 0, r, 1.0), 0.0)
    return f * x, f * y, f * z


def l2_perturbation(x, y, z, A, Rbar):
    """delta v_theta = A sin(pi rbar / Rbar) d_theta P_2(cos theta), m = 0: d_theta P_2 = -3 cos sin."""
    r = np.sqrt(x * x + y * y + z * z)
    rs = np.where(r > 0, r, 1.0)
    ct = np.where(r > 0, z / rs, 1.0)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    rxy = np.sqrt(x * x + y * y)
    cphi = np.where(rxy > 0, x / np.where(rxy > 0, rxy, 1.0), 1.0)
    sphi = np.where(rxy > 0, y / np.where(rxy > 0, rxy, 1.0), 0.0)
    vth = A * np.sin(np.pi * np.minimum(r, Rbar) / Rbar) * (-3.0 * ct * st)
    vth = np.where(r > 0, vth, 0.0)
    # e_theta = (cos t cos p, cos t sin p, -sin t)
    return vth * ct * cphi, vth * ct * sphi, -vth * st


def random_deviatoric(scale, rng):
    """Random traceless symmetric tensors (6, n: xx, yy, zz, xy, xz, yz) with von Mises stress
    sqrt(3/2 S:S) equal to `scale` (an array of n), directions drawn from rng."""
    scale = np.asarray(scale, np.float64)
    n = scale.shape[0]
    A = rng.normal(size=(n, 3, 3))
    A = 0.5 * (A + np.transpose(A, (0, 2, 1)))
    A -= np.trace(A, axis1=1, axis2=2)[:, None, None] / 3.0 * np.eye(3)
    sv = np.sqrt(1.5 * (A * A).sum(axis=(1, 2)))
    A *= (scale / sv)[:, None, None]
    return np.stack([A[:, 0, 0], A[:, 1, 1], A[:, 2, 2], A[:, 0, 1], A[:, 0, 2], A[:, 1, 2]])
