"""Seeded synthetic workloads with the shapes of the paper's runs.

lattice(): periodic 16^3 cubic lattice of an elastic solid (Newtonian), the small case.
star():    a TOV star on spherical shells in the fixed isotropic background with a solid
           crust in the outer 1 km (mu = factor * P), any particle count.
pp_star(): the same construction for the piecewise-polytrope + thermal EoS star with the
           tabulated EoS, used for the mixed-precision / surrogate runs.
ensemble(): many independent stars of uneven sizes.
Every random draw uses numpy PCG64 with the stated seed.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import Optional

import numpy as np

from . import eos_table as eos_mod
from .lattice import cfl_dt, cubic_lattice, gaussian_velocities
from .params import MethodParams
from .star import crust_mask, l2_perturbation, place_star, profile_at, radial_perturbation, random_deviatoric
from .tov import Background, Polytrope, make_background, solve_tov

GAMMA2_K = 83.0233
GAMMA2_RHOC = 2.133857e-3
PP_RHOC = 2.255428e-3
ETA_100 = (3.0 * 100.0 / (32.0 * math.pi)) ** (1.0 / 3.0)   # about 100 neighbours with support 2h


@dataclasses.dataclass
class Workload:
    name: str
    params: MethodParams
    arrays: dict
    dt: float
    steps: int
    bg: Optional[Background] = None
    star_offsets: Optional[np.ndarray] = None      # ensembles: particle ranges per star
    star_params: Optional[np.ndarray] = None       # ensembles: (nstars, 2) = m, mu factor
    extra: Optional[dict] = None                   # workload-specific set-up data

    @property
    def n(self):
        return int(self.arrays["x"].shape[0])

    def copy_arrays(self):
        return {k: v.copy() for k, v in self.arrays.items()}


def _arrays(x, y, z, vx, vy, vz, u, h, typ):
    n = x.shape[0]
    return dict(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, u=np.asarray(u, np.float64).copy(),
                h=np.asarray(h, np.float64).copy(), S=np.zeros((6, n)),
                type=np.asarray(typ, np.int8).copy(), broken=np.zeros(n, np.uint8),
                id=np.arange(n, dtype=np.int32))


def lattice(n_side: int = 16, seed: int = 1, mu: float = 1.0, y0: float = 1e9, steps: int = 10):
    """Periodic unit box, Wendland C2, h = 1.3 dx, Gamma = 5/3 with u = 1.5 (P ~ 1), mu = 1."""
    x, y, z, dx = cubic_lattice(n_side, 1.0)
    n = x.shape[0]
    gamma, u0 = 5.0 / 3.0, 1.5
    cs = math.sqrt(gamma * (gamma - 1.0) * u0)
    vx, vy, vz = gaussian_velocities(n, 1e-3 * cs, seed)
    h = np.full(n, 1.3 * dx)
    p = MethodParams(m=dx**3, kernel="WC2", h_mode="FIXED", eta=1.3, background="NEWTONIAN",
                     periodic=True, box=1.0, eos="GAMMA_LAW", gamma=gamma, mu_mode="CONST",
                     mu_const=mu, y0_mode="CONST", y0_const=y0, break_mode="OFF")
    cL = math.sqrt(cs * cs + 4.0 * mu / 3.0)
    vmax = np.sqrt(vx * vx + vy * vy + vz * vz)
    dt = cfl_dt(h, cL, vmax)
    return Workload("lattice16", p, _arrays(x, y, z, vx, vy, vz, np.full(n, u0), h, np.ones(n)),
                    dt, steps)


@functools.lru_cache(maxsize=4)
def gamma2_background(n: int = 8192) -> Background:
    return make_background(solve_tov(Polytrope(GAMMA2_K, 2.0), GAMMA2_RHOC), n)


@functools.lru_cache(maxsize=2)
def pp_background(n: int = 8192) -> Background:
    return make_background(solve_tov(eos_mod.default_pp(), PP_RHOC), n)


@functools.lru_cache(maxsize=2)
def pp_table(nr: int = 1024, nu: int = 1024):
    return eos_mod.make_table(eos_mod.default_pp(), 1.8, nr, nu)


def _star_common(bg, N, seed, kernel, eta, l, A, mu_factor, plastic, precision, eos, gamma,
                 table, steps, name, jitter=0.05, prestress=None):
    x, y, z, rr, m = place_star(bg, N, seed, jitter)
    rho, P, u, D0 = profile_at(bg, rr)
    D0 = np.maximum(D0, D0[D0 > 0].min() if np.any(D0 > 0) else 1e-12)
    h = eta * (m / D0) ** (1.0 / 3.0)
    if l == 0:
        vx, vy, vz = radial_perturbation(x, y, z, A, bg.Rbar)
    else:
        vx, vy, vz = l2_perturbation(x, y, z, A, bg.Rbar)
    rb = np.sqrt(x * x + y * y + z * z)
    typ = crust_mask(bg, rb).astype(np.int8)
    u = np.maximum(u, np.min(u[u > 0]))
    kw = dict(m=m, kernel=kernel, h_mode="ADAPTIVE", eta=eta, background="TOV",
              bg_table=bg.table, bg_dr=bg.drbar, bg_M=bg.M, periodic=False, box=0.0,
              eos=eos, gamma=gamma, table=table, mu_mode="P_FACTOR", mu_pfactor=mu_factor,
              precision=precision)
    if plastic:
        kw.update(y0_mode="E_FACTOR", y0_over_E=0.2, break_mode="FLUIDIZE", eps_break=0.1)
    else:
        kw.update(y0_mode="CONST", y0_const=1e300, break_mode="OFF")
    p = MethodParams(**kw)
    arrays = _arrays(x, y, z, vx, vy, vz, u, h, typ)
    if prestress is not None:
        # crust particles start with a deviatoric stress whose von Mises value is k P, k drawn
        # log-uniformly in [lo, hi] (the static pressure P of the profile; seed + 1000)
        lo, hi = prestress
        rs = np.random.Generator(np.random.PCG64(seed + 1000))
        k = np.exp(rs.uniform(math.log(lo), math.log(hi), N))
        S = random_deviatoric(k * P, rs)
        S[:, typ == 0] = 0.0
        arrays["S"] = S
    # Courant step from the static profile: c_L^2 = c_s^2 + 4 mu / (3 rho)
    Pm = np.maximum(P, 1e-300)
    rhom = np.maximum(rho, 1e-300)
    hen = 1.0 + u + Pm / rhom
    cs2 = gamma * Pm / (rhom * hen) if eos == "GAMMA_LAW" else eos_mod.hybrid_eos(eos_mod.default_pp(), rhom, u)[1]
    cs2 = np.maximum(cs2, 0.0)
    cL = np.sqrt(cs2 + np.where(typ == 1, 4.0 * mu_factor * Pm / (3.0 * rhom), 0.0))
    vmag = np.sqrt(vx * vx + vy * vy + vz * vz)
    dt = cfl_dt(h, cL, vmag)
    return Workload(name, p, arrays, dt, steps, bg)


def star(N: int = 200_000, seed: int = 2, kernel: str = "WC2", eta: float = 1.3, l: int = 0,
         A: float = 1e-3, mu_factor: float = 0.01, plastic: bool = False,
         precision: str = "FP64", steps: int = 100, prestress=None):
    """Gamma = 2 polytrope star, M = 1.4, R = 12 km, Gamma-law EoS (u = K rho).  prestress =
    (lo, hi): crust particles start with von Mises stress k P, k log-uniform in [lo, hi]."""
    bg = gamma2_background()
    return _star_common(bg, N, seed, kernel, eta, l, A, mu_factor, plastic, precision,
                        "GAMMA_LAW", 2.0, None, steps, f"star{N}", prestress=prestress)


def star_2m(N: int = 2_000_000, seed: int = 3, precision: str = "FP32", steps: int = 1000):
    """2M-particle star: Wendland C4, about 100 neighbours, l = 2 with A = 1e-2, plasticity and
    maximum-strain breaking (yield strain 0.1)."""
    return star(N, seed, "WC4", ETA_100, 2, 1e-2, 0.01, True, precision, steps)


def pp_star(N: int = 2_000_000, seed: int = 3, precision: str = "FP64", eos: str = "TABLE",
            steps: int = 1000):
    """Piecewise-polytrope star with the tabulated hybrid EoS (u = u_cold on the profile)."""
    bg = pp_background()
    w = _star_common(bg, N, seed, "WC4", ETA_100, 2, 1e-2, 0.01, True, precision, "TABLE",
                     1.8, pp_table(), steps, f"ppstar{N}")
    w.params = w.params.replace(eos=eos)
    return w


def ensemble(nstars: int = 64, total: int = 8_000_000, seed: int = 5, nmin: int = 20_000, nmax: int = 500_000,
             precision: str = "FP32", steps: int = 100, gap: float = 1.2, kind: str = "pp"):
    """Independent stars of uneven sizes in one particle set: kind "pp" for the piecewise-polytrope
    star with the tabulated EoS (as pp_star; its outer 1 km crust holds 0.07% of the mass),
    "gamma2" for the Gamma = 2 polytrope with the Gamma-law EoS (crust 2.9% of the mass); both
    with Wendland C4, about 100 neighbours, plasticity and breaking.

    Sizes are log-uniform in [nmin, nmax], rescaled once to `total` and clipped to the range;
    the crust shear factor is uniform in [0.005, 0.02], the perturbation amplitude uniform in
    [1e-3, 1e-2], l = 0 or 2 with probability 1/2 each.  Stars sit on a cubic grid far enough
    apart that no particle lies within `gap` times the largest support of a particle of another
    star.  Returns a Workload whose arrays carry `star` and whose star_params holds, per star,
    (centre x, y, z, particle mass, shear factor); dt is the smallest star's CFL step."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(nmin), math.log(nmax), nstars))
    sizes = np.clip(np.rint(sizes * total / sizes.sum()), nmin, nmax).astype(np.int64)
    mus = rng.uniform(0.005, 0.02, nstars)
    amps = rng.uniform(1e-3, 1e-2, nstars)
    ells = rng.choice([0, 2], nstars)
    if kind == "pp":
        bg, eos, gamma, table = pp_background(), "TABLE", 1.8, pp_table()
    elif kind == "gamma2":
        bg, eos, gamma, table = gamma2_background(), "GAMMA_LAW", 2.0, None
    else:
        raise ValueError(kind)
    stars = [_star_common(bg, int(sizes[s]), seed * 1000 + s, "WC4", ETA_100, int(ells[s]), float(amps[s]),
                          float(mus[s]), True, precision, eos, gamma, table, steps, f"ens{s}")
             for s in range(nstars)]
    hmax = max(float(w.arrays["h"].max()) for w in stars)
    spacing = 2.0 * bg.Rbar + gap * 2.0 * hmax
    side = int(math.ceil(nstars ** (1.0 / 3.0)))
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "type", "broken")
    parts = {k: [] for k in keys}
    S, star, info = [], [], []
    for s, w in enumerate(stars):
        c = np.array([s % side, (s // side) % side, s // (side * side)], np.float64) * spacing
        a = w.arrays
        for k in keys:
            v = a[k]
            if k in ("x", "y", "z"):
                v = v + c["xyz".index(k)]
            parts[k].append(v)
        S.append(a["S"])
        star.append(np.full(w.n, s, np.int32))
        info.append([c[0], c[1], c[2], w.params.m, float(mus[s])])
    arrays = {k: np.concatenate(v) for k, v in parts.items()}
    arrays["S"] = np.concatenate(S, axis=1)
    arrays["star"] = np.concatenate(star)
    arrays["id"] = np.arange(arrays["x"].shape[0], dtype=np.int32)
    dt = min(w.dt for w in stars)
    return Workload(f"ensemble{nstars}", stars[0].params, arrays, dt, steps, bg,
                    star_offsets=np.concatenate([[0], np.cumsum(sizes)]),
                    star_params=np.asarray(info, np.float64))


GAMMA_RELAX = 1.01


def relax_star(N: int = 20_000, seed: int = 6, kind: str = "gamma2", kernel: str = "WC4", eta: float = ETA_100,
               cs_relax: float = 0.15, perturb: float = 0.1, damping_per_crossing: float = 4.0):
    """The relaxation workload of the setup section: icosahedral shells with a seeded position
    perturbation, a Gamma = 1.01 law whose sound speed is about cs_relax everywhere
    (K = cs_relax^2 / Gamma, u = K D0^(Gamma - 1) / (Gamma - 1) from the target profile at each
    particle's radius), the effective potential of the target computational density D0(rbar) of
    the static star (kind "gamma2" or "pp"), a potential wall at the star's isotropic radius and a
    velocity drag of damping_per_crossing per sound crossing time; Newtonian, fluid (no crust
    stress while relaxing).  The returned Workload carries in `extra` the profile u(rbar) of the
    real EoS for the modification step, the real star's parameters (`star_params`: the
    MethodParams of the evolution in the fixed background) and the crust types."""
    from .relax import icosahedral_star, phi_eff_table
    bg = gamma2_background() if kind == "gamma2" else pp_background()
    x, y, z, m = icosahedral_star(bg, N, seed, perturb)
    n = x.shape[0]
    rb = np.sqrt(x * x + y * y + z * z)
    D0 = np.interp(rb, bg.rbar, bg.D0)
    D0 = np.maximum(D0, 1e-3 * float(bg.D0[0]))
    G = GAMMA_RELAX
    K = cs_relax**2 / G
    u = K * D0 ** (G - 1.0) / (G - 1.0)
    h = eta * (m / D0) ** (1.0 / 3.0)
    g = phi_eff_table(bg.rbar, bg.D0, K, G)
    crossing = bg.Rbar / cs_relax
    params = MethodParams(m=m, kernel=kernel, h_mode="ADAPTIVE", eta=eta, background="NEWTONIAN", eos="GAMMA_LAW",
                          gamma=G, mu_mode="CONST", mu_const=0.0, ext_table=g, ext_dr=bg.drbar, wall_out=bg.Rbar,
                          wall_k=(4.0 * cs_relax / float(np.min(h))) ** 2, damping=damping_per_crossing / crossing)
    typ = crust_mask(bg, rb).astype(np.int8)
    arrays = _arrays(x, y, z, np.zeros(n), np.zeros(n), np.zeros(n), u, h, np.zeros(n))
    dt = cfl_dt(h, np.full(n, math.sqrt(G * K * float(D0.max()) ** (G - 1.0))), np.zeros(n))
    # the wall's own oscillation sqrt(wall_k) must be resolved too
    dt = min(dt, 0.3 / math.sqrt(params.wall_k))
    w = Workload(f"relax{n}", params, arrays, dt, 0, bg)
    if kind == "gamma2":
        real = star(n, seed, kernel, eta, 0, 0.0)
    else:
        real = pp_star(n, seed)
    w.extra = {"u_profile": np.ascontiguousarray(bg.u), "u_dr": bg.drbar, "type": typ,
               "star_params": real.params.replace(m=m), "crossing": crossing}
    return w


PAPER_K, PAPER_RHOC = 100.0, 1.28e-3     # the paper's TOV test star: K = 100, Gamma = 2


@functools.lru_cache(maxsize=1)
def paper_background(n: int = 8192) -> Background:
    return make_background(solve_tov(Polytrope(PAPER_K, 2.0), PAPER_RHOC), n)


def crust_shell(N: int = 1_000_000, seed: int = 8, rho_in_cgs: float = 7e12, rho_out_cgs: float = 4e12,
                mu_cgs: float = 1e29, solid: bool = True, amp: float = 1e-3, kernel: str = "WC2", eta: float = 1.3,
                wall_layers: float = 0.25):
    """The crust-shell workload of section "Neutron stars with a solid crust in SPH": the part of
    the paper's 1.4 Msun polytrope (K = 100, Gamma = 2, rho_c = 0.00128) between the densities
    rho_in_cgs and rho_out_cgs (7e12 and 4e12 g/cm^3: a shell about 0.06 km thick at r = 9.5),
    Newtonian, held by the effective potential of that density profile (g = K Gamma rho^(Gamma-2)
    d rho / dr along the areal radius) and by potential walls at its two faces; constant shear
    modulus mu_cgs (1e29 erg/cm^3; 0 for the fluid comparison with solid=False), no yield, no
    breaking.  Particles sit on icosahedral layers, as many as the shell holds at the spacing that
    N particles give (two at 1M).  The imposed velocity, stored in extra["v_tor"], is the l = 2
    toroidal field v = amp v_s 3 sin(theta) cos(theta) e_phi with v_s = sqrt(mu / rho) the shear
    speed (the state itself starts at rest, for the radial settling the paper's walls need first).
    Wall stiffness: a wall displacement of wall_layers spacings balances the pressure push
    c_s^2 / spacing on a face layer."""
    from .relax import icosphere
    from .star import _random_rotation
    from .tov import C_CGS, DENSITY_UNIT_CGS, areal_radius, density_from_cgs
    bg = paper_background()
    r_all = areal_radius(bg, bg.rbar)
    rho = bg.rho
    inside = rho > 0
    r_of_rho = lambda q: float(np.interp(q, rho[inside][::-1], r_all[inside][::-1]))
    rin, rout = r_of_rho(density_from_cgs(rho_in_cgs)), r_of_rho(density_from_cgs(rho_out_cgs))
    # enclosed (Newtonian) shell mass on a fine radial grid
    rr = np.linspace(rin, rout, 4001)
    rho_r = np.interp(rr, r_all, rho)
    dm = 4.0 * math.pi * rr**2 * rho_r
    mcum = np.concatenate([[0.0], np.cumsum(0.5 * (dm[1:] + dm[:-1]) * np.diff(rr))])
    Ms = float(mcum[-1])
    m0 = Ms / N
    ell = (m0 / float(rho_r.mean())) ** (1.0 / 3.0)
    layers = max(1, int(math.ceil((rout - rin) / ell)))
    rng = np.random.Generator(np.random.PCG64(seed))
    pts, radii = [], []
    per = N / layers
    for k in range(layers):
        rk = float(np.interp((k + 0.5) / layers * Ms, mcum, rr))
        f = max(1, int(round(math.sqrt(max(per - 2.0, 0.0) / 10.0))))
        P = icosphere(f) @ _random_rotation(rng).T
        pts.append(P * rk)
        radii.append(np.full(P.shape[0], rk))
    X = np.concatenate(pts)
    n = X.shape[0]
    m = Ms / n
    x, y, z = X[:, 0].copy(), X[:, 1].copy(), X[:, 2].copy()
    r = np.sqrt(x * x + y * y + z * z)
    rho_p = np.interp(r, r_all, rho)
    K, G = PAPER_K, 2.0
    u = K * rho_p ** (G - 1.0) / (G - 1.0)
    # smoothing length from the larger of the volume spacing (m / rho)^(1/3) and the spacing within a
    # layer, sqrt(4 pi r^2 / particles per layer): a layer thinner than the volume spacing would
    # otherwise leave a particle with a handful of neighbours
    in_layer = np.sqrt(4.0 * math.pi * r**2 / (n / layers))
    h = eta * np.maximum((m / rho_p) ** (1.0 / 3.0), in_layer)
    # effective potential of the shell's profile on a grid from 0 to past the outer face
    dr = (rout - rin) / 400.0
    grid = np.arange(0.0, rout + 50 * dr, dr)
    rho_g = np.interp(grid, r_all, rho)
    rho_g = np.maximum(rho_g, 1e-3 * float(rho_p.min()))
    g = K * G * rho_g ** (G - 2.0) * np.gradient(rho_g, grid)
    mu = mu_cgs / (DENSITY_UNIT_CGS * C_CGS**2) if solid else 0.0
    cs2 = G * K * rho_p ** (G - 1.0)
    spacing = (m / float(rho_p.mean())) ** (1.0 / 3.0)
    wall_k = float(cs2.max()) / spacing / (wall_layers * spacing)
    params = MethodParams(m=m, kernel=kernel, h_mode="FIXED", eta=eta, background="NEWTONIAN", eos="GAMMA_LAW",
                          gamma=G, mu_mode="CONST", mu_const=mu, y0_mode="CONST", y0_const=1e300, break_mode="OFF",
                          ext_table=np.ascontiguousarray(g), ext_dr=dr, wall_in=rin, wall_out=rout, wall_k=wall_k)
    typ = np.ones(n, np.int8) if solid else np.zeros(n, np.int8)
    arrays = _arrays(x, y, z, np.zeros(n), np.zeros(n), np.zeros(n), u, h, typ)
    vs = math.sqrt(mu_cgs / (DENSITY_UNIT_CGS * C_CGS**2) / float(rho_p.mean()))
    rc = np.sqrt(x * x + y * y)
    ct, st_ = z / r, rc / r
    vphi = amp * vs * 3.0 * st_ * ct
    ephi = np.stack([-y / np.maximum(rc, 1e-300), x / np.maximum(rc, 1e-300), np.zeros(n)])
    v_tor = ephi * vphi
    cL = np.sqrt(cs2 + 4.0 * mu / (3.0 * rho_p))
    dt = min(cfl_dt(h, cL, np.zeros(n)), 0.3 / math.sqrt(wall_k))
    w = Workload(f"shell{n}", params, arrays, dt, 0, bg)
    w.extra = {"v_tor": v_tor, "r_in": rin, "r_out": rout, "layers": layers, "v_shear": vs, "R": bg.R, "M": bg.M,
               "mu": mu, "rho_mean": float(rho_p.mean())}
    return w
