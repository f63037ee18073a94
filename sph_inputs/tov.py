"""Host-side FP64 setup of a static neutron star in the fixed-background method.

Geometric units G = c = Msun = 1 throughout (section "Fixed metric background",
conventions (a)-(c)).  This module solves the TOV structure equations (section
"Setting up Neutron Stars", the s = r^2 / theta form of the TOV system) for a cold
barotropic equation of state and tabulates the static background that the particle
loop reads: lapse alpha and conformal factor psi of the 3+1 metric (section "Fixed
metric background", the 3+1 line element) in isotropic coordinates, plus the
density profile used to place particles.

The TOV system is integrated with the log-enthalpy H = ln(1 + u + P/rho) as the
independent variable.  This is the same system as the paper's theta form (theta is
a monotone function of H for a polytrope), written so that the surface is reached
exactly at H = 0.  For a perfect fluid in hydrostatic equilibrium dH = -dPhi, so
the lapse inside the star is alpha = sqrt(1 - 2M/R) * exp(-H).

This is setup code: it generates inputs that both the GPU path and the CPU oracle
consume as data.  It is not on the per-step hot path.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.integrate import solve_ivp

# Physical constants (cgs) for unit conversions only.
G_CGS = 6.67430e-8
C_CGS = 2.99792458e10
MSUN_CGS = 1.98847e33
LENGTH_UNIT_CM = G_CGS * MSUN_CGS / C_CGS**2          # 1 geometric length in cm
KM = 1.0e5 / LENGTH_UNIT_CM                           # 1 km in geometric units
DENSITY_UNIT_CGS = MSUN_CGS / LENGTH_UNIT_CM**3       # g/cm^3 per geometric density


def density_to_cgs(rho: float) -> float:
    return rho * DENSITY_UNIT_CGS


def density_from_cgs(rho_cgs: float) -> float:
    return rho_cgs / DENSITY_UNIT_CGS


def polytrope_K_to_cgs(K: float, Gamma: float) -> float:
    """Convert the polytropic constant of P = K rho^Gamma to cgs units."""
    return K * DENSITY_UNIT_CGS ** (1.0 - Gamma) * C_CGS**2


class Polytrope:
    """Cold polytrope P = K rho^Gamma, u = K rho^(Gamma-1)/(Gamma-1) (eq. poly_eos and
    the relativistic sound-speed passage, where u follows from u = int P/rho^2 drho)."""

    def __init__(self, K: float, Gamma: float):
        self.K = float(K)
        self.Gamma = float(Gamma)

    def from_rho(self, rho):
        rho = np.asarray(rho, dtype=np.float64)
        K, G = self.K, self.Gamma
        P = K * rho**G
        u = K * rho ** (G - 1.0) / (G - 1.0)
        return P, u

    def from_enthalpy(self, H):
        """(rho, P, u) for log-enthalpy H >= 0; h = 1 + u + P/rho = 1 + K G rho^(G-1)/(G-1)."""
        K, G = self.K, self.Gamma
        h = np.exp(np.maximum(H, 0.0))
        rho = ((h - 1.0) * (G - 1.0) / (K * G)) ** (1.0 / (G - 1.0))
        P, u = self.from_rho(rho)
        return rho, P, u

    def dPdrho(self, rho):
        return self.K * self.Gamma * np.asarray(rho) ** (self.Gamma - 1.0)


class PiecewisePolytrope:
    """Cold piecewise polytrope (P = K_i rho^Gamma_i on [rho_{i-1}, rho_i)), continuous in P and
    u; the construction the paper cites for refining crust and core with several polytropes.
    K_{i+1} and the additive energy constants a_i follow from continuity."""

    def __init__(self, K1: float, Gammas, rho_divs):
        self.Gammas = np.asarray(Gammas, dtype=np.float64)
        self.rho_divs = np.asarray(rho_divs, dtype=np.float64)
        assert len(self.rho_divs) == len(self.Gammas) - 1
        K = [float(K1)]
        for i, rd in enumerate(self.rho_divs):
            K.append(K[i] * rd ** (self.Gammas[i] - self.Gammas[i + 1]))
        self.Ks = np.asarray(K)
        a = [0.0]
        for i, rd in enumerate(self.rho_divs):
            Gi, Gj = self.Gammas[i], self.Gammas[i + 1]
            a.append(a[i] + K[i] * rd ** (Gi - 1) / (Gi - 1) - K[i + 1] * rd ** (Gj - 1) / (Gj - 1))
        self.a = np.asarray(a)
        # enthalpy at the dividing densities, for the inverse map
        self.h_divs = np.array([self._h_piece(i, rd) for i, rd in enumerate(self.rho_divs)])

    def piece(self, rho):
        return np.searchsorted(self.rho_divs, np.asarray(rho, dtype=np.float64), side="right")

    def _h_piece(self, i, rho):
        G, K = self.Gammas[i], self.Ks[i]
        return 1.0 + self.a[i] + K * G * rho ** (G - 1) / (G - 1)

    def from_rho(self, rho):
        rho = np.asarray(rho, dtype=np.float64)
        i = self.piece(rho)
        G, K, a = self.Gammas[i], self.Ks[i], self.a[i]
        P = K * rho**G
        u = a + K * rho ** (G - 1) / (G - 1)
        return P, u

    def gamma_of(self, rho):
        return self.Gammas[self.piece(rho)]

    def dPdrho(self, rho):
        rho = np.asarray(rho, dtype=np.float64)
        i = self.piece(rho)
        return self.Ks[i] * self.Gammas[i] * rho ** (self.Gammas[i] - 1)

    def from_enthalpy(self, H):
        h = np.exp(np.maximum(np.asarray(H, dtype=np.float64), 0.0))
        i = np.searchsorted(self.h_divs, h, side="right")
        G, K, a = self.Gammas[i], self.Ks[i], self.a[i]
        x = np.maximum(h - 1.0 - a, 0.0) * (G - 1) / (K * G)
        rho = x ** (1.0 / (G - 1))
        P, u = self.from_rho(rho)
        return rho, P, u


@dataclasses.dataclass
class TOVStar:
    eos: object
    rho_c: float
    M: float            # gravitational mass
    R: float            # areal radius
    Rbar: float         # isotropic radius of the surface
    M_b: float          # baryon mass
    # fine samples along the solution, centre -> surface
    H: np.ndarray
    r: np.ndarray
    m: np.ndarray
    rbar: np.ndarray
    mb: np.ndarray      # enclosed baryon mass

    def surface_lapse(self):
        return math.sqrt(1.0 - 2.0 * self.M / self.R)


def solve_tov(eos, rho_c: float, nsamp: int = 200001) -> TOVStar:
    """Integrate the TOV equations from the centre to the surface.

    dr/dH = -r (r - 2m) / (m + 4 pi r^3 P),  dm/dH = 4 pi r^2 eps dr/dH  (eps = rho (1+u)),
    d ln rbar/dH = dr/dH / (r sqrt(1 - 2m/r)),  dmb/dH = 4 pi r^2 rho / sqrt(1-2m/r) dr/dH.
    """
    Pc, uc = eos.from_rho(rho_c)
    Pc, uc = float(Pc), float(uc)
    Hc = math.log(1.0 + uc + Pc / rho_c)
    epsc = rho_c * (1.0 + uc)

    def rhs(H, y):
        r, m, lnrb, mb = y
        rho, P, u = eos.from_enthalpy(H)
        eps = rho * (1.0 + u)
        drdH = -r * (r - 2.0 * m) / (m + 4.0 * math.pi * r**3 * P)
        sq = math.sqrt(1.0 - 2.0 * m / r)
        return [drdH,
                4.0 * math.pi * r * r * eps * drdH,
                drdH / (r * sq),
                4.0 * math.pi * r * r * rho / sq * drdH]

    # series start: H = Hc - (2 pi / 3)(eps_c + 3 P_c) r^2 near the centre
    dH = Hc * 1e-9
    r0 = math.sqrt(3.0 * dH / (2.0 * math.pi * (epsc + 3.0 * Pc)))
    m0 = 4.0 / 3.0 * math.pi * r0**3 * epsc
    mb0 = 4.0 / 3.0 * math.pi * r0**3 * rho_c
    t = np.linspace(math.sqrt(dH / Hc), 1.0, nsamp)
    Hs = Hc - Hc * t**2
    Hs[0] = Hc - dH
    Hs[-1] = 0.0
    sol = solve_ivp(rhs, [Hc - dH, 0.0], [r0, m0, math.log(r0), mb0], method="DOP853",
                    rtol=1e-12, atol=1e-15, t_eval=Hs[1:], dense_output=False)
    if not sol.success:
        raise RuntimeError("TOV integration failed: " + sol.message)
    r = np.concatenate([[0.0, r0], sol.y[0]])
    m = np.concatenate([[0.0, m0], sol.y[1]])
    lnrb = np.concatenate([[math.log(r0)], sol.y[2]])
    mb = np.concatenate([[0.0, mb0], sol.y[3]])
    Hall = np.concatenate([[Hc], Hs])
    R, M = r[-1], m[-1]
    Rbar = 0.5 * (R - M + math.sqrt(R * R - 2.0 * M * R))
    shift = math.log(Rbar) - lnrb[-1]
    rbar = np.concatenate([[0.0], np.exp(lnrb + shift)])
    return TOVStar(eos=eos, rho_c=float(rho_c), M=float(M), R=float(R), Rbar=float(Rbar),
                   M_b=float(mb[-1]), H=Hall, r=r, m=m, rbar=rbar, mb=mb)


@dataclasses.dataclass
class Background:
    """Static isotropic background on a uniform rbar grid, rbar_i = i * Rbar/(n-1).

    table[0] = alpha, table[1] = d alpha/d rbar, table[2] = psi, table[3] = d psi/d rbar.
    Outside rbar > Rbar the exterior isotropic Schwarzschild solution with mass M applies.
    rho, P, u, D0 (= rho psi^6, the static computational density) and mc (enclosed baryon
    mass) describe the star on the same grid.
    """
    M: float
    Rbar: float
    R: float
    table: np.ndarray          # (4, n) float64, C-contiguous
    rbar: np.ndarray
    rho: np.ndarray
    P: np.ndarray
    u: np.ndarray
    D0: np.ndarray
    mc: np.ndarray

    @property
    def n(self):
        return self.table.shape[1]

    @property
    def drbar(self):
        return self.Rbar / (self.n - 1)


def exterior_metric(rbar, M):
    """Isotropic Schwarzschild exterior: psi = 1 + M/(2 rbar), alpha = (1 - M/2rbar)/(1 + M/2rbar)."""
    rbar = np.asarray(rbar, dtype=np.float64)
    a = M / (2.0 * rbar)
    psi = 1.0 + a
    alpha = (1.0 - a) / (1.0 + a)
    dpsi = -a / rbar
    dalpha = 2.0 / (1.0 + a) ** 2 * a / rbar
    return alpha, dalpha, psi, dpsi


def make_background(star: TOVStar, n: int = 8192) -> Background:
    rb = np.linspace(0.0, star.Rbar, n)
    # interpolate the solution samples (monotone in rbar) onto the grid
    r = np.interp(rb, star.rbar, star.r)
    m = np.interp(rb, star.rbar, star.m)
    H = np.interp(rb, star.rbar, star.H)
    mc = np.interp(rb, star.rbar, star.mb)
    rho, P, u = star.eos.from_enthalpy(H)
    rho = np.where(H > 0, rho, 0.0)
    P = np.where(H > 0, P, 0.0)
    alpha = star.surface_lapse() * np.exp(-H)
    with np.errstate(invalid="ignore", divide="ignore"):
        psi = np.sqrt(np.where(rb > 0, r / np.where(rb > 0, rb, 1.0), 1.0))
        sq = np.sqrt(1.0 - 2.0 * np.where(r > 0, m / np.where(r > 0, r, 1.0), 0.0))
        drdrb = psi**2 * sq
        dPhidr = (m + 4.0 * math.pi * r**3 * P) / (r * (r - 2.0 * m))
        dalpha = np.where(rb > 0, alpha * dPhidr * drdrb, 0.0)
        dpsi = np.where(rb > 0, psi / (2.0 * np.where(rb > 0, rb, 1.0)) * (sq - 1.0), 0.0)
    # centre values from the regular limits
    psi[0] = math.sqrt((star.r[1] / star.rbar[1]))
    table = np.ascontiguousarray(np.stack([alpha, dalpha, psi, dpsi]).astype(np.float64))
    D0 = rho * psi**6
    return Background(M=star.M, Rbar=star.Rbar, R=star.R, table=table, rbar=rb, rho=rho, P=P,
                      u=u, D0=D0, mc=mc)


def areal_radius(bg: Background, rbar):
    """Areal radius r = psi^2 rbar for isotropic radius rbar (inside: table psi; outside: exterior)."""
    rbar = np.asarray(rbar, dtype=np.float64)
    psi_in = np.interp(rbar, bg.rbar, bg.table[2])
    psi_out = 1.0 + bg.M / (2.0 * np.maximum(rbar, 1e-300))
    psi = np.where(rbar <= bg.Rbar, psi_in, psi_out)
    return psi**2 * rbar
