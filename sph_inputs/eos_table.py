"""Synthetic tabulated equation of state: a cold piecewise polytrope plus a thermal Gamma-law part.

Above the cold curve (u >= u_cold(rho)) the usual hybrid form
    P = P_cold(rho) + (Gamma_th - 1) rho (u - u_cold(rho))
(the piecewise polytrope is the construction the paper cites for crust/core EoS refinement).
Below the cold curve, where the linear thermal term would drive P negative, the pressure
continues as P = P_cold exp(X), X = (Gamma_th - 1) rho (u - u_cold) / P_cold, which matches the
hybrid form in value and first derivative at u = u_cold and stays positive.
Relativistic sound speed c_s^2 = (dP/drho at fixed entropy) / h, h = 1 + u + P/rho:
    above: (Gamma_i P_cold + Gamma_th P_th) / rho
    below: (P / rho) (Gamma_i + X (1 - Gamma_i) + (Gamma_th - 1)(e^X - 1))
Both are positive for Gamma_i > Gamma_th - 1, so every (rho, u) in the table range is valid.
"""
from __future__ import annotations

import math

import numpy as np

from .params import EosTable
from .tov import PiecewisePolytrope, density_from_cgs


def default_pp() -> PiecewisePolytrope:
    """3-piece cold EoS: Gamma = 1.35 / 3.0 / 2.7 split at 10^14.7 and 10^15 g/cm^3."""
    return PiecewisePolytrope(0.41817, [1.35, 3.0, 2.7],
                              [density_from_cgs(10 ** 14.7), density_from_cgs(1e15)])


def hybrid_eos(pp: PiecewisePolytrope, rho, u, gamma_th: float = 1.8):
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    Pc, uc = pp.from_rho(rho)
    Gc = pp.gamma_of(rho)
    g1 = gamma_th - 1.0
    Pth = g1 * rho * (u - uc)
    above = u >= uc
    X = np.where(above, 0.0, Pth / Pc)
    P = np.where(above, Pc + Pth, Pc * np.exp(X))
    h = 1.0 + u + P / rho
    dPdrho = np.where(above, (Gc * Pc + gamma_th * Pth) / rho,
                      P / rho * (Gc + X * (1.0 - Gc) + g1 * np.expm1(X)))
    cs2 = dPdrho / h
    return P, cs2


def make_table(pp: PiecewisePolytrope, gamma_th: float = 1.8, nr: int = 1024, nu: int = 1024,
               rho_range=(1e-10, 1e-2), u_range=(1e-5, 2.0)) -> EosTable:
    lnr = np.linspace(math.log(rho_range[0]), math.log(rho_range[1]), nr)
    lnu = np.linspace(math.log(u_range[0]), math.log(u_range[1]), nu)
    rho = np.exp(lnr)[:, None]
    u = np.exp(lnu)[None, :]
    P, cs2 = hybrid_eos(pp, rho, u, gamma_th)
    ok = (P > 0) & (cs2 > 0) & np.isfinite(P) & np.isfinite(cs2)
    with np.errstate(invalid="ignore", divide="ignore"):
        lnP = np.where(ok, np.log(np.where(ok, P, 1.0)), np.nan)
        lncs2 = np.where(ok, np.log(np.where(ok, cs2, 1.0)), np.nan)
    return EosTable(lnP=np.ascontiguousarray(lnP), lncs2=np.ascontiguousarray(lncs2),
                    lnr0=float(lnr[0]), dlnr=float(lnr[1] - lnr[0]),
                    lnu0=float(lnu[0]), dlnu=float(lnu[1] - lnu[0]))


MLP_HIDDEN = 64
MLP_NPARAM = 2 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 2 * 64 + 2


def mlp_init(seed: int = 4) -> np.ndarray:
    """Initial parameters of the 2-64-64-64-2 surrogate (flat layout W1, b1, W2, b2, W3, b3, W4,
    b4 with W[out][in]): uniform in +-sqrt(6 / (fan_in + fan_out)) (Glorot), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((2, 64), (64, 64), (64, 64), (64, 2)):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-a, a, fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    w = np.concatenate(parts).astype(np.float32)
    assert w.shape == (MLP_NPARAM,)
    return w


def mlp_samples(table: EosTable, n: int = 1_000_000, seed: int = 4) -> np.ndarray:
    """Training inputs (ln rho, ln u), uniform over the table's box."""
    rng = np.random.default_rng(seed)
    nr, nu = table.lnP.shape
    lnr = table.lnr0 + rng.uniform(0.0, 1.0, n) * (nr - 1) * table.dlnr
    lnu = table.lnu0 + rng.uniform(0.0, 1.0, n) * (nu - 1) * table.dlnu
    return np.ascontiguousarray(np.stack([lnr, lnu], axis=1))


def mlp_band_samples(pp: PiecewisePolytrope, lnr_lo: float, lnr_hi: float, width: float, n: int,
                     seed: int = 4) -> np.ndarray:
    """Training inputs (ln rho, ln u) in a band around the cold curve: ln rho uniform in
    [lnr_lo, lnr_hi], ln u = ln u_cold(rho) + a uniform offset in [-width, width]."""
    rng = np.random.default_rng(seed)
    lnr = rng.uniform(lnr_lo, lnr_hi, n)
    _, uc = pp.from_rho(np.exp(lnr))
    lnu = np.log(uc) + rng.uniform(-width, width, n)
    return np.ascontiguousarray(np.stack([lnr, lnu], axis=1))


def band_domain(pp: PiecewisePolytrope, lnr_lo: float, lnr_hi: float, width: float):
    """The box (lnr_lo, lnr_hi, lnu_lo, lnu_hi) around that band."""
    lnr = np.linspace(lnr_lo, lnr_hi, 4097)
    _, uc = pp.from_rho(np.exp(lnr))
    lnu = np.log(uc)
    return float(lnr_lo), float(lnr_hi), float(lnu.min() - width), float(lnu.max() + width)


def piece_band(pp: PiecewisePolytrope, piece: int, rho_c: float, table: EosTable, width: float = 0.06):
    """One polytrope piece of a star with central density rho_c, between the first table node
    above its lower dividing density and the last node below its upper one (table cells across a
    division interpolate over the jump of c_s^2 there), the densest piece up to 1.15 rho_c (the
    particles' densities overshoot the profile's centre a little), with a band of +-width in
    ln u: the (ln rho_lo, ln rho_hi, width) of an EoS network's domain."""
    divs = [math.log(d) for d in pp.rho_divs]
    lo = table.lnr0
    if piece > 0:
        lo = table.lnr0 + math.ceil((divs[piece - 1] - table.lnr0) / table.dlnr + 1e-9) * table.dlnr
    if piece < len(divs):
        hi = table.lnr0 + math.floor((divs[piece] - table.lnr0) / table.dlnr - 1e-9) * table.dlnr
    else:
        hi = math.log(1.15 * rho_c)
    return float(lo), float(hi), float(width)
