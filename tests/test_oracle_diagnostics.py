"""Pins of the oracle's oscillation diagnostics (sections "Spherically symmetric and static neutron
star tests" and "Neutron Star Oscillations with a solid crust"): closed forms for the energies,
exact recovery of a linear v_theta field by the slab fit, and the crust-shell geometry the
paper prints (densities 4e12 to 7e12 g/cm^3 of the 1.4 Msun star, two particle layers at 1M)."""
import math

import numpy as np
import pytest

import oracle
from sph_inputs import workloads as W
from sph_inputs.params import MethodParams
from sph_inputs.tov import DENSITY_UNIT_CGS


def _state(x, y, z, vx, vy, vz, u):
    n = x.size
    return oracle.OracleState(dict(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, u=u, h=np.full(n, 0.1), S=np.zeros((6, n)),
                                   type=np.zeros(n, np.int8), broken=np.zeros(n, np.uint8)))


def test_energies_of_a_rigid_rotation():
    rng = np.random.default_rng(1)
    n = 2000
    X = rng.normal(size=(3, n))
    w = 0.7
    vx, vy, vz = -w * X[1], w * X[0], np.zeros(n)       # v = w e_z x X: purely toroidal
    u = rng.uniform(1, 2, n)
    m = 0.125
    d = oracle.diagnostics(oracle.Oracle(MethodParams(m=m)), _state(X[0], X[1], X[2], vx, vy, vz, u),
                           0.5, 1.0, 1.0, 0.1, 2.0, 0.2)
    I = m * np.sum(X[0] ** 2 + X[1] ** 2)
    assert abs(d["kinetic"] - 0.5 * I * w * w) < 1e-12 * d["kinetic"]
    assert abs(d["toroidal"] - 0.5 * I * w * w) < 1e-12 * d["kinetic"]
    assert abs(d["internal"] - m * u.sum()) < 1e-12 * d["internal"]
    # a radial field has no toroidal part
    d = oracle.diagnostics(oracle.Oracle(MethodParams(m=m)), _state(X[0], X[1], X[2], X[0], X[1], X[2], u),
                           0.5, 1.0, 1.0, 0.1, 2.0, 0.2)
    assert d["toroidal"] < 1e-25 and abs(d["kinetic"] - 0.5 * m * np.sum(X ** 2)) < 1e-12 * d["kinetic"]


def test_slab_fit_recovers_a_linear_field():
    # particles on a shell band, v = v_theta(r, theta) e_theta with v_theta linear in (r, theta):
    # the least-squares fit over the slab returns its coefficients
    rng = np.random.default_rng(2)
    n = 20000
    R0 = 6.0
    r = rng.uniform(0.3, 0.7, n) * R0
    th = np.arccos(rng.uniform(-1, 1, n))
    ph = rng.uniform(0, 2 * np.pi, n)
    x, y, z = r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)
    rs, ths = 0.5 * R0, 2 * np.pi / 3
    c0, cr, cth = 3e-3, -2e-3, 5e-4
    vth = c0 + cr * (r - rs) + cth * (th - ths)
    et = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)])
    v = et * vth
    d = oracle.diagnostics(oracle.Oracle(MethodParams()), _state(x, y, z, v[0], v[1], v[2], np.ones(n)),
                           0.4 * R0, 0.6 * R0, rs, 0.04 * R0, ths, 0.08 * np.pi)
    sel = (np.abs(r - rs) <= 0.04 * R0) & (np.abs(th - ths) <= 0.08 * np.pi)
    assert d["n_slab"] == sel.sum() > 100
    assert abs(d["slab_c0"] - c0) < 1e-12 and abs(d["slab_cr"] - cr) < 1e-11 and abs(d["slab_cth"] - cth) < 1e-11
    band = (r >= 0.4 * R0) & (r < 0.6 * R0)
    assert d["n_band"] == band.sum()


def test_slab_fit_of_the_paper_perturbation():
    # the l = 2 perturbation delta v_theta = A sin(pi r / R0) d_theta P_2(cos theta) sampled in
    # the slab: the fit's value at the slab centre is the field there to within its curvature
    # across the slab
    rng = np.random.default_rng(3)
    n = 200000
    R0, A = 6.0, 1e-2
    r = rng.uniform(0.0, 1.0, n) ** (1 / 3) * R0
    th = np.arccos(rng.uniform(-1, 1, n))
    ph = rng.uniform(0, 2 * np.pi, n)
    x, y, z = r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)
    vth = A * np.sin(np.pi * r / R0) * (-3 * np.cos(th) * np.sin(th))
    et = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)])
    v = et * vth
    d = oracle.diagnostics(oracle.Oracle(MethodParams()), _state(x, y, z, v[0], v[1], v[2], np.ones(n)),
                           0.0, R0, 0.5 * R0, 0.04 * R0, 2 * np.pi / 3, 0.08 * np.pi)
    # the same least-squares problem solved by LAPACK on the selected particles
    rs, ts = 0.5 * R0, 2 * np.pi / 3
    sel = (np.abs(r - rs) <= 0.04 * R0) & (np.abs(th - ts) <= 0.08 * np.pi)
    Amat = np.stack([np.ones(sel.sum()), r[sel] - rs, th[sel] - ts], 1)
    c, *_ = np.linalg.lstsq(Amat, vth[sel], rcond=None)
    assert abs(d["slab_c0"] - c[0]) < 1e-10 * abs(c[0])
    assert abs(d["slab_cth"] - c[2]) < 1e-8 * abs(c[2])
    # and the intercept is the field at the slab centre up to the curvature bias of the band,
    # (1/2) f'' <dtheta^2> = -4 f (0.08 pi)^2 / 6 (about 4%)
    want = A * 1.0 * (-3 * math.cos(ts) * math.sin(ts)) * (1 - 4 * (0.08 * np.pi) ** 2 / 6)
    assert abs(d["slab_c0"] - want) < 0.01 * abs(want)


def test_crust_shell_geometry_matches_the_paper():
    w = W.crust_shell(1_000_000)
    e = w.extra
    bg = W.paper_background()
    assert abs(bg.M - 1.4) < 0.005 and abs(bg.R - 9.59) < 0.01
    # the faces sit where the profile crosses 7e12 and 4e12 g/cm^3, about 0.06 km apart, near the surface
    from sph_inputs.tov import KM, areal_radius
    r_all = areal_radius(bg, bg.rbar)
    for rr, rho_cgs in ((e["r_in"], 7e12), (e["r_out"], 4e12)):
        rho = np.interp(rr, r_all, bg.rho) * DENSITY_UNIT_CGS
        assert abs(rho / rho_cgs - 1) < 1e-3, (rr, rho)
    assert 0.03 < (e["r_out"] - e["r_in"]) / KM < 0.1
    assert e["layers"] == 2 and abs(w.n / 1e6 - 1) < 0.01
    # the fundamental l = 2 toroidal frequency of a thin shell, sqrt((l-1)(l+2)) v_s / (2 pi R), is
    # about the 30 Hz the paper reports for this shell and shear modulus
    f = math.sqrt(4.0) * e["v_shear"] / (2 * math.pi * e["r_in"]) / 4.925490947e-6
    assert 25 < f < 35, f
