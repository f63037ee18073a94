"""Pins of the set-up pieces of section "Setting up Neutron Stars": the icosahedral shells, the
effective potential of the relaxation (phi_eff = -K Gamma rho^(Gamma-1) / (Gamma-1), so that
g_eff = -grad phi_eff = K Gamma rho^(Gamma-2) grad rho balances grad P / rho of P = K rho^Gamma),
the potential walls and drag, the relaxation itself and the modification step.  Closed forms and
invariants only; the oracle is never compared with itself."""
import math

import numpy as np
import pytest

import oracle
from sph_inputs import workloads as W
from sph_inputs.params import MethodParams
from sph_inputs.relax import icosahedral_star, icosphere, phi_eff_table


@pytest.mark.parametrize("f", [1, 2, 3, 7])
def test_icosphere_counts_and_spacing(f):
    P = icosphere(f)
    assert P.shape == (10 * f * f + 2, 3)
    assert np.allclose(np.linalg.norm(P, axis=1), 1.0, rtol=1e-14)
    # no duplicates, nearly uniform nearest-neighbour distances (geodesic grid)
    d = np.linalg.norm(P[:, None, :] - P[None, :, :], axis=2)
    np.fill_diagonal(d, 9.0)
    nn = d.min(1)
    assert nn.min() > 0.5 * nn.max()
    assert abs(P.sum(0)).max() < 1e-12          # symmetric about the centre


def test_icosahedral_star_follows_the_mass_profile():
    bg = W.gamma2_background()
    x, y, z, m = icosahedral_star(bg, 20000, 7, perturb=0.0)
    n = x.size
    assert abs(n / 20000 - 1) < 0.02
    assert abs(m * n - bg.mc[-1]) < 1e-12 * bg.mc[-1]
    r = np.sqrt(x * x + y * y + z * z)
    # enclosed particle count vs enclosed mass of the profile at a few radii
    for f in (0.3, 0.5, 0.7, 0.9):
        rr = f * bg.Rbar
        want = np.interp(rr, bg.rbar, bg.mc) / m
        got = np.count_nonzero(r < rr)
        assert abs(got - want) < 0.03 * want + 60, (f, got, want)


def test_effective_potential_closed_form():
    # rho(r) = rho_c (1 - r^2/R^2): g = K Gamma rho^(Gamma - 2) d rho/dr = -2 K Gamma rho_c r rho^(Gamma-2) / R^2
    R, rc, K, G = 7.0, 2e-3, 0.02, 1.01
    r = np.linspace(0.0, R, 4001)
    rho = rc * (1 - r**2 / R**2)
    g = phi_eff_table(r, rho, K, G, floor_frac=1e-9)
    inner = r < 0.9 * R
    want = -2 * K * G * rc * r * rho ** (G - 2) / R**2
    assert np.allclose(g[inner][1:], want[inner][1:], rtol=1e-5)
    # continuum equilibrium: grad P / rho of P = K rho^Gamma equals g
    P = K * rho**G
    with np.errstate(divide="ignore", invalid="ignore"):
        gp = np.gradient(P, r) / rho
    assert np.allclose(g[inner][1:], gp[inner][1:], rtol=1e-5)


def _isolated(pos, vel):
    n = len(pos)
    pos = np.asarray(pos, float)
    vel = np.asarray(vel, float)
    return dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(), vx=vel[:, 0].copy(),
                vy=vel[:, 1].copy(), vz=vel[:, 2].copy(), u=np.full(n, 1.0), h=np.full(n, 0.1),
                S=np.zeros((6, n)), type=np.zeros(n, np.int8), broken=np.zeros(n, np.uint8))


def test_external_acceleration_walls_and_drag():
    # particles far apart feel only the external terms: a table linear in r is interpolated
    # exactly, g(r) = a + b r along n; walls add wall_k (wall_in - r) inside, -wall_k (r - wall_out)
    # outside; the drag is -damping v; beyond the table g = 0
    a0, b0, dr, nt = 0.3, -0.05, 0.01, 801           # table on [0, 8]
    tab = a0 + b0 * dr * np.arange(nt)
    rng = np.random.default_rng(2)
    radii = np.array([0.5, 1.5, 3.3, 5.0, 7.9, 9.0])
    dirs = rng.normal(size=(radii.size, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pos = dirs * radii[:, None] + np.arange(radii.size)[:, None] * 0.0
    vel = rng.normal(size=(radii.size, 3))
    # keep them apart: radii differ by more than 2 (h_a + h_b) = 0.4 unless directions separate them
    p = MethodParams(m=1e-6, kernel="WC2", eos="GAMMA_LAW", gamma=5 / 3, ext_table=tab, ext_dr=dr,
                     wall_in=1.0, wall_out=7.0, wall_k=2.0, damping=0.25)
    st = oracle.OracleState(_isolated(pos, vel))
    k = oracle.run_stages(oracle.Oracle(p), st)
    assert k["offsets"][-1] == 0                      # no neighbours
    for i, r in enumerate(radii):
        g = a0 + b0 * r if r <= (nt - 1) * dr else 0.0
        if r < 1.0:
            g += 2.0 * (1.0 - r)
        if r > 7.0:
            g -= 2.0 * (r - 7.0)
        want = g * dirs[i] - 0.25 * vel[i]
        got = np.array([st["ax"][i], st["ay"][i], st["az"][i]])
        assert np.allclose(got, want, rtol=1e-13, atol=1e-15), (r, got, want)


def test_relaxation_reduces_density_noise():
    # perturbed icosahedral shells relaxed in the effective potential of the target profile:
    # the density's deviation from the target falls (the Gamma = 1.01 law, walls, drag)
    w = W.relax_star(3000, kernel="WC2", eta=1.3)
    bg = w.bg
    orc = oracle.Oracle(w.params)
    st = oracle.OracleState(w.arrays)

    def dev():
        r = np.sqrt(st["x"] ** 2 + st["y"] ** 2 + st["z"] ** 2)
        D0 = np.interp(r, bg.rbar, bg.D0)
        inner = r < 0.8 * bg.Rbar
        return float(np.sqrt(np.mean((st["D"][inner] / D0[inner] - 1) ** 2)))

    oracle.run_stages(orc, st)
    d0 = dev()
    oracle.step(orc, st, w.dt, 150)
    d1 = dev()
    print("density deviation from the target: before", d0, "after", d1)
    assert d0 > 0.06 and d1 < 0.5 * d0
    r = np.sqrt(st["x"] ** 2 + st["y"] ** 2 + st["z"] ** 2)
    assert r.max() < bg.Rbar * 1.05                    # the wall holds the surface


def test_modification_step_reproduces_a_linear_profile():
    rng = np.random.default_rng(5)
    n = 500
    pos = rng.normal(size=(n, 3)) * 2.0
    vel = rng.normal(size=(n, 3))
    dr, nt = 0.02, 301                                 # table on [0, 6]
    tab = 1.5 - 0.2 * dr * np.arange(nt)
    st = oracle.OracleState(_isolated(pos, vel))
    oracle.modify_energy(oracle.Oracle(MethodParams()), st, tab, dr)
    r = np.linalg.norm(pos, axis=1)
    want = np.where(r <= (nt - 1) * dr, 1.5 - 0.2 * r, tab[-1])
    assert np.allclose(st["u"], want, rtol=1e-13)
    assert np.all(st["vx"] == 0) and np.all(st["vy"] == 0) and np.all(st["vz"] == 0)
