"""Pins of the oracle's solid-model updates and per-particle closures against closed forms.

Each test fixes a quantity by arithmetic written out here from the paper's definitions, never by
calling the oracle twice:
  * maximum-strain breaking (section "Solid SPH Equations", damage model): eps = sigma_max / E with
    Young's modulus E = 9 B mu / (3 B + mu), the flag set once eps reaches the breaking strain and
    kept; the two post-break readings ONSET (flag only) and FLUIDIZE (stress and modulus dropped);
  * the yield stress tied to E (Y0 = y0_over_E E, the strain form of the yield criterion);
  * the adaptive smoothing length h = eta (m / D)^(1/3);
  * the Lorentz factor of the computational density D = rho psi^6 W_L ("Fixed metric
    background", the conserved density) for a moving particle.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from sph_inputs.lattice import cubic_lattice
from sph_inputs.params import MethodParams
from sph_inputs import workloads as W
from sph_inputs.tov import exterior_metric

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    return json.load(open(os.path.join(GOLD, name)))


def _wc2_self(h):
    """Wendland C2 with support 2h at r = 0: 21 / (16 pi h^3)."""
    return 21.0 / (16.0 * math.pi * h**3)


def _isolated(S_list, typ, u=1.2, h=0.5, vel=None):
    """Particles 10 support radii apart (no neighbours), each with its own deviatoric stress."""
    n = len(S_list)
    S = np.array(S_list, np.float64).T.copy()          # (6, n)
    vx = np.zeros(n) if vel is None else np.asarray(vel[0], float)
    vy = np.zeros(n) if vel is None else np.asarray(vel[1], float)
    vz = np.zeros(n) if vel is None else np.asarray(vel[2], float)
    return dict(x=10.0 * np.arange(n, dtype=np.float64), y=np.zeros(n), z=np.zeros(n), vx=vx, vy=vy, vz=vz,
                u=np.full(n, u), h=np.full(n, h), S=S, type=np.asarray(typ, np.int8),
                broken=np.zeros(n, np.uint8))


def _rotated(s, rng):
    """Q diag(2s, -s, -s) Q^T for a random rotation Q: traceless, largest eigenvalue exactly 2s."""
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    A = q @ np.diag([2 * s, -s, -s]) @ q.T
    return [A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[0, 2], A[1, 2]]


GAMMA, U0, H0, MU = 2.0, 1.2, 0.5, 0.7


def _closed_form_E(m):
    """Young's modulus of an isolated Gamma-law particle with constant shear modulus: D = m W(0),
    rho = D (Newtonian), P = (Gamma - 1) rho u, bulk modulus B = Gamma P, E = 9 B mu / (3 B + mu)."""
    rho = m * _wc2_self(H0)
    P = (GAMMA - 1.0) * rho * U0
    B = GAMMA * P
    return 9.0 * B * MU / (3.0 * B + MU), B, P


def _solid_params(m, mode, eps_b, **kw):
    return MethodParams(m=m, kernel="WC2", background="NEWTONIAN", eos="GAMMA_LAW", gamma=GAMMA,
                        mu_mode="CONST", mu_const=MU, y0_mode="CONST", y0_const=1e300, break_mode=mode,
                        eps_break=eps_b, **kw)


@pytest.mark.parametrize("mode", ["ONSET", "FLUIDIZE"])
def test_breaking_threshold_from_closed_form_modulus(mode):
    # isolated particles have no strain rate, so S is constant over a step; the breaking test at
    # the end of the step compares lambda_max(S) / E with eps_b.  Stresses are placed 1e-9
    # (relative) below and above the threshold; a wrong E (e.g. 9 B mu / (3 B + 2 mu), or B
    # without Gamma) moves the threshold by far more than that
    m = 1.0
    E, B, P = _closed_form_E(m)
    eps_b = 0.05
    rng = np.random.default_rng(21)
    s_at = eps_b * E / 2.0            # lambda_max = 2 s
    S = [_rotated(s_at * (1 - 1e-9), rng), _rotated(s_at * (1 + 1e-9), rng),
         _rotated(3 * s_at, rng), _rotated(3 * s_at, rng), _rotated(-4 * s_at, rng)]
    # particle 3 is fluid (type 0), which never breaks whatever its stress; particle 4 holds
    # Q diag(-8, 4, 4) s_at Q^T, whose largest eigenvalue 4 s_at lies above the threshold
    typ = [1, 1, 1, 0, 1]
    p = _solid_params(m, mode, eps_b)
    orc = oracle.Oracle(p)
    st = oracle.OracleState(_isolated(S, typ, U0, H0))
    oracle.run_stages(orc, st)
    assert np.allclose(st["B"][[0, 1, 2, 4]], B, rtol=1e-14)
    S_before = st["S"].copy()
    oracle.step(orc, st, 1e-3, 1)
    assert st["broken"].tolist() == [0, 1, 1, 0, 1]
    if mode == "ONSET":
        # the flag only: the stress of a broken particle is left as it was
        assert np.array_equal(st["S"][:, [0, 1, 2, 4]], S_before[:, [0, 1, 2, 4]])
    else:
        # FLUIDIZE: the stress of a broken particle is dropped at once ...
        assert np.all(st["S"][:, [1, 2, 4]] == 0.0)
        assert np.array_equal(st["S"][:, 0], S_before[:, 0])
        # ... and from the next evaluation on it has no shear modulus, stress rate or yield stress
        oracle.run_stages(orc, st)
        assert np.all(st["mu"][[1, 2, 4]] == 0.0) and st["mu"][0] == MU
        assert np.all(st["dSdt"][:, [1, 2, 4]] == 0.0)
    # sticky: a broken particle stays broken when its stress falls back below the threshold
    st["S"][:, 1] *= 1e-3
    oracle.run_stages(orc, st)
    oracle.step(orc, st, 1e-3, 2)
    assert st["broken"].tolist() == [0, 1, 1, 0, 1]


def test_breaking_fires_at_equality():
    # the criterion is eps >= eps_b: with eps_b equal to lambda_max / E as the oracle rounds it
    # (E from the oracle's own B and mu by the same operations) the particle breaks; one ulp
    # above, it does not.  lambda_max of diag(2, -1, -1) s with s a power of two is exactly 2 s
    # in the closed-form eigenvalue (p = s, det = 2, phi = 0).
    m = 1.0
    s = 2.0 ** -6
    for bump, want in ((0, 1), (1, 0)):
        p = _solid_params(m, "ONSET", 0.1)
        orc = oracle.Oracle(p)
        st = oracle.OracleState(_isolated([[2 * s, -s, -s, 0, 0, 0]], [1], U0, H0))
        oracle.run_stages(orc, st)
        B, mu = st["B"][0], st["mu"][0]
        E = 9.0 * B * mu / (3.0 * B + mu)
        eps = (2 * s) / E
        if bump:
            eps = np.nextafter(eps, np.inf)
        orc = oracle.Oracle(p.replace(eps_break=float(eps)))
        oracle.step(orc, st, 1e-3, 1)
        assert st["broken"][0] == want, (bump, eps)


def test_breaking_off_and_zero_modulus_never_break():
    m = 1.0
    E, _, _ = _closed_form_E(m)
    rng = np.random.default_rng(5)
    S = [_rotated(10 * E, rng)]
    for mode, mu in (("OFF", MU), ("ONSET", 0.0)):
        p = _solid_params(m, mode, 1e-6).replace(mu_const=mu)
        orc = oracle.Oracle(p)
        st = oracle.OracleState(_isolated(S, [1], U0, H0))
        oracle.run_stages(orc, st)
        oracle.step(orc, st, 1e-3, 2)
        assert st["broken"][0] == 0, mode


@pytest.mark.parametrize("mu_mode", ["CONST", "P_FACTOR"])
def test_yield_stress_from_youngs_modulus_on_lattice(mu_mode):
    # Y0 = y0_over_E E on the Gamma-law lattice: D from the closed-form lattice sum, rho = D,
    # P = (Gamma - 1) rho u, B = Gamma P, mu constant or f P, E = 9 B mu / (3 B + mu)
    g = gold("lattice_density.json")
    x, y, z, dx = cubic_lattice(16)
    n = x.size
    gamma, u0, f, y0e = 5.0 / 3.0, 1.5, 0.37, 0.2
    arr = dict(x=x, y=y, z=z, vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n), u=np.full(n, u0),
               h=np.full(n, 1.3 * dx), S=np.zeros((6, n)), type=np.ones(n, np.int8), broken=np.zeros(n, np.uint8))
    p = MethodParams(m=dx**3, kernel="WC2", periodic=True, box=1.0, eos="GAMMA_LAW", gamma=gamma,
                     mu_mode=mu_mode, mu_const=0.9, mu_pfactor=f, y0_mode="E_FACTOR", y0_over_E=y0e)
    st = oracle.OracleState(arr)
    oracle.run_stages(oracle.Oracle(p), st)
    D = g["WC2_eta1.3"]["D"]
    P = (gamma - 1.0) * D * u0
    B = gamma * P
    mu = 0.9 if mu_mode == "CONST" else f * P
    E = 9.0 * B * mu / (3.0 * B + mu)
    assert np.allclose(st["mu"], mu, rtol=1e-13)
    assert np.allclose(st["Y0"], y0e * E, rtol=1e-13)
    # a fluid particle has no modulus and so no yield stress in this mode
    arr["type"] = np.zeros(n, np.int8)
    st = oracle.OracleState(arr)
    oracle.run_stages(oracle.Oracle(p), st)
    assert np.all(st["Y0"] == 0.0) and np.all(st["mu"] == 0.0)


@pytest.mark.parametrize("kernel,key", [("WC2", "WC2_eta1.3"), ("WC4", "WC4_eta1.3")])
def test_adaptive_smoothing_length_after_one_step_at_rest(kernel, key):
    # a periodic lattice at rest under uniform pressure stays put; one step with the adaptive
    # smoothing length sets h = eta (m / D)^(1/3) with D the lattice density of the old h
    g = gold("lattice_density.json")
    x, y, z, dx = cubic_lattice(16)
    n = x.size
    eta = 1.3
    arr = dict(x=x, y=y, z=z, vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n), u=np.full(n, 1.5),
               h=np.full(n, eta * dx), S=np.zeros((6, n)), type=np.zeros(n, np.int8), broken=np.zeros(n, np.uint8))
    p = MethodParams(m=dx**3, kernel=kernel, h_mode="ADAPTIVE", eta=eta, periodic=True, box=1.0,
                     eos="GAMMA_LAW", gamma=5 / 3)
    orc = oracle.Oracle(p)
    st = oracle.OracleState(arr)
    oracle.run_stages(orc, st)
    oracle.step(orc, st, 1e-3, 1)
    want = eta * (dx**3 / g[key]["D"]) ** (1.0 / 3.0)
    assert np.max(np.abs(st["h"] - want)) <= 1e-13 * want
    # fixed mode leaves h alone
    st = oracle.OracleState(arr)
    orc = oracle.Oracle(p.replace(h_mode="FIXED"))
    oracle.run_stages(orc, st)
    oracle.step(orc, st, 1e-3, 1)
    assert np.all(st["h"] == eta * dx)


def test_rest_mass_density_of_a_moving_particle():
    # outside the star the background is exterior Schwarzschild in isotropic radius (closed form);
    # an isolated particle with coordinate velocity v has rho = D / (psi^6 W_L) with the Lorentz
    # factor W_L = (1 - psi^4 |v|^2 / alpha^2)^(-1/2) of the normal-observer velocity v / alpha
    bg = W.gamma2_background()
    rng = np.random.default_rng(9)
    h = 0.4
    for k in range(6):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        rb = bg.Rbar * rng.uniform(1.3, 3.0)
        x = d * rb
        a, _, psi, _ = (float(v[0]) for v in exterior_metric(np.array([rb]), bg.M))
        vmax = a / psi**2                       # light speed in coordinate units
        v = rng.normal(size=3)
        v *= rng.uniform(0.1, 0.8) * vmax / np.linalg.norm(v)
        D = 3e-3
        m = D / _wc2_self(h)
        arr = dict(x=np.array([x[0]]), y=np.array([x[1]]), z=np.array([x[2]]), vx=np.array([v[0]]),
                   vy=np.array([v[1]]), vz=np.array([v[2]]), u=np.array([0.05]), h=np.array([h]),
                   S=np.zeros((6, 1)), type=np.zeros(1, np.int8), broken=np.zeros(1, np.uint8))
        p = MethodParams(m=m, kernel="WC2", background="TOV", bg_table=bg.table, bg_dr=bg.drbar, bg_M=bg.M,
                         eos="GAMMA_LAW", gamma=2.0)
        st = oracle.OracleState(arr)
        oracle.run_stages(oracle.Oracle(p), st)
        WL = 1.0 / math.sqrt(1.0 - psi**4 * float(v @ v) / a**2)
        assert WL > 1.004
        rho = D / (psi**6 * WL)
        assert abs(st["D"][0] / D - 1) < 1e-14
        assert abs(st["rho"][0] / rho - 1) < 1e-13, (k, st["rho"][0], rho)
        P = (2.0 - 1.0) * rho * 0.05
        assert abs(st["P"][0] / P - 1) < 1e-13


def test_fluidized_particle_keeps_no_stress_in_later_steps():
    # with neighbours a broken particle still has a strain rate; FLUIDIZE means no deviatoric
    # stress from the break on: S stays exactly 0 in every later step (its predictor included,
    # seen by the evaluation: zero stress rate and zero stress work), while unbroken neighbours
    # keep theirs
    from sph_inputs.lattice import random_box
    n = 400
    rng = np.random.default_rng(3)
    x, y, z = random_box(n, 1.0, 3)
    S = rng.normal(scale=0.3, size=(6, n))
    S[:3] -= S[:3].mean(0)
    arr = dict(x=x, y=y, z=z, vx=rng.normal(scale=0.2, size=n), vy=rng.normal(scale=0.2, size=n),
               vz=rng.normal(scale=0.2, size=n), u=rng.uniform(0.5, 2.0, n), h=0.09 * rng.uniform(0.7, 1.4, n),
               S=S, type=np.ones(n, np.int8), broken=np.zeros(n, np.uint8))
    p = MethodParams(m=1.0 / n, kernel="WC2", eos="GAMMA_LAW", gamma=5 / 3, mu_mode="CONST", mu_const=0.8,
                     break_mode="FLUIDIZE", eps_break=0.2)
    orc = oracle.Oracle(p)
    st = oracle.OracleState(arr)
    oracle.run_stages(orc, st)
    oracle.step(orc, st, 2e-4, 1)
    b = st["broken"] == 1
    assert 10 < b.sum() < n - 10
    for _ in range(3):
        before = b
        oracle.step(orc, st, 2e-4, 1)
        b = st["broken"] == 1
        assert np.all(st["S"][:, b] == 0.0) and np.all(st["dSdt"][:, b] == 0.0)
        # particles broken before this step were fluid in its evaluation: no stress work there
        assert np.all(st["sdot"][before] == 0.0)
        assert np.all(np.any(st["S"][:, ~b] != 0.0, axis=0))
