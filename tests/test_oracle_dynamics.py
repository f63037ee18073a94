"""Time-integration pins of the oracle: energy conservation and elastic wave speeds on the
periodic lattice (closed-form wave speeds of a linear elastic solid)."""
import math

import numpy as np
import pytest

import oracle
from sph_inputs import workloads as W


def _energy(st, m):
    v2 = st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2
    return float((m * (0.5 * v2 + st["u"])).sum())


def _run(w, dt, nsteps, every=1):
    orc = oracle.Oracle(w.params)
    st = oracle.OracleState(w.arrays)
    oracle.run_stages(orc, st)
    out = [{k: v.copy() for k, v in st.a.items()}]
    for _ in range(nsteps // every):
        oracle.step(orc, st, dt, every)
        out.append({k: v.copy() for k, v in st.a.items()})
    return out


def test_energy_conservation_second_order():
    # a long-wavelength longitudinal wave in the elastic lattice with viscosity on: the total
    # E = sum m (v^2/2 + u) is conserved up to the integrator's O(dt^2) oscillation
    errs = []
    for k in (2, 4):
        w = W.lattice()
        a = w.arrays
        a["vx"] = 2e-2 * np.sin(2 * np.pi * a["x"])
        a["vy"] = np.zeros(w.n)
        a["vz"] = np.zeros(w.n)
        m = w.params.m
        ek0 = float((m * 0.5 * (a["vx"] ** 2 + a["vy"] ** 2 + a["vz"] ** 2)).sum())
        traj = _run(w, w.dt / k, 15 * k, every=k)
        E = np.array([_energy(t, m) for t in traj])
        errs.append(np.abs(E - E[0]).max() / ek0)
    assert errs[0] < 1e-2
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.8, (errs, ratio)


def _wave(w, comp, A=1e-4):
    a = w.arrays
    n = w.n
    for c in ("vx", "vy", "vz"):
        a[c] = np.zeros(n)
    a[comp] = A * np.sin(2 * np.pi * a["x"])
    w.params = w.params.replace(visc_alpha=0.0, visc_beta=0.0)
    return w


def _lattice_wave_omega2(comp, k, dx, h, m, mu, gamma, u):
    """Linear dispersion relation of the discrete SPH equations on a cubic lattice (summation
    density, fixed h, no viscosity) from lattice sums of the Wendland C2 kernel written in its
    support-radius form.  Independent of the oracle's code:
      g1 = -sum m F d_x sin(k d_x),  g2_c = sum m W_cc (1 - cos(k d_x)),  W_cc = F + F' d_c^2 / r
      transverse:   w^2 = mu g1^2 / D^3 + 2 P g2_y / D^2
      longitudinal: w^2 = (Gamma - 2) P g1^2 / D^3 + 2 P g2_x / D^2 + (4/3) mu g1^2 / D^3
    (continuum limit: mu k^2 / D and (Gamma P + 4 mu / 3) k^2 / D)."""
    H = 2 * h
    R = int(math.ceil(H / dx)) + 1
    g = np.arange(-R, R + 1) * dx
    d = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    r = np.sqrt((d ** 2).sum(1))
    sel = r < H
    d, r = d[sel], r[sel]
    s = r / H
    Wv = 21 / (2 * math.pi * H ** 3) * (1 - s) ** 4 * (1 + 4 * s)
    F = -210 / (math.pi * H ** 5) * (1 - s) ** 3              # grad W = F x
    dF = 630 / (math.pi * H ** 6) * (1 - s) ** 2               # dF/dr
    rs = np.where(r > 0, r, 1.0)
    D = m * Wv.sum()
    P = (gamma - 1) * D * u
    g1 = -(m * F * d[:, 0] * np.sin(k * d[:, 0])).sum()
    Wxx = F + np.where(r > 0, dF * d[:, 0] ** 2 / rs, 0.0)
    Wyy = F + np.where(r > 0, dF * d[:, 1] ** 2 / rs, 0.0)
    g2x = (m * Wxx * (1 - np.cos(k * d[:, 0]))).sum()
    g2y = (m * Wyy * (1 - np.cos(k * d[:, 0]))).sum()
    if comp == "vy":
        return mu * g1 ** 2 / D ** 3 + 2 * P * g2y / D ** 2, D, P
    return (gamma - 2) * P * g1 ** 2 / D ** 3 + 2 * P * g2x / D ** 2 + 4 / 3 * mu * g1 ** 2 / D ** 3, D, P


@pytest.mark.parametrize("comp", ["vy", "vx"])
def test_elastic_wave_speed(comp):
    w = _wave(W.lattice(mu=1.0), comp)
    k = 2 * np.pi
    dx = 1 / 16
    om2, D, P = _lattice_wave_omega2(comp, k, dx, 1.3 * dx, dx ** 3, 1.0, 5 / 3, 1.5)
    om_pred = math.sqrt(om2)
    # continuum speeds: c_T = sqrt(mu/rho), c_L = sqrt((Gamma P + 4 mu/3)/rho)
    c_cont = math.sqrt(1.0 / D) if comp == "vy" else math.sqrt((5 / 3 * P + 4 / 3) / D)
    assert abs(om_pred / (k * c_cont) - 1) < 0.1
    period = 2 * np.pi / om_pred
    dt = w.dt / 4          # the leapfrog phase error (about (w dt)^2) is then below 1e-3
    nsteps = int(math.ceil(1.15 * period / dt))
    traj = _run(w, dt, nsteps)
    sx = np.sin(2 * np.pi * w.arrays["x"])
    amp = np.array([(t[comp] * sx).sum() / (sx * sx).sum() for t in traj])
    t = np.arange(len(amp)) * dt
    oms = np.linspace(0.9, 1.1, 4001) * om_pred
    res = [np.sum((amp - amp[0] * np.cos(o * t)) ** 2) for o in oms]
    om = oms[int(np.argmin(res))]
    assert abs(om / om_pred - 1) < 1e-3, (om, om_pred, k * c_cont)


def test_fluid_has_no_shear_restoring_force():
    # mu = 0: a transverse velocity profile does not reverse (no oscillation)
    w = _wave(W.lattice(mu=0.0), "vy")
    nsteps = int(math.ceil(0.5 / w.dt))
    traj = _run(w, w.dt, nsteps)
    s = np.sin(2 * np.pi * w.arrays["x"])
    amp = np.array([(t["vy"] * s).sum() / (s * s).sum() for t in traj])
    assert amp.min() > 0.99 * amp[0]
