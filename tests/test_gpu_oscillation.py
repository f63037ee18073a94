"""GPU checks of the oscillation analyses (sections "Spherically symmetric and static neutron star
tests", "Neutron stars with a solid crust in SPH" and "Neutron Star Oscillations with a solid
crust"): the device diagnostics against the oracle's on the same state, the radial mode of a star
with a solid and a fluid crust, and the crust shell's toroidal oscillation (solid) against its
decay-free drift (fluid)."""
import math

import numpy as np
import pytest

import oracle
from paper_2107_07315_amd import analysis
from sph_inputs import workloads as W

pytestmark = pytest.mark.gpu


def _slab(R0):
    # the paper's slab: r = (0.5 +- 0.04) R0, theta = 2 pi / 3 +- 0.08 pi; radial band: the outer half
    return dict(r_lo=0.5 * R0, r_hi=0.9 * R0, slab_r=0.5 * R0, slab_dr=0.04 * R0, slab_th=2 * np.pi / 3,
                slab_dth=0.08 * np.pi)


def test_diagnostics_match_oracle():
    from paper_2107_07315_amd import sph
    w = W.star(20000, seed=3, kernel="WC4", eta=W.ETA_100, l=2, A=1e-2)
    ctx = sph.Context(w.params, capacity=w.n)
    st = sph.DeviceState(w.arrays)
    ctx.evaluate(st)
    ctx.sph_step(st, w.dt, 3)
    dp = _slab(w.bg.Rbar)
    d = ctx.sph_diagnostics(st, **dp)
    a = st.numpy()
    ctx.close()
    ost = oracle.OracleState(a)
    o = oracle.diagnostics(oracle.Oracle(w.params), ost, dp["r_lo"], dp["r_hi"], dp["slab_r"], dp["slab_dr"],
                           dp["slab_th"], dp["slab_dth"])
    print("gpu", d, "\noracle", o, flush=True)
    assert d["n_band"] == o["n_band"] and d["n_slab"] == o["n_slab"] > 20
    for k in ("kinetic", "toroidal", "internal", "u_band", "slab_c0", "slab_cr", "slab_cth"):
        assert abs(d[k] - o[k]) <= 1e-12 * max(abs(o[k]), 1e-300), (k, d[k], o[k])


def _radial_trace(w, chunks=60, every=5):
    from paper_2107_07315_amd import sph
    ctx = sph.Context(w.params, capacity=w.n)
    st = sph.DeviceState(w.arrays)
    ctx.evaluate(st)
    dp = _slab(w.bg.Rbar)
    t, ub = [0.0], [ctx.sph_diagnostics(st, **dp)["u_band"]]
    for k in range(chunks):
        ctx.sph_step(st, w.dt, every)
        t.append((k + 1) * every * w.dt)
        ub.append(ctx.sph_diagnostics(st, **dp)["u_band"])
    ctx.close()
    return np.array(t), np.array(ub)


def test_radial_mode_with_solid_and_fluid_crust():
    # a radial (l = 0) perturbation of the star with a solid crust (mu = 0.01 P) and with the same
    # crust fluid: the u traces agree to a small part of their oscillation, as the paper finds
    ws = W.star(20000, seed=2, l=0, A=1e-3)
    wf = W.star(20000, seed=2, l=0, A=1e-3, mu_factor=0.0)
    t, us = _radial_trace(ws)
    _, uf = _radial_trace(wf)
    amp = np.ptp(us)
    diff = np.max(np.abs(us - uf))
    fs, ff = analysis.peak_frequency(t, us), analysis.peak_frequency(t, uf)
    print(f"u-band oscillation {amp:.3e}, solid - fluid {diff:.3e}; peak frequency solid {fs:.4g} fluid {ff:.4g} "
          f"(1/time unit)", flush=True)
    assert amp > 0 and diff < 0.1 * amp
    assert abs(fs / ff - 1) < 0.02


def _shell_run(solid, n=100_000, settle=600, periods=0.6, amp=1e-2):
    """Settle the shell radially against its walls with a drag, impose the l = 2 toroidal field,
    and record the mode amplitude (the projection of v_phi on 3 sin(theta) cos(theta)) over
    `periods` of the thin-shell estimate 2 pi R / (2 v_s)."""
    from paper_2107_07315_amd import sph
    w = W.crust_shell(n, solid=solid, amp=amp)
    e = w.extra
    # drag: a few wall periods, and damping dt below 1 (the kicks treat the drag explicitly)
    ctx = sph.Context(w.params.replace(damping=min(2.0 * math.sqrt(w.params.wall_k), 0.3 / w.dt)), capacity=w.n)
    st = sph.DeviceState(w.arrays)
    ctx.evaluate(st)
    ctx.sph_step(st, w.dt, settle)
    ctx.sph_sync()
    a = st.numpy()
    ctx.close()
    vt = e["v_tor"][:, a["id"]]
    a["vx"], a["vy"], a["vz"] = vt[0].copy(), vt[1].copy(), vt[2].copy()
    ctx = sph.Context(w.params, capacity=w.n)
    st = sph.DeviceState(a)
    ctx.evaluate(st)
    om = 2.0 * e["v_shear"] / e["r_in"]       # l = 2: sqrt((l-1)(l+2)) v_s / R
    period = 2 * math.pi / om
    per_chunk = max(1, int(period / 80 / w.dt))
    dp = dict(r_lo=0.0, r_hi=1e9, slab_r=0.0, slab_dr=0.0, slab_th=0.0, slab_dth=0.0)
    t, c = [0.0], [ctx.sph_diagnostics(st, **dp)["tor_l2"]]
    while t[-1] < periods * period:
        ctx.sph_step(st, w.dt, per_chunk)
        t.append(t[-1] + per_chunk * w.dt)
        c.append(ctx.sph_diagnostics(st, **dp)["tor_l2"])
    ctx.sph_sync()
    ctx.close()
    return np.array(t), np.array(c) / c[0], period


def test_crust_shell_toroidal_oscillation():
    # the paper's shell (1M particles, two layers between 7e12 and 4e12 g/cm^3, mu = 1e29 erg/cm^3):
    # the l = 2 toroidal mode of the solid shell swings through zero within the thin-shell period;
    # the same shell with a fluid crust is run beside it and reported
    ts, cs, T = _shell_run(True, n=1_000_000, settle=400, periods=1.0)
    tf, cf, _ = _shell_run(False, n=1_000_000, settle=400, periods=1.0)
    fs = analysis.zero_crossing_frequency(ts, cs) / analysis.TIME_UNIT_S
    print(f"shell mode amplitude, solid: {np.round(cs[::8], 3).tolist()}", flush=True)
    print(f"shell mode amplitude, fluid: {np.round(cf[::8], 3).tolist()}", flush=True)
    print(f"thin-shell estimate {1.0 / (T * analysis.TIME_UNIT_S):.1f} Hz; solid shell {fs:.1f} Hz "
          f"(observed {analysis.redshifted(fs, W.paper_background().M, W.paper_background().R):.1f} Hz)", flush=True)
    assert cs.min() < -0.3            # the solid shell swings back through zero ...
    assert 0.5 < fs * T * analysis.TIME_UNIT_S < 2.5   # ... near the thin-shell frequency
    assert cf.min() > 0.0 and cf[-1] < 0.8   # the fluid shell has no restoring force: its mode decays


def test_crust_shell_steps_match_oracle():
    # the shell's path (external potential, both walls, constant shear modulus, a single layer)
    # against the oracle: one evaluation to 1e-12 and five steps to 1e-12 of each field's scale
    from parity import eval_errors, gpu_run, oracle_run, step_errors
    w = W.crust_shell(20000, amp=1e-2)
    vt = w.extra["v_tor"]
    w.arrays["vx"], w.arrays["vy"], w.arrays["vz"] = vt[0].copy(), vt[1].copy(), vt[2].copy()
    g = gpu_run(w, lists=False)
    o = oracle_run(w)
    e = eval_errors(g, o)
    print("shell eval", e, flush=True)
    for k, v in e.items():
        assert v <= 1e-12, (k, v)
    g = gpu_run(w, steps=5)
    o5 = oracle_run(w, steps=5)
    e = step_errors(g, o5, ("x", "y", "z", "vx", "vy", "vz", "u", "S", "D", "ax", "dudt", "dSdt"), w.dt, 5)
    print("shell 5 steps", e, flush=True)
    for k, v in e.items():
        assert v < 1e-12, (k, v)
    # FP32 pair sums: every tile of the shell holds stressed particles, so the force pass stages
    # the neighbours' S/D^2 in LDS; evaluation and five steps to 1e-4 in density, pressure, stress
    from parity import field_errors
    g = gpu_run(w, precision="FP32", lists=False)
    e = eval_errors(g, o)
    print("shell FP32 eval", e, flush=True)
    for k in ("D", "rho", "P", "ax", "ay", "az", "dudt", "dSdt"):
        assert e[k] < 1e-4, (k, e[k])
    g = gpu_run(w, steps=5, precision="FP32")
    e = field_errors(g, o5, ("x", "vx", "u", "S", "D", "rho", "P"))
    print("shell FP32 5 steps", e, flush=True)
    for k in ("D", "rho", "P", "S"):
        assert e[k] < 1e-4, (k, e[k])
