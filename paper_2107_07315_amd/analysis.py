"""Post-processing of the diagnostic time series that sph_diagnostics records on the device.

The paper reads oscillation frequencies off time series: the internal energy for radial modes and
v_theta in a slab for non-radial modes (section "Spherically symmetric and static neutron star
tests", shown with their frequency spectra), and the crust shell's kinetic energy (section
"Neutron Star Oscillations with a solid crust"), whose frequency is then corrected for the
gravitational redshift, f_obs = f_cal sqrt(1 - r_S / R) with r_S = 2 G M / c^2.  These are
host-side transforms of a few thousand samples, not part of the particle loop.
"""
from __future__ import annotations

import math

import numpy as np

# one geometric time unit (G = c = Msun = 1) in seconds: G Msun / c^3
TIME_UNIT_S = 6.67430e-8 * 1.98847e33 / 2.99792458e10 ** 3


def spectrum(t, y):
    """Amplitude spectrum of a uniformly sampled series (mean removed, Hann window):
    (frequencies in 1 / time unit of t, amplitudes)."""
    t = np.asarray(t, np.float64)
    y = np.asarray(y, np.float64)
    if t.size < 4:
        raise ValueError("need at least 4 samples")
    dt = (t[-1] - t[0]) / (t.size - 1)
    w = np.hanning(t.size)
    a = np.abs(np.fft.rfft((y - y.mean()) * w)) * 2.0 / w.sum()
    f = np.fft.rfftfreq(t.size, dt)
    return f, a


def peak_frequency(t, y, fmin=0.0):
    """Frequency of the largest spectral peak above fmin, refined by a parabola through the three
    bins around it (in 1 / time unit of t)."""
    f, a = spectrum(t, y)
    sel = np.flatnonzero(f > fmin)
    k = int(sel[np.argmax(a[sel])])
    if 0 < k < a.size - 1:
        l, c, r = np.log(a[k - 1] + 1e-300), np.log(a[k] + 1e-300), np.log(a[k + 1] + 1e-300)
        den = l - 2 * c + r
        shift = 0.5 * (l - r) / den if den != 0 else 0.0
        return float(f[k] + shift * (f[1] - f[0]))
    return float(f[k])


def zero_crossing_frequency(t, y):
    """Frequency of an oscillation about zero from the spacing of its zero crossings (linear
    interpolation between samples; half a period between consecutive crossings), for series too
    short for a resolved spectrum; nan with fewer than two crossings."""
    t = np.asarray(t, np.float64)
    y = np.asarray(y, np.float64)
    k = np.flatnonzero(np.sign(y[:-1]) * np.sign(y[1:]) < 0)
    if k.size < 2:
        return float("nan")
    tc = t[k] - y[k] * (t[k + 1] - t[k]) / (y[k + 1] - y[k])
    return float(0.5 / np.mean(np.diff(tc)))


def redshifted(f_cal, M, R):
    """Observed frequency f_cal sqrt(1 - 2M/R) (geometric units, M and R in the same units)."""
    return f_cal * math.sqrt(1.0 - 2.0 * M / R)
