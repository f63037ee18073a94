"""CPU checks of the host post-processing of diagnostic time series."""
import math

import numpy as np

from paper_2107_07315_amd import analysis


def test_peak_frequency_of_a_sampled_sinusoid():
    t = np.arange(4096) * 0.37
    for f0 in (0.0123, 0.05, 0.2):
        y = 3.0 + 0.01 * np.sin(2 * np.pi * f0 * t + 0.3) + 0.002 * np.sin(2 * np.pi * 3.1 * f0 * t)
        f = analysis.peak_frequency(t, y)
        assert abs(f / f0 - 1) < 0.01, (f, f0)


def test_zero_crossing_frequency_of_a_short_series():
    t = np.linspace(0.0, 1.6, 81)
    for f0 in (1.5, 2.2):
        y = 0.7 * np.cos(2 * np.pi * f0 * t) * np.exp(-0.2 * t)
        assert abs(analysis.zero_crossing_frequency(t, y) / f0 - 1) < 0.01
    assert np.isnan(analysis.zero_crossing_frequency(t, np.exp(-t)))


def test_redshift_of_the_paper_crust_frequency():
    # 30 Hz computed for a 1.4 Msun star of R = 14.2 km is observed at about 25.18 Hz
    km = 1.0e5 / (6.67430e-8 * 1.98847e33 / 2.99792458e10 ** 2)
    assert abs(analysis.redshifted(30.0, 1.4, 14.2 * km) - 25.18) < 0.1
    assert abs(analysis.TIME_UNIT_S - 4.9255e-6) < 1e-9
