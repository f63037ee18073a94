"""Method configuration shared by the GPU binding and the test oracle binding.

Plain values only: each binding converts this into its own C struct.  Defaults are the
readings of the paper used throughout (see the design notes for the reasons):
Wendland kernels with support h_a + h_b, Monaghan viscosity alpha=1, beta=2, eps=0.01,
objective (Jaumann) rotation sign, the paper's von Mises factor min(Y0^2/sigma_v^2, 1).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

KERNELS = {"WC2": 0, "WC4": 1}
H_MODES = {"FIXED": 0, "ADAPTIVE": 1}
BACKGROUNDS = {"NEWTONIAN": 0, "TOV": 1}
EOS_KINDS = {"GAMMA_LAW": 0, "TABLE": 1, "MLP": 2}
MU_MODES = {"CONST": 0, "P_FACTOR": 1}
YIELD_MODES = {"PAPER": 0, "RADIAL": 1}
Y0_MODES = {"CONST": 0, "E_FACTOR": 1}
BREAK_MODES = {"OFF": 0, "ONSET": 1, "FLUIDIZE": 2}
ROTATIONS = {"OBJECTIVE": 0, "LITERAL": 1}
PRECISIONS = {"FP64": 0, "FP32": 1}
DENSITY_MODES = {"SUMMATION": 0, "CONTINUITY": 1}
ENERGY_MODES = {"PAPER": 0, "FIRST_LAW": 1}
DTP_MODES = {"OFF": 0, "LAGGED": 1}


@dataclasses.dataclass
class EosTable:
    """ln P and ln c_s^2 on a uniform (ln rho, ln u) grid, index [i_rho * nu + i_u]; NaN marks
    states outside the equation of state's domain."""
    lnP: np.ndarray
    lncs2: np.ndarray
    lnr0: float
    dlnr: float
    lnu0: float
    dlnu: float

    @property
    def nr(self):
        return self.lnP.shape[0]

    @property
    def nu(self):
        return self.lnP.shape[1]


@dataclasses.dataclass
class MethodParams:
    m: float = 1.0
    kernel: str = "WC2"
    h_mode: str = "FIXED"
    eta: float = 1.3
    background: str = "NEWTONIAN"
    bg_table: Optional[np.ndarray] = None     # (4, n): alpha, alpha', psi, psi' on rbar_i = i*bg_dr
    bg_dr: float = 0.0
    bg_M: float = 0.0
    periodic: bool = False
    box: float = 0.0
    visc_alpha: float = 1.0
    visc_beta: float = 2.0
    visc_eps: float = 0.01
    eos: str = "GAMMA_LAW"
    gamma: float = 5.0 / 3.0
    table: Optional[EosTable] = None
    mu_mode: str = "CONST"
    mu_const: float = 0.0
    mu_pfactor: float = 0.0
    yield_mode: str = "PAPER"
    y0_mode: str = "CONST"
    y0_const: float = 1e300
    y0_over_E: float = 0.0
    break_mode: str = "OFF"
    eps_break: float = 0.1
    rotation: str = "OBJECTIVE"
    precision: str = "FP64"
    # external radial acceleration table g(r_i), r_i = i * ext_dr (None: no external potential),
    # harmonic walls (radius 0: none) and a velocity drag, for relaxation and the crust shell
    ext_table: Optional[np.ndarray] = None
    ext_dr: float = 0.0
    wall_in: float = 0.0
    wall_out: float = 0.0
    wall_k: float = 0.0
    damping: float = 0.0
    density_mode: str = "SUMMATION"
    energy_mode: str = "PAPER"
    dtP_mode: str = "OFF"
    cfl: float = 0.3

    def replace(self, **kw) -> "MethodParams":
        return dataclasses.replace(self, **kw)
