"""ctypes binding of the CPU FP64 oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's
CPU-baseline leg.  The GPU package never imports this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

ORC_OK = 0
STATUS_NAMES = {0: "OK", 1: "E_ARG", 3: "E_OOM", 5: "E_NGB_CAPACITY", 6: "E_NONFINITE",
                7: "E_EOS_DOMAIN"}
BRUTE, GRID = 0, 1


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-Wextra", "-o", LIB_PATH, os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB_PATH


_dp = ctypes.POINTER(ctypes.c_double)


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_int32), ("h_mode", ctypes.c_int32), ("background", ctypes.c_int32),
        ("periodic", ctypes.c_int32), ("eta", ctypes.c_double), ("box", ctypes.c_double),
        ("m", ctypes.c_double),
        ("bg", _dp), ("bg_n", ctypes.c_int32), ("bg_dr", ctypes.c_double), ("bg_M", ctypes.c_double),
        ("visc_alpha", ctypes.c_double), ("visc_beta", ctypes.c_double), ("visc_eps", ctypes.c_double),
        ("eos", ctypes.c_int32), ("gamma", ctypes.c_double),
        ("tab_lnP", _dp), ("tab_lncs2", _dp), ("tab_nr", ctypes.c_int32), ("tab_nu", ctypes.c_int32),
        ("tab_lnr0", ctypes.c_double), ("tab_dlnr", ctypes.c_double),
        ("tab_lnu0", ctypes.c_double), ("tab_dlnu", ctypes.c_double),
        ("mu_mode", ctypes.c_int32), ("mu_const", ctypes.c_double), ("mu_pfactor", ctypes.c_double),
        ("yield_mode", ctypes.c_int32), ("y0_mode", ctypes.c_int32), ("y0_const", ctypes.c_double),
        ("y0_over_E", ctypes.c_double),
        ("break_mode", ctypes.c_int32), ("eps_break", ctypes.c_double),
        ("rotation", ctypes.c_int32),
        ("nstars", ctypes.c_int32), ("star_info", _dp),
        ("ext", ctypes.c_int32), ("ext_n", ctypes.c_int32), ("ext_g", _dp), ("ext_dr", ctypes.c_double),
        ("wall_in", ctypes.c_double), ("wall_out", ctypes.c_double), ("wall_k", ctypes.c_double),
        ("damping", ctypes.c_double), ("density_mode", ctypes.c_int32), ("energy_mode", ctypes.c_int32),
        ("dtP_mode", ctypes.c_int32), ("cfl", ctypes.c_double),
    ]


class OrcState(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, _dp) for k in
                ("x", "y", "z", "vx", "vy", "vz", "u", "h", "S")] + [
        ("type", ctypes.POINTER(ctypes.c_int8)), ("broken", ctypes.POINTER(ctypes.c_uint8))] + [
        (k, _dp) for k in ("D", "rho", "P", "cs", "mu", "Y0", "B", "ax", "ay", "az", "dudt", "dSdt",
                           "sdot")] + [("star", ctypes.POINTER(ctypes.c_int32)), ("dDdt", _dp), ("Pprev", _dp),
                                       ("dtprev", ctypes.c_double), ("dt_next", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liboracle.so is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, S = ctypes.POINTER(OrcParams), ctypes.POINTER(OrcState)
        i64p, i32p = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
        L.orc_neighbours.argtypes = [P, ctypes.c_int64, _dp, _dp, _dp, _dp, ctypes.c_int32, i64p, i32p,
                                     ctypes.c_int64]
        L.orc_kernel.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_kernel.restype = None
        L.orc_lambda_max.argtypes = [ctypes.c_int64, _dp, _dp]
        L.orc_lambda_max.restype = None
        L.orc_density.argtypes = [P, S, i64p, i32p]
        L.orc_stress_rate.argtypes = [P, S, i64p, i32p, _dp]
        L.orc_forces.argtypes = [P, S, i64p, i32p, _dp, _dp]
        L.orc_pair_forces.argtypes = [P, S, _dp]
        L.orc_yield.argtypes = [P, ctypes.c_int64, _dp, _dp]
        L.orc_yield.restype = None
        L.orc_step.argtypes = [P, S, ctypes.c_double, ctypes.c_int32, ctypes.c_int32]
        L.orc_evaluate.argtypes = [P, S, ctypes.c_int32]
        _lib = L
    return _lib


def _ptr(a, ct=ctypes.c_double):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ct))


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != ORC_OK:
        raise OracleError(f"{what}: oracle status {STATUS_NAMES.get(rc, rc)}")


class Oracle:
    """Holds an orc_params struct (and the arrays it points to) for one MethodParams."""

    def __init__(self, params, star_info=None):
        """star_info: optional [nstars, 5] array of (centre x, y, z, particle mass, shear factor)
        for an ensemble of stars (the state then carries each particle's star)."""
        from sph_inputs.params import (BACKGROUNDS, BREAK_MODES, DENSITY_MODES, DTP_MODES, ENERGY_MODES,
                                       H_MODES, KERNELS, MU_MODES, ROTATIONS, Y0_MODES, YIELD_MODES)
        self.params = params
        p = OrcParams()
        p.kernel = KERNELS[params.kernel]
        p.h_mode = H_MODES[params.h_mode]
        p.background = BACKGROUNDS[params.background]
        p.periodic = int(bool(params.periodic))
        p.eta, p.box, p.m = params.eta, params.box, params.m
        self._keep = []
        if params.bg_table is not None:
            bg = np.ascontiguousarray(params.bg_table, dtype=np.float64)
            self._keep.append(bg)
            p.bg, p.bg_n, p.bg_dr, p.bg_M = _ptr(bg), bg.shape[1], params.bg_dr, params.bg_M
        p.visc_alpha, p.visc_beta, p.visc_eps = params.visc_alpha, params.visc_beta, params.visc_eps
        if params.eos == "GAMMA_LAW":
            p.eos = 0
        elif params.eos in ("TABLE", "MLP"):
            p.eos = 1   # the oracle evaluates every EoS mode with the table itself
        p.gamma = params.gamma
        if params.table is not None:
            t = params.table
            a, b = np.ascontiguousarray(t.lnP), np.ascontiguousarray(t.lncs2)
            self._keep += [a, b]
            p.tab_lnP, p.tab_lncs2, p.tab_nr, p.tab_nu = _ptr(a), _ptr(b), t.nr, t.nu
            p.tab_lnr0, p.tab_dlnr, p.tab_lnu0, p.tab_dlnu = t.lnr0, t.dlnr, t.lnu0, t.dlnu
        p.mu_mode = MU_MODES[params.mu_mode]
        p.mu_const, p.mu_pfactor = params.mu_const, params.mu_pfactor
        p.yield_mode = YIELD_MODES[params.yield_mode]
        p.y0_mode = Y0_MODES[params.y0_mode]
        p.y0_const, p.y0_over_E = params.y0_const, params.y0_over_E
        p.break_mode = BREAK_MODES[params.break_mode]
        p.eps_break = params.eps_break
        p.rotation = ROTATIONS[params.rotation]
        if params.ext_table is not None:
            eg = np.ascontiguousarray(params.ext_table, dtype=np.float64)
            self._keep.append(eg)
            p.ext, p.ext_g, p.ext_n, p.ext_dr = 1, _ptr(eg), eg.shape[0], params.ext_dr
        p.wall_in, p.wall_out, p.wall_k, p.damping = params.wall_in, params.wall_out, params.wall_k, params.damping
        p.density_mode = DENSITY_MODES[params.density_mode]
        p.energy_mode = ENERGY_MODES[params.energy_mode]
        p.dtP_mode = DTP_MODES[params.dtP_mode]
        p.cfl = params.cfl
        if star_info is not None:
            si = np.ascontiguousarray(star_info, dtype=np.float64)
            assert si.ndim == 2 and si.shape[1] == 5
            self._keep.append(si)
            p.nstars, p.star_info = si.shape[0], _ptr(si)
        self.p = p

    # -- neighbour sets --------------------------------------------------------------
    def neighbours(self, x, y, z, h, mode=GRID, cap=None):
        n = x.shape[0]
        off = np.zeros(n + 1, np.int64)
        cap = cap if cap is not None else max(64 * n, 1024)
        for _ in range(2):
            ids = np.zeros(max(cap, 1), np.int32)
            rc = lib().orc_neighbours(ctypes.byref(self.p), n, _ptr(x), _ptr(y), _ptr(z), _ptr(h),
                                      mode, _ptr(off, ctypes.c_int64), _ptr(ids, ctypes.c_int32), cap)
            if rc == 5:
                cap = int(off[n]) + 1
                continue
            _check(rc, "orc_neighbours")
            return off, ids[: off[n]].copy()
        raise OracleError("neighbour capacity")


class OracleState:
    """numpy-backed particle state plus every output array the oracle writes."""

    FIELDS = ("x", "y", "z", "vx", "vy", "vz", "u", "h")
    OUT = ("D", "rho", "P", "cs", "mu", "Y0", "B", "ax", "ay", "az", "dudt", "sdot", "dDdt", "Pprev")

    def __init__(self, arrays):
        n = arrays["x"].shape[0]
        self.n = n
        self.a = {k: np.ascontiguousarray(arrays[k], dtype=np.float64).copy() for k in self.FIELDS}
        self.a["S"] = np.ascontiguousarray(arrays["S"], dtype=np.float64).reshape(6, n).copy()
        self.a["type"] = np.ascontiguousarray(arrays["type"], dtype=np.int8).copy()
        self.a["broken"] = np.ascontiguousarray(arrays["broken"], dtype=np.uint8).copy()
        for k in self.OUT:
            self.a[k] = np.zeros(n)
        if arrays.get("D") is not None:      # the continuity density starts from the given D
            self.a["D"] = np.ascontiguousarray(arrays["D"], dtype=np.float64).copy()
        self.dtprev = 0.0
        self.dt_next = 0.0
        self.a["dSdt"] = np.zeros((6, n))
        self.a["id"] = np.asarray(arrays.get("id", np.arange(n)), dtype=np.int32).copy()
        if arrays.get("star") is not None:
            self.a["star"] = np.ascontiguousarray(arrays["star"], dtype=np.int32).copy()

    def __getitem__(self, k):
        return self.a[k]

    def struct(self):
        s = OrcState()
        s.n = self.n
        for k in self.FIELDS + self.OUT + ("S", "dSdt"):
            setattr(s, k, _ptr(self.a[k]))
        s.type = _ptr(self.a["type"], ctypes.c_int8)
        s.broken = _ptr(self.a["broken"], ctypes.c_uint8)
        s.star = _ptr(self.a["star"], ctypes.c_int32) if "star" in self.a else None
        s.dtprev = self.dtprev
        s.dt_next = self.dt_next
        self._s = s
        return s

    def sync_scalars(self, s=None):
        """Copy the scalar fields the oracle wrote back from its struct."""
        s = s or self._s
        self.dtprev = s.dtprev
        self.dt_next = s.dt_next


def run_stages(orc: Oracle, st: OracleState, mode=GRID, want_kappa=False):
    """Neighbours, density, stress rate and forces at the current state; returns CSR and kappas."""
    a = st.a
    off, ids = orc.neighbours(a["x"], a["y"], a["z"], a["h"], mode)
    s = st.struct()
    L = lib()
    o64, i32 = _ptr(off, ctypes.c_int64), _ptr(ids, ctypes.c_int32)
    _check(L.orc_density(ctypes.byref(orc.p), ctypes.byref(s), o64, i32), "orc_density")
    kG = np.zeros(st.n) if want_kappa else None
    _check(L.orc_stress_rate(ctypes.byref(orc.p), ctypes.byref(s), o64, i32, _ptr(kG)), "orc_stress_rate")
    ka = np.zeros(st.n) if want_kappa else None
    ku = np.zeros(st.n) if want_kappa else None
    _check(L.orc_forces(ctypes.byref(orc.p), ctypes.byref(s), o64, i32, _ptr(ka), _ptr(ku)), "orc_forces")
    st.sync_scalars(s)
    return dict(offsets=off, ids=ids, kappa_G=kG, kappa_a=ka, kappa_u=ku)


def modify_energy(orc: Oracle, st: OracleState, u_of_r, dr: float):
    """Modification step: u from the profile u(r) (table on r_i = i dr), velocities zeroed."""
    L = lib()
    L.orc_modify_energy.argtypes = [ctypes.POINTER(OrcParams), ctypes.POINTER(OrcState), _dp, ctypes.c_int32,
                                    ctypes.c_double]
    L.orc_modify_energy.restype = None
    t = np.ascontiguousarray(u_of_r, np.float64)
    s = st.struct()
    L.orc_modify_energy(ctypes.byref(orc.p), ctypes.byref(s), _ptr(t), t.shape[0], float(dr))


class OrcDiagParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("r_lo", "r_hi", "slab_r", "slab_dr", "slab_th", "slab_dth")]


class OrcDiag(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("kinetic", "toroidal", "internal", "u_band", "slab_c0", "slab_cr",
                                               "slab_cth")] + [("n_band", ctypes.c_int64), ("n_slab", ctypes.c_int64),
                                                               ("tor_l2", ctypes.c_double)]


def diagnostics(orc: Oracle, st: OracleState, r_lo, r_hi, slab_r, slab_dr, slab_th, slab_dth):
    """Oscillation diagnostics of the current state (see orc_diagnostics) as a dict."""
    L = lib()
    L.orc_diagnostics.argtypes = [ctypes.POINTER(OrcParams), ctypes.POINTER(OrcState), ctypes.POINTER(OrcDiagParams),
                                  ctypes.POINTER(OrcDiag)]
    L.orc_diagnostics.restype = None
    dp = OrcDiagParams(r_lo, r_hi, slab_r, slab_dr, slab_th, slab_dth)
    out = OrcDiag()
    s = st.struct()
    L.orc_diagnostics(ctypes.byref(orc.p), ctypes.byref(s), ctypes.byref(dp), ctypes.byref(out))
    return {k: getattr(out, k) for k, _ in OrcDiag._fields_}


def threads():
    """OpenMP threads the oracle's parallel loops use."""
    L = lib()
    L.orc_threads.restype = ctypes.c_int32
    return int(L.orc_threads())


def step(orc: Oracle, st: OracleState, dt: float, nsteps: int, mode=GRID):
    """nsteps kick-drift-kick steps; dt <= 0: each step's Courant dt from the last evaluation."""
    s = st.struct()
    _check(lib().orc_step(ctypes.byref(orc.p), ctypes.byref(s), dt, nsteps, mode), "orc_step")
    st.sync_scalars(s)


def kernel(kind: int, r: float, hab: float):
    W, F = ctypes.c_double(), ctypes.c_double()
    lib().orc_kernel(kind, r, hab, ctypes.byref(W), ctypes.byref(F))
    return W.value, F.value


def lambda_max(s6_aos: np.ndarray):
    s6 = np.ascontiguousarray(s6_aos, dtype=np.float64)
    out = np.zeros(s6.shape[0])
    lib().orc_lambda_max(s6.shape[0], _ptr(s6), _ptr(out))
    return out


def pair_forces(orc: Oracle, st: OracleState):
    F = np.zeros((st.n, st.n, 3))
    s = st.struct()
    _check(lib().orc_pair_forces(ctypes.byref(orc.p), ctypes.byref(s), _ptr(F)), "orc_pair_forces")
    return F


def yield_scale(orc: Oracle, S6n: np.ndarray, Y0: np.ndarray):
    S = np.ascontiguousarray(S6n, dtype=np.float64).copy()
    Y = np.ascontiguousarray(Y0, dtype=np.float64)
    lib().orc_yield(ctypes.byref(orc.p), S.shape[1], _ptr(S), _ptr(Y))
    return S


# ---- EoS surrogate network ---------------------------------------------------------------------
MLP_NPARAM = 8642


def _mlp_lib():
    L = lib()
    L.orc_mlp_forward.argtypes = [_dp, ctypes.c_int64, _dp, _dp]
    L.orc_mlp_forward.restype = None
    L.orc_mlp_loss_grad.argtypes = [_dp, ctypes.c_int64, _dp, _dp, _dp]
    L.orc_mlp_loss_grad.restype = ctypes.c_double
    L.orc_mlp_features.argtypes = [_dp, ctypes.c_int64, _dp, _dp]
    L.orc_mlp_features.restype = None
    return L


def mlp_forward(w, x):
    """Network outputs for normalised inputs x[n, 2] with flat FP64 parameters w."""
    w = np.ascontiguousarray(w, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros_like(x)
    _mlp_lib().orc_mlp_forward(_ptr(w), x.shape[0], _ptr(x), _ptr(y))
    return y


def mlp_features(w, x):
    """The last hidden layer h[n, 64] of the network for normalised inputs x[n, 2]."""
    w = np.ascontiguousarray(w, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    h = np.zeros((x.shape[0], 64))
    _mlp_lib().orc_mlp_features(_ptr(w), x.shape[0], _ptr(x), _ptr(h))
    return h


def mlp_fit_readout(w, x, t, ridge=0.0):
    """Least-squares readout: parameters w with W4, b4 replaced by the solution of the normal
    equations (G + lambda I) [W4 b4]^T = [h 1]^T t, G = [h 1]^T [h 1] over samples x[n, 2] with
    targets t[n, 2], lambda = ridge * mean(diag G); the hidden layers are those of w."""
    w = np.array(w, np.float64)
    H = np.concatenate([mlp_features(w, x), np.ones((x.shape[0], 1))], axis=1)
    G = H.T @ H
    G[np.diag_indices_from(G)] += ridge * np.trace(G) / G.shape[0]
    sol = np.linalg.solve(G, H.T @ np.asarray(t, np.float64))   # [65, 2]
    w[8512:8640] = sol[:64].T.reshape(-1)
    w[8640:8642] = sol[64]
    return w


def mlp_loss_grad(w, x, t):
    """(loss, dloss/dw) of the mean squared error over samples x[n, 2], targets t[n, 2]."""
    w = np.ascontiguousarray(w, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    g = np.zeros(MLP_NPARAM)
    loss = _mlp_lib().orc_mlp_loss_grad(_ptr(w), x.shape[0], _ptr(x), _ptr(t), _ptr(g))
    return loss, g
