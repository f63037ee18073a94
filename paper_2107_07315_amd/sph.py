"""ctypes binding of libsph (include/sph.h).

Argument marshalling only: every stage runs in the HIP kernels of libsph.so.  PyTorch provides
device memory (tensors) and the HIP stream.  Importing this module does not need a GPU; loading
the library does, and any call fails loudly if the library or the GPU is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

STATUS = {0: "SPH_OK", 1: "SPH_E_ARG", 2: "SPH_E_HIP", 3: "SPH_E_OOM", 4: "SPH_E_ORDER",
          5: "SPH_E_NGB_CAPACITY", 6: "SPH_E_NONFINITE", 7: "SPH_E_EOS_DOMAIN"}

EXPORTED = ("sph_create", "sph_destroy", "sph_set_params", "sph_build_cells", "sph_density",
            "sph_stress_rate", "sph_forces", "sph_step", "sph_sync", "sph_export_neighbours",
            "sph_status_string", "sph_error_particle", "sph_set_timing", "sph_get_timing", "sph_neighbour_stats",
            "sph_mlp_set_params", "sph_mlp_get_params", "sph_mlp_get_norm", "sph_mlp_train", "sph_mlp_grad",
            "sph_mlp_eval", "sph_mlp_build_trust_mask", "sph_ensemble_set", "sph_autotune", "sph_mlp_load",
            "sph_last_error_detail", "sph_eos_table_create", "sph_neighbour_stats_noalloc", "sph_modify_energy",
            "sph_diagnostics", "sph_get_time", "sph_mlp_count_served", "sph_mlp_set_domain", "sph_mlp_fit_readout")
MLP_NPARAM = 8642

_dp = ctypes.c_void_p


class SphParams(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_int32), ("h_mode", ctypes.c_int32), ("background", ctypes.c_int32),
        ("periodic", ctypes.c_int32), ("eta", ctypes.c_double), ("box", ctypes.c_double),
        ("m", ctypes.c_double), ("bg", _dp), ("bg_n", ctypes.c_int32), ("bg_dr", ctypes.c_double),
        ("bg_M", ctypes.c_double), ("visc_alpha", ctypes.c_double), ("visc_beta", ctypes.c_double),
        ("visc_eps", ctypes.c_double), ("eos", ctypes.c_int32), ("gamma", ctypes.c_double),
        ("tab_lnP", _dp), ("tab_lncs2", _dp), ("tab_nr", ctypes.c_int32), ("tab_nu", ctypes.c_int32),
        ("tab_lnr0", ctypes.c_double), ("tab_dlnr", ctypes.c_double), ("tab_lnu0", ctypes.c_double),
        ("tab_dlnu", ctypes.c_double), ("mu_mode", ctypes.c_int32), ("mu_const", ctypes.c_double),
        ("mu_pfactor", ctypes.c_double), ("yield_mode", ctypes.c_int32), ("y0_mode", ctypes.c_int32),
        ("y0_const", ctypes.c_double), ("y0_over_E", ctypes.c_double), ("break_mode", ctypes.c_int32),
        ("eps_break", ctypes.c_double), ("rotation", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("max_neighbours", ctypes.c_int32), ("cell_div", ctypes.c_int32),
        ("tile_cut", ctypes.c_double), ("skin", ctypes.c_double),
        ("pass_blocks", ctypes.c_int32), ("graph", ctypes.c_int32), ("lanes", ctypes.c_int32),
        ("ext", ctypes.c_int32), ("ext_n", ctypes.c_int32), ("ext_g", _dp), ("ext_dr", ctypes.c_double),
        ("wall_in", ctypes.c_double), ("wall_out", ctypes.c_double), ("wall_k", ctypes.c_double),
        ("damping", ctypes.c_double), ("density_mode", ctypes.c_int32), ("energy_mode", ctypes.c_int32),
        ("dtP_mode", ctypes.c_int32), ("reserved", ctypes.c_int32), ("cfl", ctypes.c_double),
    ]


class SphTuneResult(ctypes.Structure):
    _fields_ = [("pass_blocks", ctypes.c_int32), ("trials", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("tile_cut", ctypes.c_double),
                ("skin", ctypes.c_double), ("ms_per_step", ctypes.c_double),
                ("ms_per_step_start", ctypes.c_double)]


class SphListStats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("max_count", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("tiles", ctypes.c_int64), ("union_total", ctypes.c_int64),
                ("candidates", ctypes.c_int64), ("rebuilds", ctypes.c_int64)]


class SphDiagParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("r_lo", "r_hi", "slab_r", "slab_dr", "slab_th", "slab_dth")]


DIAG_FIELDS = ("kinetic", "toroidal", "internal", "u_band", "slab_c0", "slab_cr", "slab_cth", "n_band", "n_slab",
               "tor_l2")


class SphState(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, _dp) for k in (
        "x", "y", "z", "vx", "vy", "vz", "u", "h", "S", "type", "broken", "id", "star",
        "D", "rho", "P", "cs", "ax", "ay", "az", "dudt", "dSdt")]


class SphError(RuntimeError):
    def __init__(self, code, what, particle=None, detail=None):
        at = f" (particle {particle})" if particle is not None and particle >= 0 else ""
        why = f" [{detail}]" if detail else ""
        super().__init__(f"{what}: {STATUS.get(code, code)}{at}{why}")
        self.code = code
        self.particle = particle
        self.detail = detail


_lib = None


def load():
    """Load libsph.so (torch first, so that the HIP runtime it carries is the one in use)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime comes with torch)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, S = ctypes.POINTER(SphParams), ctypes.POINTER(SphState)
    vp = ctypes.c_void_p
    L.sph_create.argtypes = [P, vp, ctypes.c_int64, ctypes.POINTER(vp)]
    L.sph_destroy.argtypes = [vp]
    L.sph_destroy.restype = None
    L.sph_set_params.argtypes = [vp, P]
    for f in ("sph_build_cells", "sph_density", "sph_stress_rate", "sph_forces"):
        getattr(L, f).argtypes = [vp, S]
    L.sph_step.argtypes = [vp, S, ctypes.c_double, ctypes.c_int32]
    L.sph_sync.argtypes = [vp]
    L.sph_error_particle.argtypes = [vp]
    L.sph_error_particle.restype = ctypes.c_int32
    L.sph_export_neighbours.argtypes = [vp, vp, vp, ctypes.c_int64]
    L.sph_status_string.argtypes = [ctypes.c_int]
    L.sph_status_string.restype = ctypes.c_char_p
    L.sph_set_timing.argtypes = [vp, ctypes.c_int32]
    L.sph_neighbour_stats.argtypes = [vp, ctypes.POINTER(SphListStats)]
    L.sph_neighbour_stats_noalloc.argtypes = [vp, ctypes.POINTER(SphListStats)]
    L.sph_get_timing.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_double)]
    L.sph_mlp_set_params.argtypes = [vp, vp]
    L.sph_mlp_get_params.argtypes = [vp, vp, ctypes.c_int32]
    L.sph_mlp_get_norm.argtypes = [vp, vp]
    L.sph_mlp_train.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_float, vp]
    L.sph_mlp_grad.argtypes = [vp, vp, vp, ctypes.c_int64, vp, ctypes.POINTER(ctypes.c_double)]
    L.sph_mlp_eval.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp]
    L.sph_mlp_build_trust_mask.argtypes = [vp, ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]
    L.sph_ensemble_set.argtypes = [vp, ctypes.c_int32, vp]
    L.sph_autotune.argtypes = [vp, S, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(SphTuneResult)]
    L.sph_mlp_load.argtypes = [vp, vp]
    L.sph_modify_energy.argtypes = [vp, S, vp, ctypes.c_int32, ctypes.c_double]
    L.sph_diagnostics.argtypes = [vp, S, ctypes.POINTER(SphDiagParams), vp]
    L.sph_get_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.sph_mlp_count_served.argtypes = [vp, S, ctypes.POINTER(ctypes.c_int64)]
    L.sph_mlp_set_domain.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.sph_mlp_fit_readout.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double)]
    L.sph_last_error_detail.argtypes = [vp]
    L.sph_last_error_detail.restype = ctypes.c_char_p
    L.sph_eos_table_create.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double]
    _lib = L
    return L


def _check(rc, what, h=None):
    if rc != 0:
        d = _lib.sph_last_error_detail(h) if _lib is not None else None
        raise SphError(rc, what, detail=d.decode() if d else None)


# ------------------------------------------------------------------------------------------
# state on the device


class DeviceState:
    """Particle state as torch tensors on the GPU plus the sph_state struct pointing at them."""

    F64 = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "D", "rho", "P", "cs", "ax", "ay", "az", "dudt")

    def __init__(self, arrays: dict, device="cuda", star=None):
        if star is None:
            star = arrays.get("star")
        import torch
        n = int(np.asarray(arrays["x"]).shape[0])
        self.n = n
        t = {}
        dev = torch.device(device)
        for k in self.F64:
            src = arrays.get(k)
            t[k] = (torch.as_tensor(np.ascontiguousarray(src, dtype=np.float64), device=dev).clone()
                    if src is not None else torch.zeros(n, dtype=torch.float64, device=dev))
        t["S"] = torch.as_tensor(np.ascontiguousarray(np.asarray(arrays["S"], np.float64).reshape(6, n)),
                                 device=dev).clone()
        t["dSdt"] = torch.zeros((6, n), dtype=torch.float64, device=dev)
        t["type"] = torch.as_tensor(np.asarray(arrays["type"], np.int8), device=dev).clone()
        t["broken"] = torch.as_tensor(np.asarray(arrays["broken"], np.uint8), device=dev).clone()
        t["id"] = torch.as_tensor(np.asarray(arrays.get("id", np.arange(n)), np.int32), device=dev).clone()
        if star is not None:
            t["star"] = torch.as_tensor(np.asarray(star, np.int32), device=dev).clone()
        self.t = t
        self.struct = SphState()
        self.struct.n = n
        for k, v in t.items():
            setattr(self.struct, k, v.data_ptr())
        if "star" not in t:
            self.struct.star = None

    def __getitem__(self, k):
        return self.t[k]

    def numpy(self, keys=None):
        keys = keys or list(self.t)
        return {k: self.t[k].cpu().numpy() for k in keys}


# ------------------------------------------------------------------------------------------
# context


class Context:
    """Owns an sph_ctx and the device copies of the background and EoS tables."""

    # relative Verlet skin of the candidate lists (0: rebuild at every evaluation), by pair-sum
    # precision: a larger skin means fewer list builds but more candidates, and a candidate costs
    # more in FP64 (measured optima on the 2M-particle star)
    DEFAULT_SKIN = {"FP32": 0.14, "FP64": 0.08}

    def __init__(self, params, capacity: int, stream=None, max_neighbours=0, cell_div=0, tile_cut=0.0,
                 skin=None, pass_blocks=0, graph=False, lanes=0):
        import torch
        from sph_inputs.params import (BACKGROUNDS, BREAK_MODES, DENSITY_MODES, DTP_MODES, ENERGY_MODES,
                                       EOS_KINDS, H_MODES, KERNELS, MU_MODES, PRECISIONS, ROTATIONS, Y0_MODES,
                                       YIELD_MODES)
        L = load()
        if not torch.cuda.is_available():
            raise RuntimeError("libsph needs a GPU: torch.cuda.is_available() is False")
        self.lib = L
        self.params = params
        self._keep = []
        p = SphParams()
        p.kernel = KERNELS[params.kernel]
        p.h_mode = H_MODES[params.h_mode]
        p.background = BACKGROUNDS[params.background]
        p.periodic = int(bool(params.periodic))
        p.eta, p.box, p.m = params.eta, params.box, params.m
        if params.bg_table is not None:
            bg = torch.as_tensor(np.ascontiguousarray(params.bg_table, np.float64), device="cuda")
            self._keep.append(bg)
            p.bg, p.bg_n, p.bg_dr, p.bg_M = bg.data_ptr(), bg.shape[1], params.bg_dr, params.bg_M
        p.visc_alpha, p.visc_beta, p.visc_eps = params.visc_alpha, params.visc_beta, params.visc_eps
        p.eos = EOS_KINDS[params.eos]
        p.gamma = params.gamma
        if params.table is not None:
            tb = params.table
            a = torch.as_tensor(np.ascontiguousarray(tb.lnP), device="cuda")
            b = torch.as_tensor(np.ascontiguousarray(tb.lncs2), device="cuda")
            self._keep += [a, b]
            p.tab_lnP, p.tab_lncs2, p.tab_nr, p.tab_nu = a.data_ptr(), b.data_ptr(), tb.nr, tb.nu
            p.tab_lnr0, p.tab_dlnr, p.tab_lnu0, p.tab_dlnu = tb.lnr0, tb.dlnr, tb.lnu0, tb.dlnu
        p.mu_mode = MU_MODES[params.mu_mode]
        p.mu_const, p.mu_pfactor = params.mu_const, params.mu_pfactor
        p.yield_mode = YIELD_MODES[params.yield_mode]
        p.y0_mode = Y0_MODES[params.y0_mode]
        p.y0_const, p.y0_over_E = params.y0_const, params.y0_over_E
        p.break_mode = BREAK_MODES[params.break_mode]
        p.eps_break = params.eps_break
        p.rotation = ROTATIONS[params.rotation]
        p.precision = PRECISIONS[params.precision]
        p.max_neighbours = max_neighbours
        p.cell_div = cell_div
        p.tile_cut = tile_cut
        p.skin = self.DEFAULT_SKIN[params.precision] if skin is None else skin
        p.pass_blocks = int(pass_blocks)
        p.graph = int(bool(graph))
        p.lanes = int(lanes)
        if params.ext_table is not None:
            eg = torch.as_tensor(np.ascontiguousarray(params.ext_table, np.float64), device="cuda")
            self._keep.append(eg)
            p.ext, p.ext_g, p.ext_n, p.ext_dr = 1, eg.data_ptr(), eg.shape[0], params.ext_dr
        p.wall_in, p.wall_out, p.wall_k, p.damping = params.wall_in, params.wall_out, params.wall_k, params.damping
        p.density_mode = DENSITY_MODES[params.density_mode]
        p.energy_mode = ENERGY_MODES[params.energy_mode]
        p.dtP_mode = DTP_MODES[params.dtP_mode]
        p.cfl = params.cfl
        self.p = p
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(L.sph_create(ctypes.byref(p), ctypes.c_void_p(self.stream.cuda_stream), int(capacity),
                            ctypes.byref(h)), "sph_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.sph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # stage calls -----------------------------------------------------------------------------
    def sph_build_cells(self, st: DeviceState):
        _check(self.lib.sph_build_cells(self.h, ctypes.byref(st.struct)), "sph_build_cells", self.h)

    def sph_density(self, st: DeviceState):
        _check(self.lib.sph_density(self.h, ctypes.byref(st.struct)), "sph_density", self.h)

    def sph_stress_rate(self, st: DeviceState):
        _check(self.lib.sph_stress_rate(self.h, ctypes.byref(st.struct)), "sph_stress_rate", self.h)

    def sph_forces(self, st: DeviceState):
        _check(self.lib.sph_forces(self.h, ctypes.byref(st.struct)), "sph_forces", self.h)

    def sph_step(self, st: DeviceState, dt: float, nsteps: int):
        _check(self.lib.sph_step(self.h, ctypes.byref(st.struct), float(dt), int(nsteps)), "sph_step", self.h)

    def sph_get_time(self):
        t = ctypes.c_double()
        _check(self.lib.sph_get_time(self.h, ctypes.byref(t)), "sph_get_time", self.h)
        return t.value

    def sph_sync(self):
        """Waits; raises SphError for a latched device error, with .particle the array index (in
        the current order) of the particle that raised it, or -1."""
        rc = self.lib.sph_sync(self.h)
        if rc != 0:
            d = self.lib.sph_last_error_detail(self.h)
            raise SphError(rc, "sph_sync", int(self.lib.sph_error_particle(self.h)), d.decode() if d else None)

    def sph_export_neighbours(self, n: int, cap: int = None):
        off = np.zeros(n + 1, np.int64)
        cap = cap if cap is not None else 128 * max(n, 1)
        ids = np.zeros(cap, np.int32)
        rc = self.lib.sph_export_neighbours(self.h, off.ctypes.data, ids.ctypes.data, cap)
        if rc == 5:
            cap = int(off[n])
            ids = np.zeros(max(cap, 1), np.int32)
            rc = self.lib.sph_export_neighbours(self.h, off.ctypes.data, ids.ctypes.data, cap)
        _check(rc, "sph_export_neighbours")
        return off, ids[: off[n]].copy()

    def sph_modify_energy(self, st: DeviceState, u_of_r, dr: float):
        """Modification step: u from the profile u(r) (device tensor or array on r_i = i dr)."""
        import torch
        t = torch.as_tensor(np.ascontiguousarray(u_of_r, np.float64), device="cuda")
        self._keep.append(t)
        _check(self.lib.sph_modify_energy(self.h, ctypes.byref(st.struct), t.data_ptr(), t.shape[0], float(dr)),
               "sph_modify_energy", self.h)

    def sph_diagnostics(self, st: DeviceState, r_lo, r_hi, slab_r, slab_dr, slab_th, slab_dth, out=None):
        """Oscillation diagnostics of the state.  With out (a device tensor of 72 bytes) the record is
        written there, stream-ordered, and None is returned; without, it is read back as a dict."""
        import torch
        dp = SphDiagParams(r_lo, r_hi, slab_r, slab_dr, slab_th, slab_dth)
        buf = out if out is not None else torch.zeros(10, dtype=torch.float64, device="cuda")
        _check(self.lib.sph_diagnostics(self.h, ctypes.byref(st.struct), ctypes.byref(dp), buf.data_ptr()),
               "sph_diagnostics", self.h)
        if out is not None:
            return None
        raw = buf.cpu().numpy()
        d = {k: float(raw[i]) for i, k in enumerate(DIAG_FIELDS[:7])}
        d["n_band"] = int(raw[7:8].view(np.int64)[0])
        d["n_slab"] = int(raw[8:9].view(np.int64)[0])
        d["tor_l2"] = float(raw[9])
        return d

    def sph_set_timing(self, enable: bool):
        _check(self.lib.sph_set_timing(self.h, int(bool(enable))), "sph_set_timing", self.h)

    def sph_get_timing(self, stage: str):
        n = ctypes.c_int32()
        ms = ctypes.c_double()
        _check(self.lib.sph_get_timing(self.h, stage.encode(), ctypes.byref(n), ctypes.byref(ms)),
               "sph_get_timing")
        return n.value, ms.value

    def sph_neighbour_stats(self):
        s = SphListStats()
        _check(self.lib.sph_neighbour_stats(self.h, ctypes.byref(s)), "sph_neighbour_stats", self.h)
        return {k: getattr(s, k) for k in ("pairs", "max_count", "tiles", "union_total", "candidates",
                                           "rebuilds")}

    def sph_neighbour_stats_noalloc(self):
        s = SphListStats()
        _check(self.lib.sph_neighbour_stats_noalloc(self.h, ctypes.byref(s)), "sph_neighbour_stats_noalloc", self.h)
        return {k: getattr(s, k) for k in ("pairs", "max_count", "tiles", "union_total", "candidates",
                                           "rebuilds")}

    def sph_autotune(self, st: DeviceState, dt: float, steps_per_trial: int = 64):
        r = SphTuneResult()
        _check(self.lib.sph_autotune(self.h, ctypes.byref(st.struct), float(dt), int(steps_per_trial),
                                     ctypes.byref(r)), "sph_autotune")
        return {k: getattr(r, k) for k, _ in SphTuneResult._fields_ if k != "pad"}

    def sph_ensemble_set(self, star_info):
        """star_info: [nstars, 5] rows of (centre x, y, z, particle mass, shear factor)."""
        si = np.ascontiguousarray(star_info, np.float64)
        if si.size == 0:
            _check(self.lib.sph_ensemble_set(self.h, 0, None), "sph_ensemble_set", self.h)
            return
        assert si.ndim == 2 and si.shape[1] == 5
        _check(self.lib.sph_ensemble_set(self.h, si.shape[0], si.ctypes.data), "sph_ensemble_set", self.h)

    # EoS surrogate network ------------------------------------------------------------------
    def mlp_set_params(self, params):
        w = np.ascontiguousarray(params, np.float32)
        assert w.shape == (MLP_NPARAM,)
        _check(self.lib.sph_mlp_set_params(self.h, w.ctypes.data), "sph_mlp_set_params", self.h)

    def mlp_load(self, bf16_bits):
        """bf16_bits: uint16 array of SPH_MLP_NPARAM BF16 bit patterns."""
        w = np.ascontiguousarray(bf16_bits, np.uint16)
        assert w.shape == (MLP_NPARAM,)
        _check(self.lib.sph_mlp_load(self.h, w.ctypes.data), "sph_mlp_load", self.h)

    def eos_table_create(self, table):
        """Upload an EosTable into memory the context owns (sph_eos_table_create)."""
        a = np.ascontiguousarray(table.lnP, np.float64)
        b = np.ascontiguousarray(table.lncs2, np.float64)
        _check(self.lib.sph_eos_table_create(self.h, a.ctypes.data, b.ctypes.data, table.nr, table.nu, table.lnr0,
                                             table.dlnr, table.lnu0, table.dlnu), "sph_eos_table_create", self.h)

    def last_error_detail(self):
        d = self.lib.sph_last_error_detail(self.h)
        return d.decode() if d else ""

    def mlp_get_params(self, rounded=False):
        w = np.zeros(MLP_NPARAM, np.float32)
        _check(self.lib.sph_mlp_get_params(self.h, w.ctypes.data, int(bool(rounded))), "sph_mlp_get_params", self.h)
        return w

    def mlp_get_norm(self):
        v = np.zeros(8, np.float32)
        _check(self.lib.sph_mlp_get_norm(self.h, v.ctypes.data), "sph_mlp_get_norm", self.h)
        return v

    def mlp_train(self, samples, n_holdout, epochs, batch=4096, lr=1e-3):
        """samples: device FP64 tensor [n, 2] of (ln rho, ln u).  Returns per-epoch
        (training-batch loss, holdout loss)."""
        import torch
        assert samples.dtype == torch.float64 and samples.is_cuda and samples.is_contiguous()
        hist = np.zeros((max(epochs, 1), 2), np.float32)
        _check(self.lib.sph_mlp_train(self.h, samples.data_ptr(), samples.shape[0], int(n_holdout), int(epochs),
                                      int(batch), float(lr), hist.ctypes.data), "sph_mlp_train")
        return hist[:epochs]

    def mlp_set_domain(self, lnrho_lo, lnrho_hi, lnu_lo, lnu_hi):
        _check(self.lib.sph_mlp_set_domain(self.h, float(lnrho_lo), float(lnrho_hi), float(lnu_lo), float(lnu_hi)),
               "sph_mlp_set_domain", self.h)

    def mlp_fit_readout(self, samples, n_holdout, ridge=1e-10):
        """Least-squares readout over device FP64 samples [n, 2]; returns the holdout loss after it."""
        import torch
        assert samples.dtype == torch.float64 and samples.is_cuda and samples.is_contiguous()
        hl = ctypes.c_double()
        _check(self.lib.sph_mlp_fit_readout(self.h, samples.data_ptr(), samples.shape[0], int(n_holdout), float(ridge),
                                            ctypes.byref(hl)), "sph_mlp_fit_readout", self.h)
        return hl.value

    def mlp_grad(self, x, t):
        """Gradient of the loss over device FP32 tensors x, t [n, 2] (normalised units)."""
        g = np.zeros(MLP_NPARAM, np.float32)
        loss = ctypes.c_double()
        _check(self.lib.sph_mlp_grad(self.h, x.data_ptr(), t.data_ptr(), x.shape[0], g.ctypes.data,
                                     ctypes.byref(loss)), "sph_mlp_grad")
        return g, loss.value

    def mlp_eval(self, lnrho, lnu):
        import torch
        lp = torch.empty_like(lnrho)
        lc = torch.empty_like(lnrho)
        _check(self.lib.sph_mlp_eval(self.h, lnrho.data_ptr(), lnu.data_ptr(), lnrho.shape[0], lp.data_ptr(),
                                     lc.data_ptr()), "sph_mlp_eval")
        return lp, lc

    def mlp_count_served(self, st: DeviceState):
        n = ctypes.c_int64()
        _check(self.lib.sph_mlp_count_served(self.h, ctypes.byref(st.struct), ctypes.byref(n)), "sph_mlp_count_served",
               self.h)
        return n.value

    def mlp_build_trust_mask(self, tol=1e-4):
        n = ctypes.c_int64()
        _check(self.lib.sph_mlp_build_trust_mask(self.h, float(tol), ctypes.byref(n)), "sph_mlp_build_trust_mask", self.h)
        return n.value

    # convenience ---------------------------------------------------------------------------
    def evaluate(self, st: DeviceState):
        """build_cells -> density -> stress_rate -> forces (the first evaluation of a run)."""
        self.sph_build_cells(st)
        self.sph_density(st)
        self.sph_stress_rate(st)
        self.sph_forces(st)
