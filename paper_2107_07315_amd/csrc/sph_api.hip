// C-ABI entry points of libsph: context, stage calls, time stepping, status and timing.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <chrono>

#include "sph_internal.h"

namespace {

constexpr int64_t kMaxCells = int64_t(1) << 26;

template <typename T>
sph_status dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return SPH_OK;
  if (hipMalloc((void**)p, sizeof(T) * count) != hipSuccess) {
    *p = nullptr;
    return SPH_E_OOM;
  }
  return SPH_OK;
}

// Detail of the last failure of a call without a context (sph_create), per host thread.
thread_local char g_detail[256] = "no error";

sph_status vnote(sph_ctx* c, sph_status e, const char* fmt, va_list ap) {
  char* buf = c ? c->detail : g_detail;
  const size_t cap = c ? sizeof(c->detail) : sizeof(g_detail);
  int k = snprintf(buf, cap, "%s: ", sph_status_string(e));
  if (k < 0) k = 0;
  if ((size_t)k < cap) vsnprintf(buf + k, cap - (size_t)k, fmt, ap);
  return e;
}

sph_status check_params(sph_ctx* c, const sph_params* p) {
  if (!p) return note(c, SPH_E_ARG, "params is NULL");
  if (p->kernel != SPH_WC2 && p->kernel != SPH_WC4) return note(c, SPH_E_ARG, "kernel %d is not SPH_WC2 or SPH_WC4", p->kernel);
  if (!(p->m > 0.0)) return note(c, SPH_E_ARG, "particle mass m = %g must be positive", p->m);
  if (p->background == SPH_TOV && (!p->bg || p->bg_n < 2 || !(p->bg_dr > 0.0)))
    return note(c, SPH_E_ARG, "background TOV needs bg (device), bg_n >= 2 and bg_dr > 0");
  if (p->periodic && !(p->box > 0.0)) return note(c, SPH_E_ARG, "periodic needs box > 0");
  if ((p->tab_lnP || p->tab_lncs2) && (!p->tab_lnP || !p->tab_lncs2 || p->tab_nr < 2 || p->tab_nu < 2))
    return note(c, SPH_E_ARG, "an EoS table needs tab_lnP, tab_lncs2 and tab_nr, tab_nu >= 2");
  if (p->precision != SPH_FP64 && p->precision != SPH_FP32) return note(c, SPH_E_ARG, "precision %d", p->precision);
  if (p->max_neighbours < 0 || p->max_neighbours > 4096)
    return note(c, SPH_E_ARG, "max_neighbours = %d outside [0, 4096]", p->max_neighbours);
  if (p->cell_div < 0 || p->cell_div > 4) return note(c, SPH_E_ARG, "cell_div = %d outside [0, 4]", p->cell_div);
  if (!(p->tile_cut >= 0.0) || p->tile_cut > 64.0) return note(c, SPH_E_ARG, "tile_cut = %g outside [0, 64]", p->tile_cut);
  if (!(p->skin >= 0.0) || p->skin > 1.0) return note(c, SPH_E_ARG, "skin = %g outside [0, 1]", p->skin);
  if (p->pass_blocks < 0 || p->pass_blocks > 65536)
    return note(c, SPH_E_ARG, "pass_blocks = %d outside [0, 65536]", p->pass_blocks);
  if (p->graph < 0 || p->graph > 1) return note(c, SPH_E_ARG, "graph = %d is not 0 or 1", p->graph);
  if (p->lanes != 0 && p->lanes != 1 && p->lanes != 2 && p->lanes != 4)
    return note(c, SPH_E_ARG, "lanes = %d is not 0, 1, 2 or 4", p->lanes);
  if (p->ext != SPH_EXT_NONE && p->ext != SPH_EXT_RADIAL) return note(c, SPH_E_ARG, "ext = %d", p->ext);
  if (p->ext == SPH_EXT_RADIAL && (!p->ext_g || p->ext_n < 2 || !(p->ext_dr > 0.0)))
    return note(c, SPH_E_ARG, "ext RADIAL needs ext_g (device), ext_n >= 2 and ext_dr > 0");
  if (!(p->wall_in >= 0.0) || !(p->wall_out >= 0.0) || !(p->wall_k >= 0.0) || !(p->damping >= 0.0))
    return note(c, SPH_E_ARG, "wall radii, wall_k and damping must not be negative");
  if (p->density_mode != SPH_DENS_SUMMATION && p->density_mode != SPH_DENS_CONTINUITY)
    return note(c, SPH_E_ARG, "density_mode = %d", p->density_mode);
  if (p->energy_mode != SPH_ENERGY_PAPER && p->energy_mode != SPH_ENERGY_FIRST_LAW)
    return note(c, SPH_E_ARG, "energy_mode = %d", p->energy_mode);
  if (p->dtP_mode != SPH_DTP_OFF && p->dtP_mode != SPH_DTP_LAGGED) return note(c, SPH_E_ARG, "dtP_mode = %d", p->dtP_mode);
  if (!(p->cfl >= 0.0) || p->cfl > 1.0) return note(c, SPH_E_ARG, "cfl = %g outside [0, 1]", p->cfl);
  return SPH_OK;
}

sph_status check_state(sph_ctx* c, const sph_state* st) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (!st) return note(c, SPH_E_ARG, "state is NULL");
  if (st->n < 0 || st->n > c->capacity)
    return note(c, SPH_E_ARG, "n = %lld outside [0, capacity = %lld]", (long long)st->n, (long long)c->capacity);
  if (st->n > 0) {
    const void* req[] = {st->x, st->y, st->z, st->vx, st->vy, st->vz, st->u, st->h, st->S, st->type, st->broken,
                         st->id, st->D, st->rho, st->P, st->cs, st->ax, st->ay, st->az, st->dudt, st->dSdt};
    static const char* names[] = {"x", "y", "z", "vx", "vy", "vz", "u", "h", "S", "type", "broken", "id", "D",
                                  "rho", "P", "cs", "ax", "ay", "az", "dudt", "dSdt"};
    for (size_t k = 0; k < sizeof(req) / sizeof(req[0]); ++k)
      if (!req[k]) return note(c, SPH_E_ARG, "state array %s is NULL", names[k]);
  }
  if (c->stars && st->n > 0 && !st->star) return note(c, SPH_E_ARG, "an ensemble is set but state array star is NULL");
  if ((c->p.eos == SPH_EOS_TABLE || c->p.eos == SPH_EOS_MLP) && !c->p.tab_lnP)
    return note(c, SPH_E_ARG, "eos TABLE or MLP needs a table (tab_* parameters or sph_eos_table_create)");
  return SPH_OK;
}

// The context's own table (sph_eos_table_create) stands in for table pointers left NULL.
void use_own_table(const sph_ctx* c, sph_params* p) {
  if (p->tab_lnP || !c->tab_own) return;
  p->tab_lnP = c->tab_own;
  p->tab_lncs2 = c->tab_own + (size_t)c->tab_own_nr * c->tab_own_nu;
  p->tab_nr = c->tab_own_nr;
  p->tab_nu = c->tab_own_nu;
  p->tab_lnr0 = c->tab_own_g[0];
  p->tab_dlnr = c->tab_own_g[1];
  p->tab_lnu0 = c->tab_own_g[2];
  p->tab_dlnu = c->tab_own_g[3];
}

}  // namespace

sph_status note(sph_ctx* c, sph_status e, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vnote(c, e, fmt, ap);
  va_end(ap);
  return e;
}

void timer_begin(sph_ctx* c, int which) {
  if (!c->timing) return;
  StageTimer& t = c->timers[which];
  if (t.used + 2 > t.ev.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      t.ev.push_back(e);
    }
  }
  (void)hipEventRecord(t.ev[t.used], c->stream);
}

void timer_end(sph_ctx* c, int which) {
  if (!c->timing) return;
  StageTimer& t = c->timers[which];
  if (t.used + 2 > t.ev.size()) return;
  (void)hipEventRecord(t.ev[t.used + 1], c->stream);
  t.used += 2;
}

extern "C" {

const char* sph_status_string(sph_status s) {
  switch (s) {
    case SPH_OK: return "SPH_OK";
    case SPH_E_ARG: return "SPH_E_ARG";
    case SPH_E_HIP: return "SPH_E_HIP";
    case SPH_E_OOM: return "SPH_E_OOM";
    case SPH_E_ORDER: return "SPH_E_ORDER";
    case SPH_E_NGB_CAPACITY: return "SPH_E_NGB_CAPACITY";
    case SPH_E_NONFINITE: return "SPH_E_NONFINITE";
    case SPH_E_EOS_DOMAIN: return "SPH_E_EOS_DOMAIN";
  }
  return "SPH_E_UNKNOWN";
}

void sph_destroy(sph_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  void* bufs[] = {c->grid, c->keys, c->vals, c->cell_se, c->pos_sorted, c->sort.keys_alt, c->sort.vals_alt,
                  c->sort.hist, c->sort.rowtot, c->sort.partial, c->sort.scan_bsum, c->tile_u, c->tile_start, c->tile_cnt, c->tile_uoff,
                  c->tile_usize, c->stress_tiles, c->tile_st, c->nbr16, c->nbr_count, c->nbr_count_sl, c->nbr16s, c->nbr_count_s, c->pos_build, c->drift_flag,
                  c->pos4, c->fv, c->fa, c->sig, c->pos4f, c->fvf,
                  c->faf, c->sigf, c->mu, c->Y0, c->B, c->sdot, c->tovf, c->half, c->tmp, c->stars, c->status,
                  c->dsum, c->dDdt, c->xcoef, c->dtw, c->dtpart, c->eos_list, c->eos_list_n};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (c->drift_host) (void)hipHostFree(c->drift_host);
  if (c->tab_own) (void)hipFree(c->tab_own);
  if (c->diag_part) (void)hipFree(c->diag_part);
  mlp_free(c);
  for (auto& t : c->timers)
    for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->step_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->g_eval) (void)hipGraphExecDestroy(c->g_eval);
  if (c->g_drift) (void)hipGraphExecDestroy(c->g_drift);
  if (c->g_chain) (void)hipGraphExecDestroy(c->g_chain);
  c->~sph_ctx();
  free(c);
}

sph_status sph_create(const sph_params* params, void* stream, int64_t capacity, sph_ctx** out) {
  if (!out) return note(nullptr, SPH_E_ARG, "out is NULL");
  *out = nullptr;
  sph_status e = check_params(nullptr, params);
  if (e) return e;
  if (capacity < 1 || capacity > (int64_t(1) << 30))
    return note(nullptr, SPH_E_ARG, "capacity = %lld outside [1, 2^30]", (long long)capacity);
  sph_ctx* c = (sph_ctx*)calloc(1, sizeof(sph_ctx));
  if (!c) return note(nullptr, SPH_E_OOM, "host allocation of the context failed");
  new (c) sph_ctx();
  c->p = *params;
  c->stream = (hipStream_t)stream;
  c->capacity = capacity;
  c->cap = params->max_neighbours > 0 ? params->max_neighbours : 512;
  c->cap_s = (2 * c->cap + 7) / 8 * 8;
  c->ucap = 8192;   // union members per tile; local indices are 16-bit
  // the union pool starts at 128 entries per particle and grows to what the tiles reserve
  c->upool = (int64_t)((capacity + 63) / 64 * 64) * 128;
  if (c->upool > (int64_t)0xffffffffll) c->upool = (int64_t)0xffffffffll;
  (void)hipGetDevice(&c->device);
  c->check_id = 1;   // written by failed drift tests outside a run-ahead step (flag cleared first)
  const int64_t cap = capacity;
  const int64_t capw = (cap + 63) / 64 * 64;
  c->capw = capw;
  // tiles: at most one per particle; the union pool is addressed with 32-bit offsets
  c->cap_tiles = capw;
  c->sort.scan_cap = (capw + 1023) / 1024;
  c->max_cells = kMaxCells;
  c->sort.max_blocks = (int)((cap + 4095) / 4096);
  if ((e = dalloc(&c->grid, 1)) || (e = dalloc(&c->keys, cap)) || (e = dalloc(&c->vals, cap)) ||
      (e = dalloc(&c->cell_se, c->max_cells)) || (e = dalloc(&c->pos_sorted, cap)) ||
      (e = dalloc(&c->sort.keys_alt, cap)) || (e = dalloc(&c->sort.vals_alt, cap)) ||
      (e = dalloc(&c->sort.hist, (size_t)256 * c->sort.max_blocks)) || (e = dalloc(&c->sort.rowtot, 256)) ||
      (e = dalloc(&c->sort.partial, (size_t)8 * 1024)) ||
      (e = dalloc(&c->tile_u, (size_t)c->upool)) || (e = dalloc(&c->tile_usize, c->cap_tiles)) ||
      (e = dalloc(&c->tile_start, c->cap_tiles)) || (e = dalloc(&c->tile_cnt, c->cap_tiles)) ||
      (e = dalloc(&c->stress_tiles, c->cap_tiles)) || (e = dalloc(&c->tile_st, c->cap_tiles)) ||
      (e = dalloc(&c->tile_uoff, c->cap_tiles)) ||
      (e = dalloc(&c->sort.scan_bsum, c->sort.scan_cap + 1)) ||
      (e = dalloc(&c->nbr16, (size_t)capw * slot_entries_max(c->cap))) || (e = dalloc(&c->nbr_count, capw)) ||
      (e = dalloc(&c->nbr_count_sl, (size_t)capw * 4)) ||
      (e = dalloc(&c->nbr16s, (size_t)capw * (c->cap_s + 32))) || (e = dalloc(&c->nbr_count_s, capw)) ||
      (e = dalloc(&c->pos_build, cap)) || (e = dalloc(&c->drift_flag, 1)) ||
      (e = dalloc(&c->pos4, cap)) || (e = dalloc(&c->fv, cap)) || (e = dalloc(&c->fa, cap)) ||
      (e = dalloc(&c->sig, 6 * cap)) || (e = dalloc(&c->pos4f, cap)) || (e = dalloc(&c->fvf, cap)) ||
      (e = dalloc(&c->faf, cap)) || (e = dalloc(&c->sigf, 6 * cap)) || (e = dalloc(&c->mu, cap)) ||
      (e = dalloc(&c->Y0, cap)) || (e = dalloc(&c->B, cap)) || (e = dalloc(&c->sdot, cap)) ||
      (e = dalloc(&c->tovf, cap)) ||
      (e = dalloc(&c->half, SPH_HALF_FIELDS * cap)) || (e = dalloc(&c->tmp, capw)) || (e = dalloc(&c->status, 1)) ||
      (e = dalloc(&c->dsum, cap)) || (e = dalloc(&c->dDdt, cap)) || (e = dalloc(&c->xcoef, 5 * cap)) ||
      (e = dalloc(&c->dtw, 8)) || (e = dalloc(&c->dtpart, 65536 + 4096)) || (e = dalloc(&c->eos_list, cap)) ||
      (e = dalloc(&c->eos_list_n, 1))) {
    sph_destroy(c);
    return note(nullptr, e, "device scratch for capacity %lld does not fit", (long long)capacity);
  }
  if (hipHostMalloc((void**)&c->drift_host, 4 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
    c->drift_host = nullptr;
    sph_destroy(c);
    return note(nullptr, SPH_E_OOM, "pinned host word");
  }
  if ((e = stats_scratch_init(c))) {
    sph_destroy(c);
    return note(nullptr, e, "address of the statistics scratch array on device %d", c->device);
  }

  if (hipMemsetAsync(c->status, 0, sizeof(DevStatus), c->stream) != hipSuccess ||
      hipMemsetAsync(c->nbr_count, 0, sizeof(int32_t) * cap, c->stream) != hipSuccess ||
      hipMemsetAsync(c->nbr_count_sl, 0, sizeof(int32_t) * capw * 4, c->stream) != hipSuccess ||
      hipMemsetAsync(c->nbr_count_s, 0, sizeof(int32_t) * cap, c->stream) != hipSuccess ||
      hipMemsetAsync(c->drift_flag, 0, sizeof(uint32_t), c->stream) != hipSuccess ||
      hipMemsetAsync(c->Y0, 0, sizeof(double) * cap, c->stream) != hipSuccess ||
      hipMemsetAsync(c->dDdt, 0, sizeof(double) * cap, c->stream) != hipSuccess ||
      hipMemsetAsync(c->xcoef, 0, sizeof(double) * 5 * cap, c->stream) != hipSuccess ||
      launch_dt_init(c) != SPH_OK ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    sph_destroy(c);
    return note(nullptr, SPH_E_HIP, "clearing the context's counters failed");
  }
  snprintf(c->detail, sizeof(c->detail), "no error");
  *out = c;
  return SPH_OK;
}

sph_status sph_set_params(sph_ctx* c, const sph_params* params) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  sph_status e = check_params(c, params);
  if (e) return e;
  int cap = params->max_neighbours > 0 ? params->max_neighbours : 512;
  if (cap != c->cap) return note(c, SPH_E_ARG, "max_neighbours cannot change after sph_create");
  c->p = *params;
  use_own_table(c, &c->p);
  c->gen = 0;
  c->lists_valid = false;
  ++c->graph_epoch;
  return SPH_OK;
}

}  // extern "C"

// Copy the drift word to the host and report whether the last test (check_id) saw a violation.
static sph_status read_drift(sph_ctx* c, bool* violated) {
  HIP_TRY(hipMemcpyAsync(c->drift_host, c->drift_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *violated = *c->drift_host != 0u;
  return SPH_OK;
}

// outputs_recomputed: an evaluation follows at once, so the output arrays need not be reordered
static sph_status rebuild(sph_ctx* c, sph_state* st, bool outputs_recomputed = false) {
  timer_begin(c, TIMER_CELLS);
  sph_status e = sph_rebin(c, st, outputs_recomputed);
  timer_end(c, TIMER_CELLS);
  if (e) {
    c->lists_valid = false;
    return e;
  }
  c->lists_valid = true;
  ++c->rebuilds;
  return SPH_OK;
}

extern "C" {

sph_status sph_build_cells(sph_ctx* c, sph_state* st) {
  sph_status e = check_state(c, st);
  if (e) return e;
  if (st->n != c->n) c->lists_valid = false;
  c->n = st->n;
  if (st->n == 0) { c->gen = 1; return SPH_OK; }
  bool stale = !c->lists_valid || !(c->p.skin > 0.0);
  if (!stale) {
    if ((e = launch_flag_clear(c)) || (e = launch_drift_check(c, st)) || (e = read_drift(c, &stale))) return e;
  }
  if (stale) {
    if ((e = rebuild(c, st))) return e;
  } else if ((e = launch_pack(c, st))) {
    return e;
  }
  c->gen = 1;
  return SPH_OK;
}

sph_status sph_density(sph_ctx* c, sph_state* st) {
  sph_status e = check_state(c, st);
  if (e) return e;
  if (c->gen < 1 || st->n != c->n) return note(c, SPH_E_ORDER, "sph_density needs sph_build_cells for this state first");
  if (st->n > 0) {
    timer_begin(c, TIMER_DENSITY);
    e = launch_density(c, st);
    timer_end(c, TIMER_DENSITY);
    if (e) return e;
    timer_begin(c, TIMER_EOS);
    e = launch_eos(c, st);
    timer_end(c, TIMER_EOS);
    if (e) return e;
    if ((e = launch_dt_commit(c, (int)(c->steps_done % 3)))) return e;
  }
  c->gen = 2;
  return SPH_OK;
}

sph_status sph_stress_rate(sph_ctx* c, sph_state* st) {
  sph_status e = check_state(c, st);
  if (e) return e;
  if (c->gen < 2 || st->n != c->n) return note(c, SPH_E_ORDER, "sph_stress_rate needs sph_density first");
  if (st->n > 0) {
    timer_begin(c, TIMER_STRESS);
    e = launch_stress(c, st);
    timer_end(c, TIMER_STRESS);
    if (e) return e;
  }
  c->gen = 3;
  return SPH_OK;
}

sph_status sph_forces(sph_ctx* c, sph_state* st) {
  sph_status e = check_state(c, st);
  if (e) return e;
  if (c->gen < 3 || st->n != c->n) return note(c, SPH_E_ORDER, "sph_forces needs sph_stress_rate first");
  if (st->n > 0) {
    timer_begin(c, TIMER_FORCES);
    e = launch_forces(c, st);
    timer_end(c, TIMER_FORCES);
    if (e) return e;
  }
  c->gen = 4;
  return SPH_OK;
}

}  // extern "C"

// Captures the three graphs of a step: g_drift = flag clear, kick-drift with the skin test and
// the flag copy to pinned host memory (first step of a call); g_chain = the same with the final
// kick of the previous step fused in (later steps); g_eval = density, epilogue, stress rate and
// forces.  The final kick of the call's last step is launched on its own.
static sph_status capture_step(sph_ctx* c, sph_state* st, double dt) {
  if (c->g_eval) (void)hipGraphExecDestroy(c->g_eval);
  if (c->g_drift) (void)hipGraphExecDestroy(c->g_drift);
  if (c->g_chain) (void)hipGraphExecDestroy(c->g_chain);
  c->g_eval = c->g_drift = c->g_chain = nullptr;
  const int32_t timing = c->timing;
  c->timing = 0;   // no event records inside the graphs
  sph_status e = SPH_OK;
  for (int which = 0; which < 3 && !e; ++which) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      e = SPH_E_HIP;
      break;
    }
    sph_status le = SPH_OK;
    if (which == 0) {
      c->eval_in_step = true;   // the lagged dP/dt reads the step's dt
      if (!le) le = launch_density(c, st);
      if (!le) le = launch_eos(c, st);
      if (!le) le = launch_stress(c, st);
      if (!le) le = launch_forces(c, st);
      c->eval_in_step = false;
    } else {
      if (!le) le = launch_flag_clear(c);
      if (!le) le = which == 1 ? launch_kick_drift(c, st, dt, 1u) : launch_kick_final_drift(c, st, dt, 1u);
      if (!le && hipMemcpyAsync(c->drift_host, c->drift_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream) !=
                     hipSuccess)
        le = SPH_E_HIP;
    }
    const hipError_t ee = hipStreamEndCapture(c->stream, &g);
    if (le || ee != hipSuccess) e = le ? le : SPH_E_HIP;
    hipGraphExec_t x = nullptr;
    if (!e && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) e = SPH_E_HIP;
    if (g) (void)hipGraphDestroy(g);
    if (!e) (which == 0 ? c->g_eval : which == 1 ? c->g_drift : c->g_chain) = x;
  }
  c->timing = timing;
  if (!e) {
    c->g_x = st->x;
    c->g_n = st->n;
    c->g_dt = dt;
    c->g_epoch = c->graph_epoch;
  }
  return e;
}

// sph_step with graph replay: per step, g_drift (first step) or g_chain, one word read back, an
// eager candidate-list rebuild if the skin test failed (re-capturing if that moved a buffer), then
// g_eval; the last final kick on its own.
static sph_status step_graphs(sph_ctx* c, sph_state* st, double dt, int32_t nsteps) {
  sph_status e;
  for (int32_t k = 0; k < nsteps; ++k) {
    if (!c->g_eval || c->g_x != st->x || c->g_n != st->n || c->g_dt != dt || c->g_epoch != c->graph_epoch)
      if ((e = capture_step(c, st, dt))) return e;
    HIP_TRY(hipGraphLaunch(k == 0 ? c->g_drift : c->g_chain, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (*c->drift_host != 0u) {
      if ((e = rebuild(c, st, true))) return e;
      if (c->g_epoch != c->graph_epoch && (e = capture_step(c, st, dt))) return e;
    }
    HIP_TRY(hipGraphLaunch(c->g_eval, c->stream));
  }
  return nsteps > 0 ? launch_kick_final(c, st, dt) : SPH_OK;
}

extern "C" {

// The state's x, y, z, h brought up to date from pos4 after deferred kicks.
static sph_status sync_positions(sph_ctx* c, sph_state* st) {
  if (!c->pos_deferred) return SPH_OK;
  c->pos_deferred = false;
  return launch_unpack_pos(c, st);
}

// kick of step k of a call: kick-drift for the first, else the previous final kick fused in.
// deferred: positions and h stay in pos4 (the state's copies are synced before a list build and
// at the end of the call)
// With adaptive steps (c->adaptive) step j (counted since sph_create, from 1) takes the Courant step
// that the evaluation before it committed to slot (j - 1) % 3.
static int dt_slot(const sph_ctx* c, int64_t j) { return c->adaptive ? (int)(j % 3) : -1; }

static sph_status queue_kick(sph_ctx* c, sph_state* st, double dt, int32_t k, uint32_t check, bool deferred) {
  sph_status e;
  if (!deferred && (e = sync_positions(c, st))) return e;
  timer_begin(c, TIMER_KDK);
  const int64_t j = c->steps_done + k + 1;
  e = k == 0 ? launch_kick_drift(c, st, dt, check, deferred, dt_slot(c, j - 1))
             : launch_kick_final_drift(c, st, dt, check, deferred, dt_slot(c, j - 2), dt_slot(c, j - 1));
  timer_end(c, TIMER_KDK);
  if (!e && deferred) c->pos_deferred = true;
  return e;
}

// density, EoS, stress rate and forces at the drifted positions; seq > 0: a run-ahead evaluation
// of step number seq (cancelled on the device when the skin test of that or an earlier step failed)
// k: the call-local step the evaluation belongs to (its Courant step goes to slot (j % 3))
static sph_status queue_evaluation(sph_ctx* c, sph_state* st, uint32_t seq, int32_t k) {
  c->eval_seq = seq;
  c->eval_in_step = true;
  sph_status e;
  timer_begin(c, TIMER_DENSITY);
  e = launch_density(c, st);
  timer_end(c, TIMER_DENSITY);
  if (!e) {
    timer_begin(c, TIMER_EOS);
    e = launch_eos(c, st);
    timer_end(c, TIMER_EOS);
  }
  if (!e && c->adaptive) e = launch_dt_commit(c, dt_slot(c, c->steps_done + k + 1));
  if (!e) {
    timer_begin(c, TIMER_STRESS);
    e = launch_stress(c, st);
    timer_end(c, TIMER_STRESS);
  }
  if (!e) {
    timer_begin(c, TIMER_FORCES);
    e = launch_forces(c, st);
    timer_end(c, TIMER_FORCES);
  }
  c->eval_seq = 0u;
  c->eval_in_step = false;
  return e;
}

// Steps are chained: the final kick of step k and the kick-drift of step k + 1 run as one
// kernel; the last step of the call ends with its own final kick.
// With valid lists and a positive skin the host queues step k + 1 before it reads the skin test
// of step k back, so the device never waits for the host.  Steps carry their number since the
// test word was cleared: a kick or evaluation behind a failed test finds a smaller number there
// and does nothing; the host then rebuilds the lists, evaluates the failed step again and
// carries on after it.
static sph_status step_loop(sph_ctx* c, sph_state* st, double dt, int32_t nsteps) {
  sph_status e;
  int32_t k = 0;
  while (k < nsteps) {
    if (!(c->lists_valid && c->p.skin > 0.0)) {   // no lists to test: build them for this step
      if ((e = queue_kick(c, st, dt, k, 0u, false)) || (e = rebuild(c, st, true)) ||
          (e = queue_evaluation(c, st, 0u, k)))
        return e;
      ++k;
      continue;
    }
    if ((e = launch_flag_clear(c))) return e;
    const int32_t k0 = k;   // step k0 + q - 1 has number q
    int32_t queued = k;
    while (k < nsteps) {
      while (queued < nsteps && queued <= k + 1) {
        const uint32_t q = (uint32_t)(queued - k0 + 1);
        if ((e = queue_kick(c, st, dt, queued, q, true)) || (e = queue_evaluation(c, st, q, queued))) return e;
        HIP_TRY(hipMemcpyAsync(c->drift_host, c->drift_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipEventRecord(c->step_ev[queued & 1], c->stream));
        ++queued;
      }
      HIP_TRY(hipEventSynchronize(c->step_ev[k & 1]));
      const uint32_t f = *c->drift_host;   // a later step's copy may have landed too: still exact
      if (f == 0u) {
        ++k;
        continue;
      }
      // the drift of step v broke the skin bound; the steps queued after it did nothing
      const int32_t v = k0 + (int32_t)f - 1;
      if ((e = sync_positions(c, st)) || (e = rebuild(c, st, true)) || (e = queue_evaluation(c, st, 0u, v))) return e;
      k = v + 1;
      break;
    }
  }
  return SPH_OK;
}

sph_status sph_step(sph_ctx* c, sph_state* st, double dt, int32_t nsteps) {
  sph_status e = check_state(c, st);
  if (e) return e;
  if (std::isnan(dt) || nsteps < 0) return note(c, SPH_E_ARG, "dt = %g must be a number and nsteps = %d not negative", dt, nsteps);
  const bool adaptive = !(dt > 0.0);
  if (adaptive && c->p.graph) return note(c, SPH_E_ARG, "graph replay needs a fixed dt > 0");
  if (!adaptive && c->p.damping > 0.0 && c->p.damping * dt >= 1.0)
    return note(c, SPH_E_ARG, "damping dt = %g must be below 1 (the kicks treat the drag explicitly)", c->p.damping * dt);
  if (c->gen < 4 || st->n != c->n) return note(c, SPH_E_ORDER, "sph_step needs a full evaluation (build, density, stress rate, forces) of this state first");
  if (st->n == 0) return SPH_OK;
  if (c->p.graph && !c->stream) return note(c, SPH_E_ARG, "graph replay needs a non-default stream");
  if (c->p.graph && c->p.skin > 0.0 && c->lists_valid) {
    e = step_graphs(c, st, dt, nsteps);
    if (!e) {
      c->gen = 4;
      c->steps_done += nsteps;
    }
    return e;
  }
  for (hipEvent_t& ev : c->step_ev)
    if (!ev) HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  c->adaptive = adaptive;
  e = step_loop(c, st, dt, nsteps);
  const sph_status es = sync_positions(c, st);   // also after an error: the state stays whole
  if (!e && !es && nsteps > 0) {
    timer_begin(c, TIMER_KDK);
    e = launch_kick_final(c, st, dt, dt_slot(c, c->steps_done + nsteps - 1));
    timer_end(c, TIMER_KDK);
  }
  c->adaptive = false;
  if (e) return e;
  if (es) return es;
  c->steps_done += nsteps;
  c->gen = 4;
  return SPH_OK;
}


}  // extern "C"

namespace {

// A device copy of a state for the autotuner's trial runs.
struct StateCopy {
  std::vector<void*> bufs;
  sph_state st;
  ~StateCopy() {
    for (void* b : bufs) (void)hipFree(b);
  }
  template <typename T>
  sph_status alloc(T** p, size_t count) {
    if (hipMalloc((void**)p, sizeof(T) * (count ? count : 1)) != hipSuccess) {
      *p = nullptr;
      return SPH_E_OOM;
    }
    bufs.push_back(*p);
    return SPH_OK;
  }
  sph_status make(const sph_state* src) {
    const size_t n = (size_t)src->n;
    st = *src;
    double** d64[] = {&st.x, &st.y, &st.z, &st.vx, &st.vy, &st.vz, &st.u, &st.h, &st.D, &st.rho, &st.P, &st.cs,
                      &st.ax, &st.ay, &st.az, &st.dudt};
    sph_status e;
    for (double** p : d64)
      if ((e = alloc(p, n))) return e;
    if ((e = alloc(&st.S, 6 * n)) || (e = alloc(&st.dSdt, 6 * n)) || (e = alloc(&st.type, n)) ||
        (e = alloc(&st.broken, n)) || (e = alloc(&st.id, n)))
      return e;
    if (src->star && (e = alloc(&st.star, n))) return e;
    return SPH_OK;
  }
  sph_status load(const sph_state* src, hipStream_t s) {
    const size_t n = (size_t)src->n;
    // D and P too: the continuity density and the lagged dP/dt read them as state
    const double* a[] = {src->x, src->y, src->z, src->vx, src->vy, src->vz, src->u, src->h, src->D, src->P};
    double* b[] = {st.x, st.y, st.z, st.vx, st.vy, st.vz, st.u, st.h, st.D, st.P};
    for (int k = 0; k < 10; ++k) HIP_TRY(hipMemcpyAsync(b[k], a[k], 8 * n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(st.S, src->S, 48 * n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(st.type, src->type, n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(st.broken, src->broken, n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(st.id, src->id, 4 * n, hipMemcpyDeviceToDevice, s));
    if (src->star) HIP_TRY(hipMemcpyAsync(st.star, src->star, 4 * n, hipMemcpyDeviceToDevice, s));
    return SPH_OK;
  }
};

}  // namespace

extern "C" {

sph_status sph_autotune(sph_ctx* c, const sph_state* st, double dt, int32_t steps, sph_tune_result* out) {
  sph_status e = check_state(c, st);
  if (e) return e;
  if (!out || !(dt > 0.0) || steps < 1 || st->n == 0)
    return note(c, SPH_E_ARG, "sph_autotune needs out, dt > 0, steps_per_trial >= 1 and n > 0");
  StateCopy cp;
  if ((e = cp.make(st))) return e;
  const int32_t timing = c->timing;
  c->timing = 0;
  auto trial = [&](const sph_params& p, double* ms) -> sph_status {
    c->p = p;
    c->lists_valid = false;
    c->gen = 0;
    ++c->graph_epoch;
    sph_status te;
    if ((te = cp.load(st, c->stream)) || (te = sph_build_cells(c, &cp.st)) || (te = sph_density(c, &cp.st)) ||
        (te = sph_stress_rate(c, &cp.st)) || (te = sph_forces(c, &cp.st)) || (te = sph_step(c, &cp.st, dt, 1)))
      return te;
    // timed: one call of `steps` chained steps, with the list rebuilds they need (as in a run)
    HIP_TRY(hipStreamSynchronize(c->stream));
    const auto t0 = std::chrono::steady_clock::now();
    if ((te = sph_step(c, &cp.st, dt, steps))) return te;
    HIP_TRY(hipStreamSynchronize(c->stream));
    const auto t1 = std::chrono::steady_clock::now();
    *ms = std::chrono::duration<double, std::milli>(t1 - t0).count() / steps;
    return sph_sync(c);
  };
  sph_params best = c->p;
  best.tile_cut = tile_cut_of(best);
  if (best.lanes <= 0) best.lanes = pass_lanes(best);
  double best_ms = 0.0;
  int32_t trials = 1;
  if ((e = trial(best, &best_ms))) {
    c->timing = timing;
    return e;
  }
  const double start_ms = best_ms;
  // coordinate descent: lanes per target, workgroup schedule of the pair passes, tile cut, skin;
  // a setting replaces the best only if it is faster by more than the timing noise (2%)
  for (int dim = 0; dim < 4 && !e; ++dim) {
    const double vals[4][4] = {{1, 2, 4, -1}, {0, 1024, 4096, 16384}, {6, 8, 10, 12}, {0.07, 0.1, 0.14, 0.18}};
    const sph_params base = best;
    for (int k = 0; k < 4 && !e; ++k) {
      const double v = vals[dim][k];
      if (v < 0) continue;
      sph_params p = base;
      if (dim == 0) {
        if ((int32_t)v == base.lanes) continue;
        p.lanes = (int32_t)v;
      } else if (dim == 1) {
        if ((int32_t)v == base.pass_blocks) continue;
        p.pass_blocks = (int32_t)v;
      } else if (dim == 2) {
        if (v == base.tile_cut) continue;
        p.tile_cut = v;
      } else {
        if (v == base.skin || base.skin == 0.0) continue;
        p.skin = v;
      }
      double ms;
      e = trial(p, &ms);
      ++trials;
      if (!e && ms < 0.98 * best_ms) {
        best_ms = ms;
        best = p;
      }
    }
  }
  c->timing = timing;
  c->p = best;
  c->lists_valid = false;
  c->gen = 0;
  ++c->graph_epoch;
  if (e) return e;
  out->pass_blocks = best.pass_blocks;
  out->lanes = best.lanes;
  out->pad = 0;
  out->tile_cut = best.tile_cut;
  out->skin = best.skin;
  out->trials = trials;
  out->ms_per_step = best_ms;
  out->ms_per_step_start = start_ms;
  return SPH_OK;
}

sph_status sph_ensemble_set(sph_ctx* c, int32_t nstars, const double* star_info) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (nstars < 0 || (nstars > 0 && !star_info)) return note(c, SPH_E_ARG, "nstars = %d needs star_info", nstars);
  std::vector<StarInfo> h((size_t)nstars);
  for (int32_t s = 0; s < nstars; ++s) {
    const double* q = star_info + 5 * (int64_t)s;
    if (!(q[3] > 0.0) || !(q[4] >= 0.0))
      return note(c, SPH_E_ARG, "star %d: particle mass must be positive and shear factor not negative", s);
    h[s] = StarInfo{q[0], q[1], q[2], q[3], q[4], {0.0, 0.0, 0.0}};
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->stars) (void)hipFree(c->stars);
  c->stars = nullptr;
  c->nstars = 0;
  if (nstars > 0) {
    if (hipMalloc((void**)&c->stars, sizeof(StarInfo) * nstars) != hipSuccess) {
      c->stars = nullptr;
      return SPH_E_OOM;
    }
    HIP_TRY(hipMemcpy(c->stars, h.data(), sizeof(StarInfo) * nstars, hipMemcpyHostToDevice));
    c->nstars = nstars;
  }
  c->gen = 0;
  ++c->graph_epoch;
  return SPH_OK;
}

int32_t sph_error_particle(const sph_ctx* c) { return c ? c->err_particle : -1; }

sph_status sph_sync(sph_ctx* c) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  hipError_t he = hipStreamSynchronize(c->stream);
  if (he != hipSuccess) return note(c, SPH_E_HIP, "waiting for the stream: %s", hipGetErrorString(he));
  DevStatus s;
  if ((he = hipMemcpy(&s, c->status, sizeof(s), hipMemcpyDeviceToHost)) != hipSuccess)
    return note(c, SPH_E_HIP, "reading the status word: %s", hipGetErrorString(he));
  if (s.code) {
    c->err_particle = s.particle;
    DevStatus z = {0, 0};
    if ((he = hipMemcpy(c->status, &z, sizeof(z), hipMemcpyHostToDevice)) != hipSuccess)
      return note(c, SPH_E_HIP, "clearing the status word: %s", hipGetErrorString(he));
    static const char* why[8] = {"", "a periodic box too small for one image per pair (2h >= box/2)", "",
                                 "", "", "a neighbour list exceeded its capacity (exact: max_neighbours, candidate: twice that)",
                                 "a field became NaN or Inf", "(rho, u) outside the tabulated equation of state"};
    const char* w = (s.code > 0 && s.code < 8) ? why[s.code] : "";
    if (s.particle >= 0)
      return note(c, (sph_status)s.code, "latched on the device by particle %d (index in the current order): %s",
                  s.particle, w);
    return note(c, (sph_status)s.code, "latched on the device by a tile: %s", w);
  }
  return SPH_OK;
}

const char* sph_last_error_detail(const sph_ctx* c) { return c ? c->detail : g_detail; }

sph_status sph_get_time(sph_ctx* c, double* t) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (!t) return note(c, SPH_E_ARG, "t is NULL");
  hipError_t he = hipStreamSynchronize(c->stream);
  if (he == hipSuccess) he = hipMemcpy(t, c->dtw + 3, sizeof(double), hipMemcpyDeviceToHost);
  if (he != hipSuccess) return note(c, SPH_E_HIP, "reading the simulated time: %s", hipGetErrorString(he));
  return SPH_OK;
}

sph_status sph_modify_energy(sph_ctx* c, sph_state* st, const double* u_of_r, int32_t nr, double dr) {
  sph_status e = check_state(c, st);
  if (e) return e;
  if (!u_of_r || nr < 2 || !(dr > 0.0)) return note(c, SPH_E_ARG, "u_of_r (device) needs nr >= 2 and dr > 0");
  if (st->n == 0) return SPH_OK;
  if ((e = sync_positions(c, st))) return e;
  if ((e = launch_modify_energy(c, st, u_of_r, nr, dr))) return e;
  if (c->gen > 1) c->gen = 1;   // u changed: the evaluation starts again at the density pass
  return SPH_OK;
}

sph_status sph_eos_table_create(sph_ctx* c, const double* lnP, const double* lncs2, int32_t nr, int32_t nu,
                                double lnr0, double dlnr, double lnu0, double dlnu) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (!lnP || !lncs2) return note(c, SPH_E_ARG, "lnP and lncs2 (host arrays) must not be NULL");
  if (nr < 2 || nu < 2 || (int64_t)nr * nu > (int64_t(1) << 28))
    return note(c, SPH_E_ARG, "table size %d x %d outside [2, 2^28 nodes]", nr, nu);
  if (!(dlnr > 0.0) || !(dlnu > 0.0) || !std::isfinite(lnr0) || !std::isfinite(lnu0))
    return note(c, SPH_E_ARG, "table spacing must be positive and origins finite");
  const size_t nn = (size_t)nr * nu;
  hipError_t he = hipStreamSynchronize(c->stream);
  if (he != hipSuccess) return note(c, SPH_E_HIP, "waiting for the stream: %s", hipGetErrorString(he));
  double* t = nullptr;
  if (hipMalloc((void**)&t, sizeof(double) * 2 * nn) != hipSuccess) return note(c, SPH_E_OOM, "table of %zu nodes", nn);
  if ((he = hipMemcpy(t, lnP, sizeof(double) * nn, hipMemcpyHostToDevice)) != hipSuccess ||
      (he = hipMemcpy(t + nn, lncs2, sizeof(double) * nn, hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(t);
    return note(c, SPH_E_HIP, "uploading the table: %s", hipGetErrorString(he));
  }
  if (c->tab_own) (void)hipFree(c->tab_own);
  c->tab_own = t;
  c->tab_own_nr = nr;
  c->tab_own_nu = nu;
  c->tab_own_g[0] = lnr0;
  c->tab_own_g[1] = dlnr;
  c->tab_own_g[2] = lnu0;
  c->tab_own_g[3] = dlnu;
  c->p.tab_lnP = nullptr;
  use_own_table(c, &c->p);
  mlp_free(c);   // a network belongs to the table it was fitted to
  c->gen = 0;
  ++c->graph_epoch;
  return SPH_OK;
}

sph_status sph_export_neighbours(sph_ctx* c, int64_t* offsets, int32_t* ids, int64_t cap) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (!offsets) return note(c, SPH_E_ARG, "offsets is NULL");
  if (c->n > 0 && (c->gen < 2 || !c->lists_valid)) return SPH_E_ORDER;
  const int64_t n = c->n;
  if (n > 0 && !exact_lists_written(c)) {
    sph_status e = launch_exact_lists(c);
    if (e) return e;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SPH_E_HIP;
  if (n == 0) { offsets[0] = 0; return SPH_OK; }
  GridInfo g;
  if (hipMemcpy(&g, c->grid, sizeof(g), hipMemcpyDeviceToHost) != hipSuccess) return SPH_E_HIP;
  const int64_t ntiles = g.ntiles;
  std::vector<int32_t> cnt(n), tst(ntiles), tcn(ntiles);
  std::vector<uint32_t> uoff(ntiles);
  std::vector<int32_t> U((size_t)(g.upool_used < c->upool ? g.upool_used : c->upool));
  const int L = pass_lanes(c->p);
  std::vector<uint16_t> raw((size_t)slot_capacity(c->cap, L) * c->capw * L);
  std::vector<int32_t> cnt_sl((size_t)n * L);
  if (hipMemcpy(cnt.data(), c->nbr_count, sizeof(int32_t) * n, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(cnt_sl.data(), c->nbr_count_sl, sizeof(int32_t) * n * L, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(tst.data(), c->tile_start, sizeof(int32_t) * ntiles, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(tcn.data(), c->tile_cnt, sizeof(int32_t) * ntiles, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(uoff.data(), c->tile_uoff, sizeof(uint32_t) * ntiles, hipMemcpyDeviceToHost) != hipSuccess ||
      (U.size() && hipMemcpy(U.data(), c->tile_u, sizeof(int32_t) * U.size(), hipMemcpyDeviceToHost) != hipSuccess) ||
      hipMemcpy(raw.data(), c->nbr16, sizeof(uint16_t) * raw.size(), hipMemcpyDeviceToHost) != hipSuccess)
    return SPH_E_HIP;
  offsets[0] = 0;
  for (int64_t a = 0; a < n; ++a) offsets[a + 1] = offsets[a] + cnt[a];
  if (offsets[n] > cap || !ids) return SPH_E_NGB_CAPACITY;
  std::vector<uint16_t> loc;
  for (int64_t t = 0; t < ntiles; ++t)
    for (int l = 0; l < tcn[t]; ++l) {
      const int64_t a = (int64_t)tst[t] + l;
      loc.clear();   // the particle's slot lists, merged in ascending local index
      for (int j = 0; j < L; ++j) {
        const int64_t s = a * L + j;
        for (int k = 0; k < cnt_sl[(size_t)s]; ++k) loc.push_back(raw[(size_t)nbr_index(k, s, c->capw * L)]);
      }
      std::sort(loc.begin(), loc.end());
      if ((int64_t)loc.size() != cnt[a]) return SPH_E_NGB_CAPACITY;   // lists of an overflowed evaluation
      for (size_t k = 0; k < loc.size(); ++k) ids[offsets[a] + (int64_t)k] = U[(size_t)uoff[t] + loc[k]];
    }
  return SPH_OK;
}

sph_status sph_neighbour_stats(sph_ctx* c, sph_list_stats* out) {
  if (!c || !out) return SPH_E_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SPH_E_HIP;
  return sph_count_stats(c, out);
}

sph_status sph_set_timing(sph_ctx* c, int32_t enable) {
  if (!c) return SPH_E_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SPH_E_HIP;
  c->timing = enable;
  for (auto& t : c->timers) t.used = 0;
  return SPH_OK;
}

sph_status sph_get_timing(sph_ctx* c, const char* stage, int32_t* launches, double* ms) {
  if (!c || !stage || !launches || !ms) return SPH_E_ARG;
  static const char* names[6] = {"cells", "density", "stress", "forces", "kdk", "eos"};
  int which = -1;
  for (int k = 0; k < 6; ++k)
    if (!strcmp(stage, names[k])) which = k;
  if (which < 0) return SPH_E_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SPH_E_HIP;
  StageTimer& t = c->timers[which];
  double tot = 0.0;
  for (size_t i = 0; i + 1 < t.used; i += 2) {
    float f = 0.f;
    if (hipEventElapsedTime(&f, t.ev[i], t.ev[i + 1]) != hipSuccess) return SPH_E_HIP;
    tot += f;
  }
  *launches = (int32_t)(t.used / 2);
  *ms = tot;
  return SPH_OK;
}

}  // extern "C"
