// C-ABI entry points of libsph: context, stage calls, time stepping, status and timing.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sph_internal.h"

namespace {

constexpr int64_t kMaxCells = int64_t(1) << 25;

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

sph_status check_params(const sph_params* p) {
  if (!p) return SPH_E_ARG;
  if (p->kernel != SPH_WC2 && p->kernel != SPH_WC4) return SPH_E_ARG;
  if (!(p->m > 0.0)) return SPH_E_ARG;
  if (p->background == SPH_TOV && (!p->bg || p->bg_n < 2 || !(p->bg_dr > 0.0))) return SPH_E_ARG;
  if (p->periodic && !(p->box > 0.0)) return SPH_E_ARG;
  if ((p->eos == SPH_EOS_TABLE || p->eos == SPH_EOS_MLP) &&
      (!p->tab_lnP || !p->tab_lncs2 || p->tab_nr < 2 || p->tab_nu < 2))
    return SPH_E_ARG;
  if (p->precision != SPH_FP64 && p->precision != SPH_FP32) return SPH_E_ARG;
  if (p->max_neighbours < 0 || p->max_neighbours > 4096) return SPH_E_ARG;
  if (p->cell_div < 0 || p->cell_div > 4) return SPH_E_ARG;
  return SPH_OK;
}

sph_status check_state(const sph_ctx* c, const sph_state* st) {
  if (!c || !st) return SPH_E_ARG;
  if (st->n < 0 || st->n > c->capacity) return SPH_E_ARG;
  if (st->n > 0 && (!st->x || !st->y || !st->z || !st->vx || !st->vy || !st->vz || !st->u || !st->h ||
                    !st->S || !st->type || !st->broken || !st->id || !st->D || !st->rho || !st->P ||
                    !st->cs || !st->ax || !st->ay || !st->az || !st->dudt || !st->dSdt))
    return SPH_E_ARG;
  if (c->stars && st->n > 0 && !st->star) return SPH_E_ARG;
  return SPH_OK;
}

}  // namespace

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
  void* bufs[] = {c->grid, c->keys, c->vals, c->cell_start, c->cell_end, c->sort.keys_alt, c->sort.vals_alt,
                  c->sort.hist, c->sort.rowtot, c->sort.partial, c->sort.scan_bsum, c->tile_start, c->tile_cnt, c->tile_flag, c->tile_u, c->tile_uoff,
                  c->tile_usize, c->nbr16, c->nbr_count, c->pos4, c->fv, c->fa, c->sig, c->pos4f, c->fvf,
                  c->faf, c->sigf, c->mu, c->Y0, c->B, c->sdot, c->half, c->tmp, c->stars, c->status};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (auto& t : c->timers)
    for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
  c->~sph_ctx();
  free(c);
}

sph_status sph_create(const sph_params* params, void* stream, int64_t capacity, sph_ctx** out) {
  if (!out) return SPH_E_ARG;
  *out = nullptr;
  sph_status e = check_params(params);
  if (e) return e;
  if (capacity < 1 || capacity > (int64_t(1) << 30)) return SPH_E_ARG;
  sph_ctx* c = (sph_ctx*)calloc(1, sizeof(sph_ctx));
  if (!c) return SPH_E_OOM;
  new (c) sph_ctx();
  c->p = *params;
  c->stream = (hipStream_t)stream;
  c->capacity = capacity;
  c->cap = params->max_neighbours > 0 ? params->max_neighbours : 512;
  c->ucap = 8192;   // union members per tile; local indices are 16-bit
  c->upool = (int64_t)((capacity + 63) / 64 * 64) * c->cap;
  if (c->upool > (int64_t)0xffffffffll) {   // pool offsets are 32-bit: lower max_neighbours
    c->~sph_ctx();
    free(c);
    return SPH_E_ARG;
  }
  (void)hipGetDevice(&c->device);
  const int64_t cap = capacity;
  const int64_t capw = (cap + 63) / 64 * 64;
  c->capw = capw;
  // every tile holds at least one particle, so capw tiles always suffice; the union pool holds
  // up to cap entries per particle (the worst case of one particle per tile), capped by 32-bit
  // offsets
  c->cap_tiles = capw;
  c->sort.scan_cap = (capw + 1023) / 1024;
  c->max_cells = kMaxCells;
  c->sort.max_blocks = (int)((cap + 4095) / 4096);
  if ((e = dalloc(&c->grid, 1)) || (e = dalloc(&c->keys, cap)) || (e = dalloc(&c->vals, cap)) ||
      (e = dalloc(&c->cell_start, c->max_cells)) || (e = dalloc(&c->cell_end, c->max_cells)) ||
      (e = dalloc(&c->sort.keys_alt, cap)) || (e = dalloc(&c->sort.vals_alt, cap)) ||
      (e = dalloc(&c->sort.hist, (size_t)256 * c->sort.max_blocks)) || (e = dalloc(&c->sort.rowtot, 256)) ||
      (e = dalloc(&c->sort.partial, (size_t)8 * 1024)) ||
      (e = dalloc(&c->tile_u, (size_t)c->upool)) || (e = dalloc(&c->tile_uoff, c->cap_tiles)) ||
      (e = dalloc(&c->tile_usize, c->cap_tiles)) ||
      (e = dalloc(&c->tile_start, c->cap_tiles)) || (e = dalloc(&c->tile_cnt, c->cap_tiles)) ||
      (e = dalloc(&c->tile_flag, capw)) || (e = dalloc(&c->sort.scan_bsum, c->sort.scan_cap + 1)) ||
      (e = dalloc(&c->nbr16, (size_t)capw * c->cap)) || (e = dalloc(&c->nbr_count, capw)) ||
      (e = dalloc(&c->pos4, cap)) || (e = dalloc(&c->fv, cap)) || (e = dalloc(&c->fa, cap)) ||
      (e = dalloc(&c->sig, 6 * cap)) || (e = dalloc(&c->pos4f, cap)) || (e = dalloc(&c->fvf, cap)) ||
      (e = dalloc(&c->faf, cap)) || (e = dalloc(&c->sigf, 6 * cap)) || (e = dalloc(&c->mu, cap)) ||
      (e = dalloc(&c->Y0, cap)) || (e = dalloc(&c->B, cap)) || (e = dalloc(&c->sdot, cap)) ||
      (e = dalloc(&c->half, 10 * cap)) || (e = dalloc(&c->tmp, cap)) || (e = dalloc(&c->status, 1))) {
    sph_destroy(c);
    return e;
  }
  // cell tables are validated against the sorted keys on every lookup, so they are cleared once
  if (hipMemsetAsync(c->cell_start, 0xff, sizeof(int32_t) * c->max_cells, c->stream) != hipSuccess ||
      hipMemsetAsync(c->cell_end, 0xff, sizeof(int32_t) * c->max_cells, c->stream) != hipSuccess ||
      hipMemsetAsync(c->status, 0, sizeof(DevStatus), c->stream) != hipSuccess ||
      hipMemsetAsync(c->nbr_count, 0, sizeof(int32_t) * cap, c->stream) != hipSuccess ||
      hipMemsetAsync(c->Y0, 0, sizeof(double) * cap, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    sph_destroy(c);
    return SPH_E_HIP;
  }
  *out = c;
  return SPH_OK;
}

sph_status sph_set_params(sph_ctx* c, const sph_params* params) {
  if (!c) return SPH_E_ARG;
  sph_status e = check_params(params);
  if (e) return e;
  int cap = params->max_neighbours > 0 ? params->max_neighbours : 512;
  if (cap != c->cap) return SPH_E_ARG;   // list capacity is fixed at creation
  c->p = *params;
  c->gen = 0;
  return SPH_OK;
}

sph_status sph_build_cells(sph_ctx* c, sph_state* st) {
  sph_status e = check_state(c, st);
  if (e) return e;
  c->n = st->n;
  if (st->n == 0) { c->gen = 1; return SPH_OK; }
  timer_begin(c, TIMER_CELLS);
  e = sph_rebin(c, st, true);
  timer_end(c, TIMER_CELLS);
  if (e) return e;
  c->steps_since_sort = 0;
  c->gen = 1;
  return SPH_OK;
}

sph_status sph_density(sph_ctx* c, sph_state* st) {
  sph_status e = check_state(c, st);
  if (e) return e;
  if (c->gen < 1 || st->n != c->n) return SPH_E_ORDER;
  if (st->n > 0) {
    timer_begin(c, TIMER_DENSITY);
    e = launch_density(c, st);
    timer_end(c, TIMER_DENSITY);
    if (e) return e;
  }
  c->gen = 2;
  return SPH_OK;
}

sph_status sph_stress_rate(sph_ctx* c, sph_state* st) {
  sph_status e = check_state(c, st);
  if (e) return e;
  if (c->gen < 2 || st->n != c->n) return SPH_E_ORDER;
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
  if (c->gen < 3 || st->n != c->n) return SPH_E_ORDER;
  if (st->n > 0) {
    timer_begin(c, TIMER_FORCES);
    e = launch_forces(c, st);
    timer_end(c, TIMER_FORCES);
    if (e) return e;
  }
  c->gen = 4;
  return SPH_OK;
}

sph_status sph_step(sph_ctx* c, sph_state* st, double dt, int32_t nsteps) {
  sph_status e = check_state(c, st);
  if (e) return e;
  if (!(dt > 0.0) || nsteps < 0) return SPH_E_ARG;
  if (c->gen < 4 || st->n != c->n) return SPH_E_ORDER;
  if (st->n == 0) return SPH_OK;
  const int every = c->p.resort_every > 0 ? c->p.resort_every : 10;
  for (int32_t k = 0; k < nsteps; ++k) {
    timer_begin(c, TIMER_KDK);
    if ((e = launch_kick_drift(c, st, dt))) return e;
    timer_end(c, TIMER_KDK);
    bool resort = ++c->steps_since_sort >= every;
    timer_begin(c, TIMER_CELLS);
    e = sph_rebin(c, st, resort);
    timer_end(c, TIMER_CELLS);
    if (e) return e;
    if (resort) c->steps_since_sort = 0;
    timer_begin(c, TIMER_DENSITY);
    if ((e = launch_density(c, st))) return e;
    timer_end(c, TIMER_DENSITY);
    timer_begin(c, TIMER_STRESS);
    if ((e = launch_stress(c, st))) return e;
    timer_end(c, TIMER_STRESS);
    timer_begin(c, TIMER_FORCES);
    if ((e = launch_forces(c, st))) return e;
    timer_end(c, TIMER_FORCES);
    timer_begin(c, TIMER_KDK);
    if ((e = launch_kick_final(c, st, dt))) return e;
    timer_end(c, TIMER_KDK);
  }
  c->gen = 4;
  return SPH_OK;
}

sph_status sph_sync(sph_ctx* c) {
  if (!c) return SPH_E_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SPH_E_HIP;
  DevStatus s;
  if (hipMemcpy(&s, c->status, sizeof(s), hipMemcpyDeviceToHost) != hipSuccess) return SPH_E_HIP;
  if (s.code) {
    DevStatus z = {0, 0};
    if (hipMemcpy(c->status, &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess) return SPH_E_HIP;
    return (sph_status)s.code;
  }
  return SPH_OK;
}

sph_status sph_export_neighbours(sph_ctx* c, int64_t* offsets, int32_t* ids, int64_t cap) {
  if (!c || !offsets) return SPH_E_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SPH_E_HIP;
  const int64_t n = c->n;
  if (n == 0) { offsets[0] = 0; return SPH_OK; }
  GridInfo g;
  if (hipMemcpy(&g, c->grid, sizeof(g), hipMemcpyDeviceToHost) != hipSuccess) return SPH_E_HIP;
  const int64_t ntiles = (int64_t)g.ntiles < c->cap_tiles ? (int64_t)g.ntiles : c->cap_tiles;
  std::vector<int32_t> cnt(n), usz(ntiles), tst(ntiles), tcn(ntiles);
  std::vector<uint32_t> uoff(ntiles);
  std::vector<int32_t> U((size_t)(g.upool_used < c->upool ? g.upool_used : c->upool));
  std::vector<uint32_t> perm(n);
  std::vector<uint16_t> raw((size_t)c->cap * c->capw);
  if (hipMemcpy(cnt.data(), c->nbr_count, sizeof(int32_t) * n, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(usz.data(), c->tile_usize, sizeof(int32_t) * ntiles, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(tst.data(), c->tile_start, sizeof(int32_t) * ntiles, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(tcn.data(), c->tile_cnt, sizeof(int32_t) * ntiles, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(uoff.data(), c->tile_uoff, sizeof(uint32_t) * ntiles, hipMemcpyDeviceToHost) != hipSuccess ||
      (U.size() && hipMemcpy(U.data(), c->tile_u, sizeof(int32_t) * U.size(), hipMemcpyDeviceToHost) != hipSuccess) ||
      hipMemcpy(perm.data(), c->vals, sizeof(uint32_t) * n, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(raw.data(), c->nbr16, sizeof(uint16_t) * raw.size(), hipMemcpyDeviceToHost) != hipSuccess)
    return SPH_E_HIP;
  std::vector<int32_t> cnt_a(n, 0);
  for (int64_t p = 0; p < n; ++p) cnt_a[c->identity_perm ? p : perm[p]] = cnt[p];
  offsets[0] = 0;
  for (int64_t a = 0; a < n; ++a) offsets[a + 1] = offsets[a] + cnt_a[a];
  if (offsets[n] > cap || !ids) return SPH_E_NGB_CAPACITY;
  for (int64_t t = 0; t < ntiles; ++t)
    for (int l = 0; l < tcn[t]; ++l) {
      const int64_t p = (int64_t)tst[t] + l;
      const int64_t a = c->identity_perm ? p : perm[p];
      for (int k = 0; k < cnt[p]; ++k) {
        const uint16_t loc = raw[(size_t)k * c->capw + p];
        ids[offsets[a] + k] = U[(size_t)uoff[t] + loc];
      }
    }
  return SPH_OK;
}

sph_status sph_neighbour_stats(sph_ctx* c, int64_t* total_pairs, int32_t* max_count) {
  if (!c || !total_pairs || !max_count) return SPH_E_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SPH_E_HIP;
  return sph_count_stats(c, total_pairs, max_count);
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
  static const char* names[5] = {"cells", "density", "stress", "forces", "kdk"};
  int which = -1;
  for (int k = 0; k < 5; ++k)
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
