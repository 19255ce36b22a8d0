// C ABI entry points: parameter checks, workspace carving, step bookkeeping.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "lbmd_internal.hpp"

using namespace lbmd_impl;

struct lbmd : Context {};

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t a) { return (a + kAlign - 1) / kAlign * kAlign; }

bool valid(const lbmd_params* p) {
  if (!p) return false;
  if (p->nx < 2 || p->ny < 2 || p->nz < 2) return false;
  const int64_t S = (int64_t)p->nx * p->ny * p->nz;
  if (S > (int64_t)0x7FFFFFFF - 64) return false;
  if (p->n_sub < 1) return false;
  if (p->variant != 1 && p->variant != 2) return false;
  if (p->precision != 32 && p->precision != 64) return false;
  if (p->n_particles < 0) return false;
  if (!(p->rho0 > 0.0) || !(p->nu > 0.0) || !(p->kT >= 0.0) || !(p->friction >= 0.0)) return false;
  if (!(p->nu_bulk < 0.0 || p->nu_bulk > 0.0)) return false;
  if (!(fabs(p->gamma_ghost) < 1.0)) return false;
  if (p->n_particles > 0 && !(p->particle_mass > 0.0)) return false;
  if (p->force_model < 0 || p->force_model > 2) return false;
  if (p->force_model == 2) {
    if (p->chain_len < 1 || (p->n_particles % p->chain_len) != 0) return false;
    if (!(p->wca_sigma > 0.0) || !(p->wca_eps >= 0.0) || !(p->k_bond >= 0.0)) return false;
    if (!isfinite(p->r0_bond)) return false;
  }
  for (int d = 0; d < 3; ++d)
    if (!isfinite(p->body_force[d]) || !isfinite(p->f_ext[d])) return false;
  return true;
}

Layout layout(const lbmd_params* p) {
  Layout L;
  const size_t S = (size_t)p->nx * p->ny * p->nz;
  const size_t N = (size_t)std::max(p->n_particles, 1);
  const size_t t = p->precision == 32 ? 4 : 8;
  size_t o = 0;
  L.pop[0] = o; o = up(o + 19 * S * t);
  L.pop[1] = o; o = up(o + 19 * S * t);
  L.transfer = o; o = up(o + 4 * S * t);
  L.mark = o; o = up(o + ((S + 63) / 64) * 8);
  L.fcons = o; o = up(o + 3 * N * 8);
  L.rec_cell = o; o = up(o + 3 * N * 4);
  L.rec_frac = o; o = up(o + 3 * N * 8);
  L.rec_dp = o; o = up(o + 3 * N * 8);
  L.cc = o; o = up(o + 32 * N * t);
  L.cc_cell = o; o = up(o + N * 4);
  L.cc_stamp = o; o = up(o + N * 4);
  L.fc_held = o; o = up(o + 3 * N * 8);
  const size_t ncell = (size_t)std::max<int64_t>(force_cells(p), 1);
  L.bin_count = o; o = up(o + ncell * 4);
  L.bin_start = o; o = up(o + (ncell + 1) * 4);
  L.bin_tiles = o; o = up(o + ((ncell + 1023) / 1024 + 1) * 4);
  L.bin_of = o; o = up(o + N * 4);
  L.bin_rank = o; o = up(o + N * 4);
  L.bin_sorted = o; o = up(o + N * 4);
  L.flags = o; o = up(o + 16 * 4);
  L.partials = o; o = up(o + (size_t)kRedBlocks * kRedWidth * 8);
  L.totals = o; o = up(o + kRedWidth * 8);
  L.total = o;
  return L;
}

// Mode norms b_k of the D3Q19 basis, k = 4..18 (stress, then kinetic modes).
const double kNorm[15] = {2.0 / 3, 4.0 / 3, 4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 2.0 / 3, 2.0 / 3,
                          2.0 / 3, 2.0 / 9, 2.0 / 9, 2.0 / 9, 2.0,     4.0 / 3, 4.0 / 9};

void derive(Context* c) {
  const lbmd_params& p = c->p;
  c->gs = (6.0 * p.nu - 1.0) / (6.0 * p.nu + 1.0);
  c->gb = p.nu_bulk < 0.0 ? c->gs : (9.0 * p.nu_bulk - 1.0) / (9.0 * p.nu_bulk + 1.0);
  c->gg = p.gamma_ghost;
  c->mu = 3.0 * p.kT;
  for (int v = 0; v < 15; ++v) {
    const int k = v + 4;
    const double g = k == 4 ? c->gb : (k <= 9 ? c->gs : c->gg);
    c->ns[v] = sqrt(kNorm[v] * (1.0 - g * g)) * sqrt(12.0) / 65536.0;
  }
  c->geom.nx = p.nx;
  c->geom.ny = p.ny;
  c->geom.nz = p.nz;
  c->geom.S = (int)c->S;
  c->geom.inv_nx = 1.0 / p.nx;
  c->geom.inv_ny = 1.0 / p.ny;
}

int fail(Context* c, hipError_t e) {
  if (e == hipSuccess) return LBMD_OK;
  c->sticky = LBMD_EHIP;
  return LBMD_EHIP;
}

}  // namespace

extern "C" {

size_t lbmd_workspace_bytes(const lbmd_params* p) {
  if (!valid(p)) return 0;
  return layout(p).total;
}

int lb_create(const lbmd_params* p, void* d_ws, size_t ws_bytes, void* hip_stream, lbmd** out) {
  if (!out) return LBMD_EINVAL;
  *out = nullptr;
  if (!valid(p) || !d_ws || ((uintptr_t)d_ws % kAlign) != 0) return LBMD_EINVAL;
  const Layout L = layout(p);
  if (ws_bytes < L.total) return LBMD_ENOSPACE;
  lbmd* c = new (std::nothrow) lbmd();
  if (!c) return LBMD_EINVAL;
  c->p = *p;
  c->lay = L;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)d_ws;
  c->S = (int64_t)p->nx * p->ny * p->nz;
  c->cur = 0;
  c->x = c->v = nullptr;
  c->img = nullptr;
  c->bound = false;
  c->t_lb = c->t_md = 0;
  c->subs = 0;
  c->sticky = LBMD_OK;
  derive(c);
  // fluid at rest (all deviations zero), nothing transferred yet
  hipError_t e = hipMemsetAsync(c->ws, 0, L.total, c->stream);
  if (e != hipSuccess) {
    delete c;
    return LBMD_EHIP;
  }
  *out = c;
  return LBMD_OK;
}

int lb_destroy(lbmd* c) {
  delete c;
  return LBMD_OK;
}

int lbmd_bind_particles(lbmd* c, void* d_x, void* d_v, int32_t* d_img) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->p.n_particles > 0 && (!d_x || !d_v || !d_img)) return LBMD_EINVAL;
  c->x = d_x;
  c->v = d_v;
  c->img = d_img;
  c->bound = c->p.n_particles > 0;
  return fail(c, launch_init_forces(c));
}

int md_couple_substep(lbmd* c) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->subs >= c->p.n_sub) return LBMD_ESTATE;
  if (c->p.n_particles > 0 && !c->bound) return LBMD_ESTATE;
  int rc = fail(c, launch_couple(c));
  if (rc) return rc;
  if (c->p.force_model == 2 && c->p.n_particles > 0) {
    rc = fail(c, launch_forces_and_kick(c));
    if (rc) return rc;
  }
  c->t_md += 1;
  c->subs += 1;
  return LBMD_OK;
}

int lb_step(lbmd* c) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->p.n_particles > 0 && c->subs != c->p.n_sub) return LBMD_ESTATE;
  const int rc = fail(c, launch_collide_stream(c));
  if (rc) return rc;
  c->cur = 1 - c->cur;
  c->t_lb += 1;
  c->subs = 0;
  return LBMD_OK;
}

int lb_moments(lbmd* c, void* d_rho, void* d_u, double* h_totals) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  double* d_tot = h_totals ? (double*)at(c, c->lay.totals) : nullptr;
  int rc = fail(c, launch_moments(c, d_rho, d_u, d_tot));
  if (rc || !h_totals) return rc;
  double tot[kRedWidth];
  int32_t flags[16];
  rc = fail(c, hipMemcpyAsync(tot, d_tot, sizeof(tot), hipMemcpyDeviceToHost, c->stream));
  if (rc) return rc;
  rc = fail(c, hipMemcpyAsync(flags, at(c, c->lay.flags), sizeof(flags), hipMemcpyDeviceToHost,
                              c->stream));
  if (rc) return rc;
  rc = fail(c, hipStreamSynchronize(c->stream));
  if (rc) return rc;
  const double m = c->p.particle_mass;
  h_totals[LBMD_TOT_MASS] = c->p.rho0 * (double)c->S + tot[0];
  for (int d = 0; d < 3; ++d) {
    h_totals[LBMD_TOT_PFLUID + d] = tot[1 + d] + tot[4 + d];
    h_totals[LBMD_TOT_PSEEN + d] = tot[1 + d] + (c->p.variant == 2 ? tot[4 + d] : 0.0);
    h_totals[LBMD_TOT_PPART + d] = m * tot[8 + d];
  }
  h_totals[LBMD_TOT_KEPART] = 0.5 * m * tot[11];
  h_totals[LBMD_TOT_U2FLUID] = tot[7] / (double)c->S;
  h_totals[LBMD_TOT_TLB] = (double)c->t_lb;
  h_totals[LBMD_TOT_TMD] = (double)c->t_md;
  return flags[0] ? LBMD_ENONFINITE : LBMD_OK;
}

int lbmd_get_populations(lbmd* c, void* d_dst) {
  if (!c || !d_dst) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  return fail(c, launch_get_populations(c, d_dst));
}

int lbmd_set_populations(lbmd* c, const void* d_src) {
  if (!c || !d_src) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  const int rc = fail(c, launch_set_populations(c, d_src));
  if (rc) return rc;
  return fail(c, invalidate_corner_cache(c));
}

int lbmd_get_transfer(lbmd* c, void* d_dst) {
  if (!c || !d_dst) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  return fail(c, launch_get_transfer(c, d_dst));
}

int lbmd_get_counters(lbmd* c, int64_t* t_lb, int64_t* t_md, int32_t* subs) {
  if (!c) return LBMD_EINVAL;
  if (t_lb) *t_lb = c->t_lb;
  if (t_md) *t_md = c->t_md;
  if (subs) *subs = c->subs;
  return LBMD_OK;
}

int lbmd_set_counters(lbmd* c, int64_t t_lb, int64_t t_md, int32_t subs) {
  if (!c || t_lb < 0 || t_md < 0 || subs < 0 || subs > c->p.n_sub) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  c->t_lb = t_lb;
  c->t_md = t_md;
  c->subs = subs;
  return fail(c, invalidate_corner_cache(c));
}

const char* lbmd_strerror(int code) {
  switch (code) {
    case LBMD_OK: return "ok";
    case LBMD_EINVAL: return "invalid parameter or argument";
    case LBMD_ESTATE: return "call out of order (MD steps per LB step must equal n_sub)";
    case LBMD_EHIP: return "HIP runtime failure (context disabled)";
    case LBMD_ENOSPACE: return "workspace too small";
    case LBMD_ENONFINITE: return "a particle position or velocity became non-finite";
  }
  return "unknown status";
}

}  // extern "C"
