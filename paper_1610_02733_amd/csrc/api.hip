// C ABI entry points: parameter checks, workspace carving, per-replica
// tables, step bookkeeping, captured cycles and the launch-shape autotuner.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>

#include "lbmd_internal.hpp"

using namespace lbmd_impl;

struct lbmd : Context {
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph_def = nullptr;
  hipGraphExec_t graph_exec = nullptr;
};

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t a) { return (a + kAlign - 1) / kAlign * kAlign; }

bool valid_one(const lbmd_params* p) {
  if (!p) return false;
  if (p->nx < 2 || p->ny < 2 || p->nz < 2) return false;
  const int64_t S = (int64_t)p->nx * p->ny * p->nz;
  if (S > (int64_t)0x3FFFFFFF) return false;
  if (p->n_sub < 1) return false;
  if (p->variant < 1 || p->variant > 3) return false;
  if (p->precision != 32 && p->precision != 64) return false;
  if (p->n_particles < 0) return false;
  if (!(p->rho0 > 0.0) || !(p->nu > 0.0) || !(p->kT >= 0.0) || !(p->friction >= 0.0)) return false;
  if (!(p->nu_bulk < 0.0 || p->nu_bulk > 0.0)) return false;
  if (!(fabs(p->gamma_ghost) < 1.0)) return false;
  if (p->n_particles > 0 && !(p->particle_mass > 0.0)) return false;
  if (p->force_model < 0 || p->force_model > 3) return false;
  if (p->stencil < 0 || p->stencil > 1) return false;
  if (p->force_model >= 2) {
    if (p->chain_len < 1 || (p->n_particles % p->chain_len) != 0) return false;
    if (!(p->wca_sigma > 0.0) || !(p->wca_eps >= 0.0) || !(p->k_bond >= 0.0)) return false;
    if (!isfinite(p->r0_bond)) return false;
    if (p->force_model == 3 && !(p->r0_bond > 0.0)) return false;  // FENE R0
  }
  for (int d = 0; d < 3; ++d)
    if (!isfinite(p->body_force[d]) || !isfinite(p->f_ext[d])) return false;
  return true;
}

// Replicas advance in lockstep through shared kernels: they must agree on
// the time-scale contrast, the precision and the coupling variant.
bool valid_set(const lbmd_params* p, int32_t R) {
  if (!p || R < 1 || R > (1 << 20)) return false;
  int64_t S = 0, N = 0, C = 0;
  for (int r = 0; r < R; ++r) {
    if (!valid_one(p + r)) return false;
    if (p[r].n_sub != p[0].n_sub || p[r].precision != p[0].precision ||
        p[r].variant != p[0].variant || p[r].stencil != p[0].stencil)
      return false;
    S += ((int64_t)p[r].nx * p[r].ny * p[r].nz + 63) / 64 * 64;
    N += p[r].n_particles;
    C += force_cells(p + r);
  }
  return S < (int64_t)0x7FFFFFFF - 256 && N < (int64_t)0x7FFFFFFF / 32 &&
         C < ((int64_t)1 << 30) - 1;  // two halves of counts: 32-bit entries
}

Plan make_plan(const lbmd_params* p, int32_t R) {
  Plan pl;
  pl.R = R;
  pl.prec = p[0].precision;
  pl.n_sub = p[0].n_sub;
  pl.Stot = pl.Ntot = pl.Ctot = 0;
  pl.cell_cap = 0;
  pl.nitems = 0;
  pl.any_forces2 = false;
  pl.row_replicas = 0;
  for (int r = 0; r < R; ++r) {
    pl.row_replicas += row_path(p[r]) ? 1 : 0;
    const int64_t S = (int64_t)p[r].nx * p[r].ny * p[r].nz;
    pl.site_off.push_back(pl.Stot);
    pl.part_off.push_back(pl.Ntot);
    pl.cell_off.push_back(pl.Ctot);
    pl.item_off.push_back(pl.nitems);
    pl.Stot += (S + 63) / 64 * 64;
    pl.Ntot += p[r].n_particles;
    pl.Ctot += force_cells(p + r);
    pl.cell_cap = std::max(pl.cell_cap, force_cell_capacity(p + r));
    pl.nitems += (int)((S + kBlock - 1) / kBlock);
    pl.any_forces2 = pl.any_forces2 || (p[r].force_model >= 2 && p[r].n_particles > 0);
  }
  pl.item_off.push_back(pl.nitems);
  pl.P = pl.Stot;  // each buffer holds 19 * Stot values: replica r at 19 * site_off[r]
  Layout& L = pl.lay;
  const size_t S = (size_t)pl.Stot, N = (size_t)std::max<int64_t>(pl.Ntot, 1);
  const size_t C = (size_t)std::max<int64_t>(pl.Ctot, 1);
  const size_t t = pl.prec == 32 ? 4 : 8;
  size_t o = 0;
  const size_t P = (size_t)pl.P;
  L.pop[0] = o; o = up(o + 19 * P * t);
  L.pop[1] = o; o = up(o + 19 * P * t);
  L.transfer = o; o = up(o + 4 * S * t);
  L.mark = o; o = up(o + (S / 64) * 8);
  L.rep_lb = o; o = up(o + (size_t)R * (pl.prec == 32 ? sizeof(RepLB<float>) : sizeof(RepLB<double>)));
  L.rep_md = o; o = up(o + (size_t)R * sizeof(RepMD));
  L.item_rep = o; o = up(o + (size_t)(R + 1) * 4);
  L.part_rep = o; o = up(o + N * 4);
  L.pid = o; o = up(o + N * 4);
  L.clock = o; o = up(o + sizeof(Clock));
  L.fcons = o; o = up(o + 3 * N * 8);
  L.sort_x = o; o = up(o + 3 * N * 8);
  L.sort_v = o; o = up(o + 3 * N * 8);
  L.sort_img = o; o = up(o + 3 * N * 4);
  L.fc_held = o; o = up(o + 3 * N * 8);
  L.cc = o; o = up(o + (p[0].stencil == 1 ? 4 * 27 : 4 * 8) * N * t);  // site cache
  L.own = o; o = up(o + (p[0].stencil == 1 ? 4 * 27 : 4 * 8) * N * t);
  L.owner = o; o = up(o + S * 4);
  L.moved_at = o; o = up(o + N * 8);
  // transfer lists: per segment of kBlock coupling lanes, kBlock * (sites
  // per lane) transfer entries and kBlock / lanes particles; lanes x sites
  // per lane is 8 for the cube (8 x 1 while recording, 2 x 4) and 32 for the
  // three-point stencil (8 x 4)
  const size_t lanes_max = p[0].stencil == 1 ? 32 : 8;
  pl.nseg = (int64_t)((N * lanes_max + kBlock - 1) / kBlock);
  const size_t nent = (size_t)pl.nseg * kBlock;  // >= every launch's lanes x sites per lane
  L.slist_site = o; o = up(o + nent * 4);
  L.slist_delta = o; o = up(o + nent * 4 * t);
  L.mlist = o; o = up(o + nent * 8);  // kBlock / lanes int4 per segment, lanes >= 2
  L.seg_count = o; o = up(o + 2 * (size_t)pl.nseg * 4);
  L.bin_count = o; o = up(o + (2 * C + 2) * 4);
  L.bin_of = o; o = up(o + N * 4);
  L.bin_slot = o; o = up(o + C * (size_t)pl.cell_cap * 4);
  L.bin_ovf = o; o = up(o + N * 4);
  L.sort_keys = o; o = up(o + 2 * N * 8);
  L.sort_vals = o; o = up(o + 2 * N * 4);
  L.sort_temp = o; o = up(o + sort_temp_bytes((int64_t)N));
  L.flags = o; o = up(o + 16 * 4);
  L.partials = o; o = up(o + (size_t)pl.nitems * kRedWidth * 8);
  L.totals = o; o = up(o + (size_t)R * kRedWidth * 8);
  L.total = o;
  return pl;
}

// Mode norms b_k of the D3Q19 basis, k = 4..18 (stress, then kinetic modes).
const double kNorm[15] = {2.0 / 3, 4.0 / 3, 4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 2.0 / 3, 2.0 / 3,
                          2.0 / 3, 2.0 / 9, 2.0 / 9, 2.0 / 9, 2.0,     4.0 / 3, 4.0 / 9};

Geom geom_of(const lbmd_params& p) {
  Geom g;
  g.nx = p.nx;
  g.ny = p.ny;
  g.nz = p.nz;
  g.S = p.nx * p.ny * p.nz;
  g.A = p.nx * p.ny;
  g.inv_nx = 1.0 / p.nx;
  g.inv_ny = 1.0 / p.ny;
  return g;
}

template <typename T>
RepLB<T> rep_lb(const Context* c, int r) {
  const lbmd_params& p = c->p[r];
  RepLB<T> q;
  q.g = geom_of(p);
  q.site_off = (int)c->plan.site_off[r];
  q.item_off = (int)c->plan.item_off[r];
  q.rows = row_path(p) ? 1 : 0;
  q.key0 = (uint32_t)(p.seed & 0xFFFFFFFFu);
  q.key1 = (uint32_t)(p.seed >> 32);
  q.tag0 = lbmd_dev::noise_tag(lbmd_dev::kPurposeFluid, p.replica, 0);
  q.tag1 = lbmd_dev::noise_tag(lbmd_dev::kPurposeFluid, p.replica, 1);
  const double gs = (6.0 * p.nu - 1.0) / (6.0 * p.nu + 1.0);
  const double gb = p.nu_bulk < 0.0 ? gs : (9.0 * p.nu_bulk - 1.0) / (9.0 * p.nu_bulk + 1.0);
  const double gg = p.gamma_ghost;
  q.k.rho0 = (T)p.rho0;
  q.k.gs = (T)gs;
  q.k.gb = (T)gb;
  q.k.gg = (T)gg;
  q.k.hs = (T)(0.5 * (1.0 + gs));
  q.k.hb = (T)(0.5 * (1.0 + gb));
  q.k.mu = (T)(3.0 * p.kT);
  for (int v = 0; v < 15; ++v) {
    const int k = v + 4;
    const double g = k == 4 ? gb : (k <= 9 ? gs : gg);
    q.k.ns[v] = (T)(sqrt(kNorm[v] * (1.0 - g * g)) * sqrt(12.0) / 65536.0);
  }
  for (int d = 0; d < 3; ++d) q.k.g[d] = (T)p.body_force[d];
  q.k.noise = p.kT > 0.0 ? 1 : 0;
  return q;
}

RepMD rep_md(const Context* c, int r) {
  const lbmd_params& p = c->p[r];
  RepMD m;
  memset(&m, 0, sizeof(m));
  m.g = geom_of(p);
  m.site_off = (int)c->plan.site_off[r];
  m.part_off = (int)c->plan.part_off[r];
  m.N = p.n_particles;
  m.cell_off = (int)c->plan.cell_off[r];
  m.variant = p.variant;
  m.noise = (p.kT > 0.0 && p.friction > 0.0) ? 1 : 0;
  m.split_kick = p.force_model >= 2 ? 1 : 0;
  m.force_model = p.force_model;
  m.stencil = p.stencil;
  m.chain_len = p.force_model >= 2 ? p.chain_len : 1;
  m.key0 = (uint32_t)(p.seed & 0xFFFFFFFFu);
  m.key1 = (uint32_t)(p.seed >> 32);
  m.tag = lbmd_dev::noise_tag(lbmd_dev::kPurposeParticle, p.replica, 0);
  const double tau = 1.0 / p.n_sub;
  m.rho0 = p.rho0;
  m.gamma = p.friction;
  m.amp = sqrt(2.0 * p.friction * p.kT / tau);
  m.tau = tau;
  m.h = p.n_particles > 0 ? tau / (2.0 * p.particle_mass) : 0.0;
  m.inv_m = p.n_particles > 0 ? 1.0 / p.particle_mass : 0.0;
  m.L[0] = p.nx;
  m.L[1] = p.ny;
  m.L[2] = p.nz;
  for (int d = 0; d < 3; ++d) m.f_ext[d] = p.f_ext[d];
  m.k_bond = p.k_bond;
  m.r0_bond = p.r0_bond;
  m.wca_eps = p.wca_eps;
  m.wca_sigma = p.wca_sigma;
  const int Ls[3] = {p.nx, p.ny, p.nz};
  for (int d = 0; d < 3; ++d) {
    const int n = cells_per_axis(&p, d);
    m.nb[d] = n;
    m.inv_edge[d] = (double)n / (double)Ls[d];
  }
  return m;
}

int fail(Context* c, hipError_t e) {
  if (e == hipSuccess) return LBMD_OK;
  c->sticky = LBMD_EHIP;
  return LBMD_EHIP;
}

// Per-replica tables and the clock, uploaded once at creation.
hipError_t upload_tables(Context* c) {
  const Plan& pl = c->plan;
  const int R = pl.R;
  hipError_t e;
  if (pl.prec == 32) {
    std::vector<RepLB<float>> lb(R);
    for (int r = 0; r < R; ++r) lb[r] = rep_lb<float>(c, r);
    e = hipMemcpyAsync(at(c, pl.lay.rep_lb), lb.data(), sizeof(RepLB<float>) * R,
                       hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  } else {
    std::vector<RepLB<double>> lb(R);
    for (int r = 0; r < R; ++r) lb[r] = rep_lb<double>(c, r);
    e = hipMemcpyAsync(at(c, pl.lay.rep_lb), lb.data(), sizeof(RepLB<double>) * R,
                       hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  if (e != hipSuccess) return e;
  std::vector<RepMD> md(R);
  for (int r = 0; r < R; ++r) md[r] = rep_md(c, r);
  std::vector<int32_t> items(pl.item_off.begin(), pl.item_off.end());
  std::vector<int32_t> prep((size_t)std::max<int64_t>(pl.Ntot, 1), 0);
  for (int r = 0; r < R; ++r)
    for (int q = 0; q < c->p[r].n_particles; ++q) prep[pl.part_off[r] + q] = r;
  Clock clk{0, 0, 0, 0};
  if ((e = hipMemcpyAsync(at(c, pl.lay.rep_md), md.data(), sizeof(RepMD) * R,
                          hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(at(c, pl.lay.item_rep), items.data(), sizeof(int32_t) * items.size(),
                          hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(at(c, pl.lay.part_rep), prep.data(), sizeof(int32_t) * prep.size(),
                          hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(at(c, pl.lay.clock), &clk, sizeof(clk), hipMemcpyHostToDevice,
                          c->stream)) != hipSuccess)
    return e;
  return hipStreamSynchronize(c->stream);
}

hipError_t write_clock(Context* c) {
  Clock clk{(long long)c->t_lb, (long long)(c->t_md - c->subs), c->cur, 0};
  hipError_t e = hipMemcpyAsync(at(c, c->plan.lay.clock), &clk, sizeof(clk), hipMemcpyHostToDevice,
                                c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

void drop_graph(lbmd* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph_def) (void)hipGraphDestroy(c->graph_def);
  c->graph_exec = nullptr;
  c->graph_def = nullptr;
}

// No particle has changed stencils at the current MD step count and no
// stencil records a particle (owner_of_shared): at creation, at a new
// binding, and where the step counters or the particles are set from
// outside.  The next MD step refills the cache, which records every
// particle's stencil again.
hipError_t reset_stencil_records(Context* c) {
  hipError_t e = hipMemsetAsync(at(c, c->plan.lay.owner), 0xFF, (size_t)c->plan.Stot * 4,
                                c->stream);
  if (e == hipSuccess && c->plan.Ntot > 0)
    e = hipMemsetAsync(at(c, c->plan.lay.moved_at), 0xFF, (size_t)c->plan.Ntot * 8, c->stream);
  return e;
}

int create(const lbmd_params* p, int32_t R, void* d_ws, size_t ws_bytes, void* hip_stream,
           lbmd** out) {
  if (!out) return LBMD_EINVAL;
  *out = nullptr;
  if (!valid_set(p, R) || !d_ws || ((uintptr_t)d_ws % kAlign) != 0) return LBMD_EINVAL;
  Plan pl = make_plan(p, R);
  if (ws_bytes < pl.lay.total) return LBMD_ENOSPACE;
  lbmd* c = new (std::nothrow) lbmd();
  if (!c) return LBMD_EINVAL;
  c->p.assign(p, p + R);
  c->plan = pl;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)d_ws;
  c->x = c->v = nullptr;
  c->img = nullptr;
  c->bound = false;
  c->cache_dirty = true;
  c->retag = false;
  c->t_lb = c->t_md = 0;
  c->subs = 0;
  c->cur = 0;
  c->sticky = LBMD_OK;
  c->tune.lb_blocks = 0;
  c->tune.part_blocks = 0;
  c->tune.couple_lanes = 0;
  c->graph_ok = false;
  c->popv[0] = at(c, pl.lay.pop[0]);
  c->popv[1] = at(c, pl.lay.pop[1]);
  c->rec_part = nullptr;
  c->rec_J = nullptr;
  c->rec_mark = nullptr;
  c->scratch_rows = nullptr;
  // fluid at rest (all deviations zero), nothing transferred yet
  hipError_t e = hipMemsetAsync(c->ws, 0, pl.lay.total, c->stream);
  if (e == hipSuccess) e = reset_stencil_records(c);
  if (e == hipSuccess) e = upload_tables(c);
  // set-up of lb_moments_noalloc: this GPU's address of the library's fixed
  // reduction array (looked up once per device)
  if (e == hipSuccess) e = moments_scratch(&c->scratch_rows);
  if (e != hipSuccess) {
    delete c;
    return LBMD_EHIP;
  }
  *out = c;
  return LBMD_OK;
}

int check_rep(lbmd* c, int32_t rep) {
  if (!c || rep < 0 || rep >= c->plan.R) return LBMD_EINVAL;
  return c->sticky;
}

// One MD step of every replica (no host-side checks).
hipError_t substep_launches(Context* c, int substep) {
  hipError_t e = launch_couple(c, substep);
  if (e == hipSuccess && c->plan.any_forces2) e = launch_forces_and_kick(c, substep);
  return e;
}

}  // namespace

extern "C" {

size_t lbmd_workspace_bytes(const lbmd_params* p) {
  if (!valid_set(p, 1)) return 0;
  return make_plan(p, 1).lay.total;
}

size_t lbmd_batch_workspace_bytes(const lbmd_params* per_rep, int32_t n_rep) {
  if (!valid_set(per_rep, n_rep)) return 0;
  return make_plan(per_rep, n_rep).lay.total;
}

int lb_create(const lbmd_params* p, void* d_ws, size_t ws_bytes, void* hip_stream, lbmd** out) {
  return create(p, 1, d_ws, ws_bytes, hip_stream, out);
}

int lb_create_batch(const lbmd_params* per_rep, int32_t n_rep, void* d_ws, size_t ws_bytes,
                    void* hip_stream, lbmd** out) {
  return create(per_rep, n_rep, d_ws, ws_bytes, hip_stream, out);
}

int lb_destroy(lbmd* c) {
  if (!c) return LBMD_OK;
  drop_graph(c);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  delete c;
  return LBMD_OK;
}

int lbmd_replica_count(lbmd* c) { return c ? c->plan.R : LBMD_EINVAL; }

int lbmd_bind_particles(lbmd* c, void* d_x, void* d_v, int32_t* d_img) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->plan.Ntot > 0 && (!d_x || !d_v || !d_img)) return LBMD_EINVAL;
  // the pending transfer is kept: the bound particles' own transfers go to J
  int rc0 = fail(c, launch_leave_transfers(c));
  if (rc0) return rc0;
  c->x = d_x;
  c->v = d_v;
  c->img = d_img;
  c->bound = c->plan.Ntot > 0;
  drop_graph(c);
  int rc = fail(c, launch_init_pid(c));
  if (!rc) rc = fail(c, reset_stencil_records(c));
  if (rc) return rc;
  return fail(c, launch_init_forces(c));
}

int lbmd_sort_particles(lbmd* c, int32_t* d_perm) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  for (int r = 0; r < c->plan.R; ++r)
    if (c->p[r].force_model >= 2) return LBMD_EINVAL;  // bonds follow the particle order
  if (c->plan.Ntot == 0) return LBMD_OK;
  if (!c->bound || c->subs != 0 || c->rec_part) return LBMD_ESTATE;
  bool too_small = false;
  const int rc = fail(c, launch_sort_particles(c, d_perm, &too_small));
  if (rc) return rc;
  return too_small ? LBMD_ENOSPACE : LBMD_OK;
}

int md_couple_substep(lbmd* c) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->subs >= c->plan.n_sub) return LBMD_ESTATE;
  if (c->plan.Ntot > 0 && !c->bound) return LBMD_ESTATE;
  const int rc = fail(c, substep_launches(c, c->subs));
  if (rc) return rc;
  c->t_md += 1;
  c->subs += 1;
  return LBMD_OK;
}

int lb_step(lbmd* c) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->plan.Ntot > 0 && c->subs != c->plan.n_sub) return LBMD_ESTATE;
  int rc = fail(c, launch_collide_stream(c));
  if (!rc) rc = fail(c, launch_clock_advance(c));
  if (rc) return rc;
  c->cur = 1 - c->cur;
  c->t_lb += 1;
  c->subs = 0;
  return LBMD_OK;
}

int lbmd_run_cycles(lbmd* c, int32_t ncycles) {
  if (!c || ncycles < 0) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->subs != 0) return LBMD_ESTATE;
  if (c->plan.Ntot > 0 && !c->bound) return LBMD_ESTATE;
  if (ncycles == 0) return LBMD_OK;
  const int n = c->plan.Ntot > 0 ? c->plan.n_sub : 0;
  if (!c->graph_exec) {
    // capture one cycle (n MD steps + one LB step) on a private stream; the
    // kernels read the step clock from device memory, so the same graph
    // serves every cycle
    if (!c->capture_stream) {
      int rc = fail(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
      if (rc) return rc;
    }
    hipStream_t user = c->stream;
    c->stream = c->capture_stream;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    const int32_t saved_subs = c->subs;
    for (int s = 0; s < n && e == hipSuccess; ++s) e = substep_launches(c, s);
    c->subs = n;  // MD steps the clock advance accounts for
    if (e == hipSuccess) e = launch_collide_stream(c);
    if (e == hipSuccess) e = launch_clock_advance(c);
    c->subs = saved_subs;
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    c->stream = user;
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    c->graph_def = g;
    int rc = fail(c, e);
    if (rc) {
      drop_graph(c);
      return rc;
    }
  }
  for (int32_t k = 0; k < ncycles; ++k) {
    int rc = fail(c, hipGraphLaunch(c->graph_exec, c->stream));
    if (rc) return rc;
  }
  c->t_lb += ncycles;
  c->t_md += (int64_t)ncycles * n;
  if (ncycles & 1) c->cur = 1 - c->cur;
  return LBMD_OK;
}

// Totals of replica r (LBMD_TOT_* layout) from its reduction row t (columns:
// 0 sum drho, 1-3 sum j, 4-6 sum J, 7 sum |u|^2, 8-10 sum v, 11 sum |v|^2).
static void fill_totals(const lbmd* c, int r, const double* t, double* h) {
  const lbmd_params& p = c->p[r];
  const double m = p.particle_mass;
  const double S = (double)p.nx * p.ny * p.nz;
  h[LBMD_TOT_MASS] = p.rho0 * S + t[0];
  for (int d = 0; d < 3; ++d) {
    h[LBMD_TOT_PFLUID + d] = t[1 + d] + t[4 + d];
    h[LBMD_TOT_PSEEN + d] = t[1 + d] + (p.variant >= 2 ? t[4 + d] : 0.0);
    h[LBMD_TOT_PPART + d] = m * t[8 + d];
  }
  h[LBMD_TOT_KEPART] = 0.5 * m * t[11];
  h[LBMD_TOT_U2FLUID] = t[7] / S;
  h[LBMD_TOT_TLB] = (double)c->t_lb;
  h[LBMD_TOT_TMD] = (double)c->t_md;
  h[LBMD_TOT_TPART] = p.n_particles > 0 ? m * t[11] / (3.0 * p.n_particles) : 0.0;
}

static int moments_common(lbmd* c, int32_t rep, void* d_rho, void* d_u, double* h_totals,
                          int all) {
  int rc = check_rep(c, rep);
  if (rc) return rc;
  const int R = c->plan.R;
  double* d_tot = h_totals ? (double*)at(c, c->plan.lay.totals) : nullptr;
  rc = fail(c, launch_leave_transfers(c));
  if (!rc) rc = fail(c, launch_moments(c, rep, d_rho, d_u, d_tot));
  if (rc || !h_totals) return rc;
  std::vector<double> tot((size_t)R * kRedWidth);
  int32_t flags[16];
  rc = fail(c, hipMemcpyAsync(tot.data(), d_tot, sizeof(double) * tot.size(),
                              hipMemcpyDeviceToHost, c->stream));
  if (!rc)
    rc = fail(c, hipMemcpyAsync(flags, at(c, c->plan.lay.flags), sizeof(flags),
                                hipMemcpyDeviceToHost, c->stream));
  if (!rc) rc = fail(c, hipStreamSynchronize(c->stream));
  if (rc) return rc;
  const int r0 = all ? 0 : rep, r1 = all ? R : rep + 1;
  for (int r = r0; r < r1; ++r)
    fill_totals(c, r, &tot[(size_t)r * kRedWidth], h_totals + (size_t)(all ? r : 0) * LBMD_NTOTALS);
  return flags[0] ? LBMD_ENONFINITE : LBMD_OK;
}

int lb_moments(lbmd* c, void* d_rho, void* d_u, double* h_totals) {
  return moments_common(c, 0, d_rho, d_u, h_totals, 0);
}

int lb_moments_noalloc(lbmd* c, void* d_rho, void* d_u, double* h_totals) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->plan.R != 1) return LBMD_EINVAL;  // single system only
  if (!c->scratch_rows) return LBMD_ESTATE;
  // the reduction needs min(items, kScratchRows) block rows plus the totals
  // row; the grid is capped at the array's row count, so any lattice fits
  const int64_t rows = std::min<int64_t>(c->plan.nitems, kScratchRows) + 1;
  if (rows * kRedWidth > kScratchDoubles) return LBMD_ENOSPACE;
  int rc = fail(c, launch_leave_transfers(c));
  if (!rc) rc = fail(c, launch_moments_rows(c, d_rho, d_u, c->scratch_rows));
  if (rc || !h_totals) return rc;
  double tot[kRedWidth];
  int32_t flags[16];
  rc = fail(c, hipMemcpyAsync(tot, c->scratch_rows + (size_t)kScratchRows * kRedWidth,
                              sizeof(tot), hipMemcpyDeviceToHost, c->stream));
  if (!rc)
    rc = fail(c, hipMemcpyAsync(flags, at(c, c->plan.lay.flags), sizeof(flags),
                                hipMemcpyDeviceToHost, c->stream));
  if (!rc) rc = fail(c, hipStreamSynchronize(c->stream));
  if (rc) return rc;
  fill_totals(c, 0, tot, h_totals);
  return flags[0] ? LBMD_ENONFINITE : LBMD_OK;
}

int lbmd_batch_moments(lbmd* c, double* h_totals) {
  if (!h_totals) return LBMD_EINVAL;
  return moments_common(c, 0, nullptr, nullptr, h_totals, 1);
}

int lbmd_batch_get_populations(lbmd* c, int32_t rep, void* d_dst) {
  int rc = check_rep(c, rep);
  if (rc || !d_dst) return rc ? rc : LBMD_EINVAL;
  rc = fail(c, launch_leave_transfers(c));  // variant 3 reads J
  if (rc) return rc;
  return fail(c, launch_get_populations(c, rep, d_dst));
}

int lbmd_batch_set_populations(lbmd* c, int32_t rep, const void* d_src) {
  int rc = check_rep(c, rep);
  if (rc || !d_src) return rc ? rc : LBMD_EINVAL;
  // the pending transfer is kept (variants 1, 2) and the cache is refilled
  // from J: the particles' own transfers first go there
  rc = fail(c, launch_leave_transfers(c));
  if (!rc) rc = fail(c, launch_set_populations(c, rep, d_src));
  if (rc) return rc;
  if (c->p[0].variant == 3) {
    // the transfer received in the current interval is part of the
    // variant-3 state that the new populations replace
    const size_t t = c->plan.prec == 32 ? 4 : 8, off = (size_t)c->plan.site_off[rep];
    const size_t n = (size_t)c->p[rep].nx * c->p[rep].ny * c->p[rep].nz;
    rc = fail(c, hipMemsetAsync((char*)at(c, c->plan.lay.transfer) + off * 4 * t, 0, n * 4 * t,
                                c->stream));
    if (rc) return rc;
  }
  return fail(c, invalidate_corner_cache(c));
}

int lbmd_batch_get_transfer(lbmd* c, int32_t rep, void* d_dst) {
  int rc = check_rep(c, rep);
  if (rc || !d_dst) return rc ? rc : LBMD_EINVAL;
  rc = fail(c, launch_leave_transfers(c));
  if (rc) return rc;
  return fail(c, launch_get_transfer(c, rep, d_dst));
}

int lbmd_get_populations(lbmd* c, void* d_dst) { return lbmd_batch_get_populations(c, 0, d_dst); }
int lbmd_set_populations(lbmd* c, const void* d_src) {
  return lbmd_batch_set_populations(c, 0, d_src);
}
int lbmd_get_transfer(lbmd* c, void* d_dst) { return lbmd_batch_get_transfer(c, 0, d_dst); }

int lbmd_get_counters(lbmd* c, int64_t* t_lb, int64_t* t_md, int32_t* subs) {
  if (!c) return LBMD_EINVAL;
  if (t_lb) *t_lb = c->t_lb;
  if (t_md) *t_md = c->t_md;
  if (subs) *subs = c->subs;
  return LBMD_OK;
}

int lbmd_set_counters(lbmd* c, int64_t t_lb, int64_t t_md, int32_t subs) {
  if (!c || t_lb < 0 || t_md < subs || subs < 0 || subs > c->plan.n_sub) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  int rc0 = fail(c, launch_leave_transfers(c));  // J complete before the cache is rebuilt
  if (rc0) return rc0;
  c->t_lb = t_lb;
  c->t_md = t_md;
  c->subs = subs;
  int rc = fail(c, write_clock(c));
  if (!rc) rc = fail(c, reset_stencil_records(c));
  // the force cells are kept in halves by MD-step parity: bin again under
  // the new count
  if (!rc && c->bound && c->plan.any_forces2) rc = fail(c, launch_forces(c));
  if (rc) return rc;
  return fail(c, invalidate_corner_cache(c));
}

}  // extern "C"


// ---------------------------------------------------------------------------
// Saved states and the reverse sweep.
// ---------------------------------------------------------------------------
namespace {

// Saved state: counters, the stored populations (pull storage, as held by
// the context), particle positions, velocities and image counts.  Taken at
// an LB-step boundary, where the transfer field is empty.
struct StateLayout {
  size_t counters, pop, x, v, img, pid, total;
};

StateLayout state_layout(const Context* c) {
  StateLayout s;
  const size_t P = (size_t)c->plan.P, N = (size_t)c->plan.Ntot;
  const size_t t = c->plan.prec == 32 ? 4 : 8;
  size_t o = 0;
  s.counters = o; o = up(o + 16);
  s.pop = o; o = up(o + 19 * P * t);
  s.x = o; o = up(o + 3 * N * 8);
  s.v = o; o = up(o + 3 * N * 8);
  s.img = o; o = up(o + 3 * N * 4);
  s.pid = o; o = up(o + N * 4);
  s.total = o;
  return s;
}

AdjLayout adj_layout(const Context* c, int K) {
  AdjLayout L;
  const size_t S = (size_t)c->plan.Stot, N = (size_t)std::max<int64_t>(c->plan.Ntot, 1);
  const size_t t = c->plan.prec == 32 ? 4 : 8, n = (size_t)c->plan.n_sub, k = (size_t)K;
  size_t o = 0;
  const size_t P = (size_t)c->plan.P;
  L.slots = o; o = up(o + (k - 1) * 19 * P * t);
  L.jrec = o; o = up(o + k * S * 4 * t);
  L.mrec = o; o = up(o + k * (S / 64) * 8);
  L.prec = o; o = up(o + k * n * kAdjRec * N * 8);
  L.pbar[0] = o; o = up(o + 19 * P * t);
  L.pbar[1] = o; o = up(o + 19 * P * t);
  L.jbar = o; o = up(o + S * 4 * t);
  L.abar = o; o = up(o + S * 4 * t);
  L.xbar = o; o = up(o + 3 * N * 8);
  L.vbar = o; o = up(o + 3 * N * 8);
  L.ubar = o; o = up(o + 3 * N * 8);
  L.pacc = o; o = up(o + 4 * N * 8);
  L.nuacc = o; o = up(o + (size_t)kAdjBlocks * 4 * 8);
  L.total = o;
  return L;
}

bool adjoint_supported(const Context* c) {
  return c->plan.R == 1 && c->p[0].force_model <= 1 && c->p[0].variant <= 2 &&
         c->p[0].stencil == 0;
}

// Particles, counters and an empty transfer field from a saved state (the
// populations are handled by the caller).
int load_common(lbmd* c, const char* src, const StateLayout& sl) {
  const size_t N = (size_t)c->plan.Ntot, S = (size_t)c->plan.Stot;
  long long cnt[2];
  int rc = fail(c, hipMemcpyAsync(cnt, src + sl.counters, sizeof(cnt), hipMemcpyDeviceToHost,
                                  c->stream));
  if (!rc) rc = fail(c, hipStreamSynchronize(c->stream));
  if (rc) return rc;
  if (cnt[0] < 0 || cnt[1] < 0) return LBMD_EINVAL;
  if (N > 0) {
    rc = fail(c, hipMemcpyAsync(c->x, src + sl.x, 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
    if (!rc)
      rc = fail(c, hipMemcpyAsync(c->v, src + sl.v, 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
    if (!rc)
      rc = fail(c, hipMemcpyAsync(c->img, src + sl.img, 3 * N * 4, hipMemcpyDeviceToDevice,
                                  c->stream));
    if (!rc)
      rc = fail(c, hipMemcpyAsync(at(c, c->plan.lay.pid), src + sl.pid, N * 4,
                                  hipMemcpyDeviceToDevice, c->stream));
    if (rc) return rc;
  }
  const size_t t = c->plan.prec == 32 ? 4 : 8;
  rc = fail(c, hipMemsetAsync(at(c, c->plan.lay.transfer), 0, S * 4 * t, c->stream));
  if (!rc) rc = fail(c, hipMemsetAsync(at(c, c->plan.lay.mark), 0, (S / 64) * 8, c->stream));
  if (rc) return rc;
  c->t_lb = cnt[0];
  c->t_md = cnt[1];
  c->subs = 0;
  rc = fail(c, write_clock(c));
  if (!rc) rc = fail(c, reset_stencil_records(c));
  if (!rc) rc = fail(c, invalidate_corner_cache(c));
  if (!rc && c->bound) rc = fail(c, launch_init_forces(c));
  return rc;
}

}  // namespace

extern "C" {

size_t lbmd_state_bytes(lbmd* c) { return c ? state_layout(c).total : 0; }

int lbmd_save_state(lbmd* c, void* d_dst) {
  if (!c || !d_dst) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->subs != 0) return LBMD_ESTATE;
  if (c->plan.Ntot > 0 && !c->bound) return LBMD_ESTATE;
  const StateLayout sl = state_layout(c);
  char* dst = (char*)d_dst;
  const size_t N = (size_t)c->plan.Ntot;
  const size_t t = c->plan.prec == 32 ? 4 : 8;
  int rc = fail(c, launch_store_counters(c, dst + sl.counters, c->t_lb, c->t_md));
  if (!rc)
    rc = fail(c, hipMemcpyAsync(dst + sl.pop, c->popv[c->cur], 19 * (size_t)c->plan.P * t,
                                hipMemcpyDeviceToDevice, c->stream));
  if (!rc && N > 0) {
    rc = fail(c, hipMemcpyAsync(dst + sl.x, c->x, 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
    if (!rc)
      rc = fail(c, hipMemcpyAsync(dst + sl.v, c->v, 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
    if (!rc)
      rc = fail(c, hipMemcpyAsync(dst + sl.img, c->img, 3 * N * 4, hipMemcpyDeviceToDevice,
                                  c->stream));
    if (!rc)
      rc = fail(c, hipMemcpyAsync(dst + sl.pid, at(c, c->plan.lay.pid), N * 4,
                                  hipMemcpyDeviceToDevice, c->stream));
  }
  return rc;
}

int lbmd_load_state(lbmd* c, const void* d_src) {
  if (!c || !d_src) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->plan.Ntot > 0 && !c->bound) return LBMD_ESTATE;
  const StateLayout sl = state_layout(c);
  const char* src = (const char*)d_src;
  const size_t t = c->plan.prec == 32 ? 4 : 8;
  int rc = fail(c, hipMemcpyAsync(c->popv[c->cur], src + sl.pop, 19 * (size_t)c->plan.P * t,
                                  hipMemcpyDeviceToDevice, c->stream));
  if (rc) return rc;
  return load_common(c, src, sl);
}

size_t lbmd_adjoint_workspace_bytes(lbmd* c, int32_t seg_cycles) {
  if (!c || seg_cycles < 1 || !adjoint_supported(c)) return 0;
  return adj_layout(c, seg_cycles).total;
}

int lbmd_adjoint_attach(lbmd* c, void* d_ws, size_t bytes, int32_t seg_cycles) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (seg_cycles < 1 || !adjoint_supported(c) || !d_ws || ((uintptr_t)d_ws % kAlign) != 0)
    return LBMD_EINVAL;
  const AdjLayout L = adj_layout(c, seg_cycles);
  if (bytes < L.total) return LBMD_ENOSPACE;
  AdjState& a = c->adj;
  a.attached = true;
  a.ws = (char*)d_ws;
  a.K = seg_cycles;
  a.lay = L;
  a.ncyc = 0;
  a.slot = -1;
  a.sub = -1;
  a.pbar_cur = 0;
  return LBMD_OK;
}

int lbmd_adjoint_seed(lbmd* c, const double* d_xbar, const double* d_vbar) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  AdjState& a = c->adj;
  if (!a.attached) return LBMD_ESTATE;
  const AdjLayout& L = a.lay;
  const size_t N3 = 3 * (size_t)c->plan.Ntot * 8;
  // everything from the population adjoints to the per-block sums is zeroed
  int rc = fail(c, hipMemsetAsync(a.ws + L.pbar[0], 0, L.total - L.pbar[0], c->stream));
  if (!rc && N3 && d_xbar)
    rc = fail(c, hipMemcpyAsync(a.ws + L.xbar, d_xbar, N3, hipMemcpyDeviceToDevice, c->stream));
  if (!rc && N3 && d_vbar)
    rc = fail(c, hipMemcpyAsync(a.ws + L.vbar, d_vbar, N3, hipMemcpyDeviceToDevice, c->stream));
  if (rc) return rc;
  a.pbar_cur = 0;
  a.ncyc = 0;
  a.slot = -1;
  a.sub = -1;
  return LBMD_OK;
}

int lbmd_adjoint_record(lbmd* c, const void* d_state, int32_t ncycles) {
  if (!c || !d_state) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  AdjState& a = c->adj;
  if (!a.attached) return LBMD_ESTATE;
  if (ncycles < 1 || ncycles > a.K) return LBMD_EINVAL;
  if (c->plan.Ntot > 0 && !c->bound) return LBMD_ESTATE;
  const StateLayout sl = state_layout(c);
  const char* st = (const char*)d_state;
  int rc = load_common(c, st, sl);
  if (rc) return rc;
  const AdjLayout& L = a.lay;
  const size_t S = (size_t)c->plan.Stot, N = (size_t)c->plan.Ntot;
  const size_t t = c->plan.prec == 32 ? 4 : 8;
  const int n = c->plan.Ntot > 0 ? c->plan.n_sub : 0;
  void* base[2] = {at(c, c->plan.lay.pop[0]), at(c, c->plan.lay.pop[1])};
  const size_t P = (size_t)c->plan.P;
  auto slot_ptr = [&](int j) { return (void*)(a.ws + L.slots + (size_t)(j - 1) * 19 * P * t); };
  a.src.assign(ncycles, nullptr);
  a.t_lb.assign(ncycles, 0);
  a.t_md.assign(ncycles, 0);
  hipError_t e = hipSuccess;
  for (int j = 0; j < ncycles && e == hipSuccess; ++j) {
    void* src = j == 0 ? (void*)(st + sl.pop) : slot_ptr(j);
    void* dst = j == ncycles - 1 ? base[1 - c->cur] : slot_ptr(j + 1);
    c->popv[c->cur] = src;
    c->popv[1 - c->cur] = dst;
    c->rec_part = (double*)(a.ws + L.prec) + (size_t)j * c->plan.n_sub * kAdjRec * N;
    c->rec_J = a.ws + L.jrec + (size_t)j * S * 4 * t;
    c->rec_mark = (unsigned long long*)(a.ws + L.mrec) + (size_t)j * (S / 64);
    a.src[j] = src;
    a.t_lb[j] = c->t_lb;
    a.t_md[j] = c->t_md;
    for (int s = 0; s < n && e == hipSuccess; ++s) e = substep_launches(c, s);
    c->subs = n;
    if (e == hipSuccess) e = launch_collide_stream(c);
    if (e == hipSuccess) e = launch_clock_advance(c);
    c->subs = 0;
    c->cur = 1 - c->cur;
    c->t_lb += 1;
    c->t_md += n;
  }
  c->popv[0] = base[0];
  c->popv[1] = base[1];
  c->rec_part = nullptr;
  c->rec_J = nullptr;
  c->rec_mark = nullptr;
  rc = fail(c, e);
  if (rc) return rc;
  a.ncyc = ncycles;
  a.slot = ncycles - 1;
  a.sub = -1;
  return LBMD_OK;
}

static void adjoint_end_cycle(AdjState& a) {
  a.pbar_cur = 1 - a.pbar_cur;
  a.slot -= 1;
  a.sub = -1;
}

int lb_step_adjoint(lbmd* c) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  AdjState& a = c->adj;
  if (!a.attached || a.slot < 0 || a.sub != -1) return LBMD_ESTATE;
  int rc = fail(c, launch_collide_stream_adjoint(c));
  if (rc) return rc;
  if (c->plan.Ntot > 0)
    a.sub = c->plan.n_sub - 1;
  else
    adjoint_end_cycle(a);
  return LBMD_OK;
}

int md_couple_substep_adjoint(lbmd* c) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  AdjState& a = c->adj;
  if (!a.attached || a.slot < 0 || a.sub < 0) return LBMD_ESTATE;
  int rc = fail(c, launch_couple_adjoint(c));
  if (rc) return rc;
  if (a.sub == 0) {
    rc = fail(c, launch_adjoint_fold(c));
    if (rc) return rc;
    adjoint_end_cycle(a);
  } else {
    a.sub -= 1;
  }
  return LBMD_OK;
}

int lbmd_adjoint_result(lbmd* c, double* d_xbar, double* d_vbar, double* h_grads) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  AdjState& a = c->adj;
  if (!a.attached) return LBMD_ESTATE;
  const AdjLayout& L = a.lay;
  const size_t N = (size_t)c->plan.Ntot;
  int rc = LBMD_OK;
  if (N && d_xbar)
    rc = fail(c, hipMemcpyAsync(d_xbar, a.ws + L.xbar, 3 * N * 8, hipMemcpyDeviceToDevice,
                                c->stream));
  if (!rc && N && d_vbar)
    rc = fail(c, hipMemcpyAsync(d_vbar, a.ws + L.vbar, 3 * N * 8, hipMemcpyDeviceToDevice,
                                c->stream));
  if (rc || !h_grads) return rc;
  std::vector<double> pacc(4 * N), nuacc((size_t)kAdjBlocks * 4);
  if (N)
    rc = fail(c, hipMemcpyAsync(pacc.data(), a.ws + L.pacc, 4 * N * 8, hipMemcpyDeviceToHost,
                                c->stream));
  if (!rc)
    rc = fail(c, hipMemcpyAsync(nuacc.data(), a.ws + L.nuacc, nuacc.size() * 8,
                                hipMemcpyDeviceToHost, c->stream));
  if (!rc) rc = fail(c, hipStreamSynchronize(c->stream));
  if (rc) return rc;
  double g[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < 4; ++k)
    for (size_t p = 0; p < N; ++p) g[k] += pacc[k * N + p];
  double gb = 0.0, gs = 0.0;
  for (int b = 0; b < kAdjBlocks; ++b) {
    gb += nuacc[(size_t)b * 4 + 0];
    gs += nuacc[(size_t)b * 4 + 1];
  }
  const lbmd_params& p = c->p[0];
  const double dgs_dnu = 12.0 / ((6.0 * p.nu + 1.0) * (6.0 * p.nu + 1.0));
  h_grads[0] = g[0];
  h_grads[1] = (gs + (p.nu_bulk < 0.0 ? gb : 0.0)) * dgs_dnu;
  h_grads[2] = g[1];
  h_grads[3] = g[2];
  h_grads[4] = g[3];
  return LBMD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner: times candidate persistent-grid sizes of the LB kernels and of
// the particle kernels on this context and keeps the fastest; results are
// cached in a small JSON file keyed by device, precision, variant and size
// class.  Must run at an LB-step boundary; it leaves the state as it was
// (the collide-stream launches write only the spare population buffer and
// find no pending transfer; particle state is saved and restored).
// ---------------------------------------------------------------------------
namespace {

std::string tune_key(lbmd* c) {
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    snprintf(prop.gcnArchName, sizeof(prop.gcnArchName), "unknown");
  char buf[256];
  const int ls = (int)std::floor(std::log2((double)std::max<int64_t>(c->plan.Stot, 1)));
  const int ln = (int)std::floor(std::log2((double)std::max<int64_t>(c->plan.Ntot, 1)));
  snprintf(buf, sizeof(buf), "%s|fp%d|v%d|R%d|S2^%d|N2^%d", prop.gcnArchName, c->plan.prec,
           c->p[0].variant, c->plan.R, ls, ln);
  for (char* q = buf; *q; ++q)
    if (*q == '"' || *q == ':') *q = '_';
  return std::string(buf);
}

struct TuneEntry {
  int lb_blocks, part_blocks, couple_lanes;
};

std::map<std::string, TuneEntry> read_cache(const char* path) {
  std::map<std::string, TuneEntry> m;
  FILE* f = path ? fopen(path, "r") : nullptr;
  if (!f) return m;
  char line[512];
  while (fgets(line, sizeof(line), f)) {
    char key[300];
    int a, b, l;
    if (sscanf(line, " \"%299[^\"]\": [%d, %d, %d]", key, &a, &b, &l) == 4) m[key] = {a, b, l};
  }
  fclose(f);
  return m;
}

void write_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
  if (!path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : m)
    fprintf(f, "  \"%s\": [%d, %d, %d]%s\n", kv.first.c_str(), kv.second.lb_blocks,
            kv.second.part_blocks, kv.second.couple_lanes, ++i < m.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
}

// mean milliseconds of `reps` calls of fn on the context stream
template <typename F>
double time_ms(lbmd* c, F fn, int reps, hipError_t* err) {
  hipEvent_t a, b;
  *err = hipEventCreate(&a);
  if (*err == hipSuccess) *err = hipEventCreate(&b);
  if (*err != hipSuccess) return 0.0;
  *err = fn();  // warm-up
  if (*err == hipSuccess) *err = hipEventRecord(a, c->stream);
  for (int k = 0; k < reps && *err == hipSuccess; ++k) *err = fn();
  if (*err == hipSuccess) *err = hipEventRecord(b, c->stream);
  if (*err == hipSuccess) *err = hipEventSynchronize(b);
  float ms = 0.f;
  if (*err == hipSuccess) *err = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

}  // namespace

extern "C" {

int lbmd_autotune(lbmd* c, const char* cache_path, int32_t* out_lb_blocks,
                  int32_t* out_part_blocks, int32_t* out_couple_lanes) {
  if (!c) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->subs != 0 || c->rec_part) return LBMD_ESTATE;
  const std::string key = tune_key(c);
  auto cache = read_cache(cache_path);
  auto hit = cache.find(key);
  if (hit != cache.end()) {
    c->tune.lb_blocks = hit->second.lb_blocks;
    c->tune.part_blocks = hit->second.part_blocks;
    c->tune.couple_lanes = hit->second.couple_lanes;
  } else {
    hipError_t e = hipSuccess;
    int cu = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cu = 256;
    // LB kernels: blocks in flight of the collide-stream kernel, timed on
    // its own (writes only the spare population buffer; at an LB-step
    // boundary no transfer is pending)
    const int lb_cand[5] = {0, 4 * cu, 8 * cu, 16 * cu, 32 * cu};
    double best = 1e30;
    int best_lb = 0;
    for (int q : lb_cand) {
      c->tune.lb_blocks = q;
      const double ms = time_ms(c, [&] { return launch_collide_stream(c); }, 3, &e);
      if (e != hipSuccess) return fail(c, e);
      if (ms < best) {
        best = ms;
        best_lb = q;
      }
    }
    c->tune.lb_blocks = best_lb;
    int best_part = 0, best_lanes = 0;
    if (c->plan.Ntot > 0 && c->bound) {
      const Layout& L = c->plan.lay;
      const size_t S = (size_t)c->plan.Stot, N = (size_t)c->plan.Ntot;
      const size_t t = c->plan.prec == 32 ? 4 : 8;
      // the particle kernels' grid, timed on the corner refill (reads
      // particle positions; writes the cache and the claims only)
      const int part_cand[5] = {0, 2 * cu, 4 * cu, 8 * cu, 16 * cu};
      best = 1e30;
      for (int q : part_cand) {
        c->tune.part_blocks = q;
        const double ms = time_ms(c, [&] { return launch_couple_refill_only(c); }, 3, &e);
        if (e != hipSuccess) return fail(c, e);
        if (ms < best) {
          best = ms;
          best_part = q;
        }
      }
      c->tune.part_blocks = best_part;
      // lanes per particle of the coupling kernel, timed on whole MD steps
      // (coupling kernel + after-step work) from a fresh refill; the
      // particles move, so their state is saved in the sort scratch and put
      // back afterwards (force models 0 and 1: nothing else depends on it)
      bool movable = true;
      for (int r = 0; r < c->plan.R; ++r) movable = movable && c->p[r].force_model <= 1;
      if (movable) {
        int32_t flags_saved[16];
        e = hipMemcpyAsync(flags_saved, at(c, L.flags), sizeof(flags_saved),
                           hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(at(c, L.sort_x), c->x, 3 * N * 8,
                                                hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(at(c, L.sort_v), c->v, 3 * N * 8,
                                                hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(at(c, L.sort_img), c->img, 3 * N * 4,
                                                hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(c, e);
        int cand[4];
        const int nc = couple_lane_candidates(c->p[0].stencil, cand);
        best = 1e30;
        for (int k = 0; k < nc && e == hipSuccess; ++k) {
          c->tune.couple_lanes = cand[k];
          e = hipMemsetAsync(at(c, L.transfer), 0, S * 4 * t, c->stream);
          if (e == hipSuccess) e = hipMemsetAsync(at(c, L.mark), 0, (S / 64) * 8, c->stream);
          if (e == hipSuccess) e = launch_couple_refill_only(c);
          c->cache_dirty = false;
          if (e != hipSuccess) break;
          const double ms = time_ms(c, [&] { return launch_couple(c, 1); }, 3, &e);
          if (e == hipSuccess && ms < best) {
            best = ms;
            best_lanes = cand[k];
          }
        }
        // put the state back: particles, an empty transfer field and marks,
        // the non-finite flags; the cache is refilled at the next MD step
        if (e == hipSuccess) e = hipMemcpyAsync(c->x, at(c, L.sort_x), 3 * N * 8,
                                                hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(c->v, at(c, L.sort_v), 3 * N * 8,
                                                hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(c->img, at(c, L.sort_img), 3 * N * 4,
                                                hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(at(c, L.flags), flags_saved, sizeof(flags_saved),
                                                hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return fail(c, e);
      }
      // the refills left claims (marks, shared flags) of this interval and
      // the trial steps stencil records and stencil-change steps: start it
      // clean
      e = hipMemsetAsync(at(c, L.transfer), 0, S * 4 * t, c->stream);
      if (e == hipSuccess) e = hipMemsetAsync(at(c, L.mark), 0, (S / 64) * 8, c->stream);
      if (e == hipSuccess) e = reset_stencil_records(c);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return fail(c, e);
      c->cache_dirty = true;
    }
    c->tune.part_blocks = best_part;
    c->tune.couple_lanes = best_lanes;
    cache[key] = {c->tune.lb_blocks, c->tune.part_blocks, c->tune.couple_lanes};
    write_cache(cache_path, cache);
  }
  drop_graph(c);
  if (out_lb_blocks) *out_lb_blocks = c->tune.lb_blocks;
  if (out_part_blocks) *out_part_blocks = c->tune.part_blocks;
  if (out_couple_lanes) *out_couple_lanes = c->tune.couple_lanes;
  return LBMD_OK;
}

int lbmd_set_launch_shape(lbmd* c, int32_t lb_blocks, int32_t part_blocks,
                          int32_t couple_lanes) {
  if (!c || lb_blocks < 0 || part_blocks < 0 || couple_lanes < 0) return LBMD_EINVAL;
  if (c->sticky) return c->sticky;
  if (c->subs != 0 || c->rec_part) return LBMD_ESTATE;
  if (couple_lanes > 0) {
    int cand[4];
    const int nc = couple_lane_candidates(c->p[0].stencil, cand);
    bool ok = false;
    for (int k = 0; k < nc; ++k) ok = ok || cand[k] == couple_lanes;
    if (!ok) return LBMD_EINVAL;
  }
  c->tune.lb_blocks = lb_blocks;
  c->tune.part_blocks = part_blocks;
  c->tune.couple_lanes = couple_lanes;
  drop_graph(c);
  return LBMD_OK;
}

int lbmd_stream_copy(void* d_dst, const void* d_src, size_t bytes, void* hip_stream) {
  if (!d_dst || !d_src || bytes % 16 != 0 || ((uintptr_t)d_dst % 16) != 0 ||
      ((uintptr_t)d_src % 16) != 0)
    return LBMD_EINVAL;
  if (bytes == 0) return LBMD_OK;
  return launch_stream_copy(d_dst, d_src, bytes, (hipStream_t)hip_stream) == hipSuccess
             ? LBMD_OK
             : LBMD_EHIP;
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
