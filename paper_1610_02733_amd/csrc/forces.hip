// Conservative particle forces F_cons (Eq. 4; they act on the particles
// only) for the bead-spring workloads, with pairs found through a cell list:
// model 2, harmonic bonds between consecutive beads of a chain and the purely
// repulsive WCA potential between all pairs; model 3, the paper's
// Kremer-Grest polymer (Sec. 3), FENE bonds and the Lennard-Jones potential
// cut at 2^(7/6) sigma.  Also the binning of particles into cells.
#include <algorithm>
#include <cmath>

#include "couple_state.hpp"

namespace lbmd_impl {

// ---------------------------------------------------------------------------
// Binning: cell = floor(x / edge) per axis on each replica's grid of
// nb[0] x nb[1] x nb[2] cells of edge L / nb >= the pair cut-off (local_cell);
// cells of all replicas share one global index space (offset cell_off).
// Non-finite particles go to no cell (they are left out of the force loop).
// A cell holds up to cell_cap particles in slots of its own, taken in the
// order of an atomic count; the rest go to an overflow list (cell_insert).
// After an MD step the coupling kernel bins the particles (it knows the new
// positions first) and clears the other half of the counts (bin_parity), so
// the force kernel follows it directly.  At bound positions both halves are
// cleared and k_bin_count bins the particles.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bin_clear(int32_t* __restrict__ count, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) count[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_bin_count(const double* __restrict__ x, int64_t N,
                                                      const RepMD* __restrict__ md,
                                                      const int32_t* __restrict__ part_rep,
                                                      const Clock* __restrict__ clock,
                                                      int pos_step, int64_t ncells, int cap,
                                                      int32_t* __restrict__ count,
                                                      int32_t* __restrict__ bin,
                                                      int32_t* __restrict__ slot,
                                                      int32_t* __restrict__ ovf) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const int par = bin_parity(clock, pos_step);
  const double X[3] = {x[p], x[N + p], x[2 * N + p]};
  const RepMD& m = md[part_rep[p]];
  if (m.force_model < 2 || !(isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2]))) {
    bin[p] = -1;
    return;
  }
  const int c = m.cell_off + local_cell(X, m);
  bin[p] = (int32_t)(par * ncells + c);
  cell_insert(count + par * ncells, slot, ovf, count + 2 * ncells + par, cap, c, (int)p);
}

// ---------------------------------------------------------------------------
// Forces: each particle sums its own bond and WCA forces (no atomics; every
// pair is evaluated from both sides, so the pair forces cancel up to
// rounding), with minimum-image separations.  Force models 0 and 1 give zero
// or the constant f_ext.
//
// 32 lanes per particle: lanes 0-26 scan the slots of one neighbouring cell
// each (offsets -1, 0, +1 per axis; on an axis with fewer than 3 cells,
// cells 0, 1, 2 of that axis instead, so every distinct cell is scanned
// once), lane 27 adds the two chain bonds, lane 28 scans the overflow list
// (empty unless a cell holds more than cell_cap particles; a pair closer
// than the cut-off lies in neighbouring cells, so the list's particles need
// only the distance test); the lane sums are a butterfly reduction.  The
// half of the counts comes with the particle's own count entry.  Lane 0
// stores the force and, after an MD step, applies the second half-kick of
// velocity Verlet (new conservative force + the coupling force held over the
// step).  After an MD step the launch also carries the step's after-step
// work in extra blocks: this kernel runs after every particle of the step
// has read the transfer field.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double min_image(double d, double L) { return d - L * rint(d / L); }

constexpr int kForceLanes = 32;

__device__ __forceinline__ double lane32_sum(double v) {
  v += __shfl_xor(v, 16, kForceLanes);
  v += __shfl_xor(v, 8, kForceLanes);
  v += __shfl_xor(v, 4, kForceLanes);
  v += __shfl_xor(v, 2, kForceLanes);
  v += __shfl_xor(v, 1, kForceLanes);
  return v;
}

template <typename T>
struct ForceArgs {
  const double* __restrict__ x;
  double* __restrict__ v;
  double* __restrict__ f;
  const double* __restrict__ fc_held;
  const RepMD* __restrict__ md;
  const int32_t* __restrict__ part_rep;
  const int32_t* __restrict__ count;  // [2][ncells] + [2] overflow lengths (CoupleArgs::bin_count)
  const int32_t* __restrict__ bin;    // [N] count entries (CoupleArgs::bin)
  const int32_t* __restrict__ slot;
  const int32_t* __restrict__ ovf;
  int64_t N;
  int64_t ncells;
  int cap;
};

// Pair force of the WCA or cut Lennard-Jones potential on the particle at X
// from particle q, added to F when q lies within the cut-off.
__device__ __forceinline__ void add_pair_force(const double* __restrict__ x, int64_t N,
                                               const double X[3], int q, const RepMD& m,
                                               double rc2, double sig2, double F[3]) {
  double dx[3], r2 = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    dx[d] = min_image(X[d] - x[d * N + q], m.L[d]);
    r2 += dx[d] * dx[d];
  }
  if (r2 >= rc2) return;
  const double sr2 = sig2 / r2;
  const double sr6 = sr2 * sr2 * sr2;
  const double fm = 24.0 * m.wca_eps * (2.0 * sr6 * sr6 - sr6) / r2;
#pragma unroll
  for (int d = 0; d < 3; ++d) F[d] += fm * dx[d];
}

// Blocks [0, nfb) compute the forces; with AfterST >= 0 (after an MD step,
// not recording) blocks [nfb, nfb + 2 nseg) do the after-step work
// of the MD step just taken (after_step_item), which is independent of the
// forces: it touches J, the claims and the corner cache only.
// One (a single replica): its constants are read once, before the loop
// (uniform, scalar loads), so the particle's loads need not wait for them.
// The loads of a particle are issued together where they do not depend on
// each other: its cell, position and (lane 0) velocity and held coupling
// force; a cell's count with its first two slots; the two bond partners.
template <typename T, bool Kick, int AfterST, bool One>
__global__ __launch_bounds__(kBlock) void k_forces(ForceArgs<T> a, CoupleArgs<T> ca, int64_t nseg,
                                                   int per, int L, int64_t nfb) {
  if constexpr (AfterST >= 0) {
    if (blockIdx.x >= nfb) {
      after_step_item<T, AfterST, false, false>(ca, (int64_t)blockIdx.x - nfb, nseg, per, L);
      return;
    }
  }
  const int64_t N = a.N;
  RepMD m1;
  if constexpr (One) m1 = a.md[0];
  // lanes come in whole particles (32 | kBlock), as the shuffles require
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < N * kForceLanes;
       t += nfb * kBlock) {
    const int64_t p = t / kForceLanes;
    const int lane = (int)(t & (kForceLanes - 1));
    RepMD mr;
    if constexpr (!One) mr = a.md[a.part_rep[p]];
    const RepMD& m = One ? m1 : mr;
    double F[3] = {0.0, 0.0, 0.0};
    // (the cells are written for every particle when a replica has them)
    const int g = m.force_model >= 2 ? a.bin[p] : -1;
    const double X[3] = {a.x[p], a.x[N + p], a.x[2 * N + p]};
    const bool kick = Kick && lane == 0 && m.split_kick;
    double vv[3] = {0.0, 0.0, 0.0}, fh[3] = {0.0, 0.0, 0.0};
    if (kick) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        vv[d] = a.v[d * N + p];
        fh[d] = a.fc_held[d * N + p];
      }
    }
    if (g >= 0) {
      const int half = g >= a.ncells ? 1 : 0;
      const int c = g - (half ? (int)a.ncells : 0);
      const int32_t* __restrict__ cnt = a.count + half * a.ncells;
      // pair cut-off squared: (2^(1/6) sigma)^2 (WCA) or (2^(7/6) sigma)^2
      const double rc2 = (m.force_model == 2 ? 1.2599210498948732 : 5.0396841995794928) *
                         m.wca_sigma * m.wca_sigma;
      const double sig2 = m.wca_sigma * m.wca_sigma;
      if (lane < 27) {
        const int o[3] = {lane % 3, (lane / 3) % 3, lane / 9};
        const int lc = c - m.cell_off;
        const int cc[3] = {lc % m.nb[0], (lc / m.nb[0]) % m.nb[1], lc / (m.nb[0] * m.nb[1])};
        int q3[3];
        bool use = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          if (m.nb[d] < 3) {
            q3[d] = o[d];
            use = use && o[d] < m.nb[d];
          } else {
            const int qq = cc[d] + o[d] - 1;
            q3[d] = qq < 0 ? qq + m.nb[d] : (qq >= m.nb[d] ? qq - m.nb[d] : qq);
          }
        }
        if (use) {
          const int cell = m.cell_off + q3[0] + m.nb[0] * (q3[1] + m.nb[1] * q3[2]);
          const int32_t* __restrict__ sl = a.slot + (int64_t)cell * a.cap;
          // the count and the first two slots at once (cap >= 2; a slot past
          // the count holds a stale index, replaced by p and not used)
          const int n = min(cnt[cell], a.cap);
          const int s0 = sl[0], s1 = sl[1];
          const int q0 = n > 0 ? s0 : (int)p, q1 = n > 1 ? s1 : (int)p;
          double F0[3] = {0.0, 0.0, 0.0}, F1[3] = {0.0, 0.0, 0.0};
          add_pair_force(a.x, N, X, q0, m, rc2, sig2, F0);
          add_pair_force(a.x, N, X, q1, m, rc2, sig2, F1);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            if (q0 != p) F[d] += F0[d];
            if (q1 != p) F[d] += F1[d];
          }
          for (int s = 2; s < n; ++s) {
            const int q = sl[s];
            if (q != p) add_pair_force(a.x, N, X, q, m, rc2, sig2, F);
          }
        }
      } else if (lane == 27) {
        // bonds to the chain neighbours: harmonic (model 2) or FENE (model 3,
        // no finite force at r >= R0); both partners' positions at once
        const int pos = (int)((p - m.part_off) % m.chain_len);
        const bool has[2] = {pos > 0, pos < m.chain_len - 1};
        const int64_t qs[2] = {has[0] ? p - 1 : p, has[1] ? p + 1 : p};
        double dx[2][3], r2[2] = {0.0, 0.0};
#pragma unroll
        for (int side = 0; side < 2; ++side)
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            dx[side][d] = min_image(X[d] - a.x[d * N + qs[side]], m.L[d]);
            r2[side] += dx[side][d] * dx[side][d];
          }
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          if (!has[side]) continue;
          double fm;
          if (m.force_model == 2) {
            const double r = sqrt(r2[side]);
            fm = -m.k_bond * (r - m.r0_bond) / r;
          } else {
            const double x2 = r2[side] / (m.r0_bond * m.r0_bond);
            fm = x2 < 1.0 ? -m.k_bond / (1.0 - x2) : __builtin_nan("");
          }
#pragma unroll
          for (int d = 0; d < 3; ++d) F[d] += fm * dx[side][d];
        }
      } else if (lane == 28) {
        const int no = a.count[2 * a.ncells + half];
        const int rep = a.part_rep[p];
        for (int e = 0; e < no; ++e) {
          const int q = a.ovf[e];
          if (q != p && a.part_rep[q] == rep) add_pair_force(a.x, N, X, q, m, rc2, sig2, F);
        }
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] = lane32_sum(F[d]);
    if (lane == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (m.force_model == 1) F[d] = m.f_ext[d];
        a.f[d * N + p] = F[d];
        if (kick && isfinite(vv[d])) a.v[d * N + p] = vv[d] + m.h * (F[d] + fh[d]);
      }
    }
  }
}

// Force cells per axis: edge just above the pair cut-off (2^(1/6) sigma for
// WCA, 2^(7/6) sigma for the Kremer-Grest model), so the 27 neighbouring
// cells hold every interacting pair.  Larger cells (about one
// particle per cell on average) were measured slower on chains: a chain's
// beads then crowd a few cells and the per-lane cell loops serialise.
int cells_per_axis(const lbmd_params* p, int d) {
  const double rc = std::pow(2.0, p->force_model == 3 ? 7.0 / 6.0 : 1.0 / 6.0) * p->wca_sigma;
  const int L[3] = {p->nx, p->ny, p->nz};
  const int q = (int)std::floor((double)L[d] / rc);
  return q < 1 ? 1 : q;
}

int64_t force_cells(const lbmd_params* p) {
  if (p->force_model < 2) return 0;
  int64_t n = 1;
  for (int d = 0; d < 3; ++d) n *= cells_per_axis(p, d);
  return n;
}

// Particle slots per force cell.  A WCA cell (edge ~1.12 sigma, ~1.4
// sigma^3) holds about one bead even at melt density; a Kremer-Grest cell
// (edge ~2.24 sigma, ~11 sigma^3) holds about ten there.  Particles past the
// capacity are still found, through the overflow list, at a cost per pair.
int force_cell_capacity(const lbmd_params* p) {
  if (p->force_model < 2) return 0;
  return p->force_model == 3 ? 32 : 8;
}

template <typename T>
static ForceArgs<T> force_args(Context* c) {
  const Layout& L = c->plan.lay;
  ForceArgs<T> a;
  a.x = (const double*)c->x;
  a.v = (double*)c->v;
  a.f = (double*)at(c, L.fcons);
  a.fc_held = (const double*)at(c, L.fc_held);
  a.md = (const RepMD*)at(c, L.rep_md);
  a.part_rep = (const int32_t*)at(c, L.part_rep);
  a.count = (const int32_t*)at(c, L.bin_count);
  a.bin = (const int32_t*)at(c, L.bin_of);
  a.slot = (const int32_t*)at(c, L.bin_slot);
  a.ovf = (const int32_t*)at(c, L.bin_ovf);
  a.N = c->plan.Ntot;
  a.ncells = c->plan.Ctot;
  a.cap = c->plan.cell_cap;
  return a;
}

// Bin the particles of bead-spring replicas (models 2, 3) at the current
// positions, those of MD step clock->t_md + pos_step, from scratch: both
// halves of the counts are cleared first (a fill kernel, so the sequence
// may be captured in a graph).
static hipError_t launch_binning(Context* c, int pos_step) {
  const int64_t N = c->plan.Ntot, C = c->plan.Ctot;
  const Layout& L = c->plan.lay;
  int32_t* count = (int32_t*)at(c, L.bin_count);
  const int64_t nc = 2 * C + 2;
  hipLaunchKernelGGL(k_bin_clear, dim3((unsigned)((nc + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     c->stream, count, nc);
  hipLaunchKernelGGL(k_bin_count, dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     c->stream, (const double*)c->x, N, (const RepMD*)at(c, L.rep_md),
                     (const int32_t*)at(c, L.part_rep), (const Clock*)at(c, L.clock), pos_step,
                     C, c->plan.cell_cap, count, (int32_t*)at(c, L.bin_of),
                     (int32_t*)at(c, L.bin_slot), (int32_t*)at(c, L.bin_ovf));
  return hipGetLastError();
}

template <typename T, bool Kick, int AfterST>
static hipError_t forces_t(Context* c, int substep = 0) {
  const ForceArgs<T> a = force_args<T>(c);
  const int64_t nfb = (a.N * kForceLanes + kBlock - 1) / kBlock;
  CoupleArgs<T> ca{};
  int64_t nseg = 0;
  int per = 0, L = 0;
  if (AfterST >= 0) {
    constexpr int ST = AfterST >= 0 ? AfterST : 0;
    ca = couple_args<T>(c, substep);
    // the coupling kernel's lanes per particle (tuned or default)
    L = c->tune.couple_lanes > 0 ? c->tune.couple_lanes : DirectShape<ST>::kLanes;
    per = (Stencil<ST>::kSites + L - 1) / L;
    nseg = (a.N * L + kBlock - 1) / kBlock;
  }
  const dim3 grid((unsigned)(nfb + 2 * nseg));
  if (c->plan.R == 1)
    hipLaunchKernelGGL((k_forces<T, Kick, AfterST, true>), grid, dim3(kBlock), 0, c->stream, a,
                       ca, nseg, per, L, nfb);
  else
    hipLaunchKernelGGL((k_forces<T, Kick, AfterST, false>), grid, dim3(kBlock), 0, c->stream, a,
                       ca, nseg, per, L, nfb);
  return hipGetLastError();
}

// Conservative forces at the current positions (all force models).
hipError_t launch_forces(Context* c) {
  if (c->plan.Ntot == 0) return hipSuccess;
  hipError_t e;
  if (c->plan.any_forces2 && (e = launch_binning(c, c->subs)) != hipSuccess) return e;
  return c->plan.prec == 32 ? forces_t<float, false, -1>(c) : forces_t<double, false, -1>(c);
}

// Forces at the bound positions; the corner cache is stale from here on.
hipError_t launch_init_forces(Context* c) {
  hipError_t e = launch_forces(c);
  if (e != hipSuccess) return e;
  return invalidate_corner_cache(c);
}

// After an MD step of replicas with position-dependent forces: forces at
// the new positions (binned by the coupling kernel, or here while
// recording), the second half-kick and the step's after-step work in the
// same launch (so the coupling step launches no after-step kernel of its
// own).
template <typename T>
static hipError_t forces_and_kick_t(Context* c, int substep) {
  if (c->rec_part) return forces_t<T, true, -1>(c, substep);
  return c->p[0].stencil == 1 ? forces_t<T, true, 1>(c, substep)
                              : forces_t<T, true, 0>(c, substep);
}

hipError_t launch_forces_and_kick(Context* c, int substep) {
  if (c->plan.Ntot == 0) return hipSuccess;
  if (c->rec_part) {
    const hipError_t e = launch_binning(c, substep + 1);
    if (e != hipSuccess) return e;
  }
  return c->plan.prec == 32 ? forces_and_kick_t<float>(c, substep)
                            : forces_and_kick_t<double>(c, substep);
}

}  // namespace lbmd_impl
