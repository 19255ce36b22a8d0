// Conservative particle forces F_cons (Eq. 4; they act on the particles
// only) for the bead-spring workloads, with pairs found through a cell list:
// model 2, harmonic bonds between consecutive beads of a chain and the purely
// repulsive WCA potential between all pairs; model 3, the paper's
// Kremer-Grest polymer (Sec. 3), FENE bonds and the Lennard-Jones potential
// cut at 2^(7/6) sigma.  Also the counting-sort binning of particles
// into cells (histogram, three-level exclusive scan, scatter).
#include <algorithm>
#include <cmath>

#include "couple_state.hpp"

namespace lbmd_impl {

// ---------------------------------------------------------------------------
// Binning: cell = floor(x / edge) per axis on each replica's grid of
// nb[0] x nb[1] x nb[2] cells of edge L / nb >= the pair cut-off (local_cell);
// cells of all replicas share one global index space (offset cell_off).
// Non-finite particles go to no cell (they are left out of the force loop).
// After an MD step the coupling kernel has already counted the particles
// into their cells (it knows the new positions first), so only the scan and
// the scatter follow; k_bin_count serves the binning at bound positions.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bin_count(const double* __restrict__ x, int64_t N,
                                                      const RepMD* __restrict__ md,
                                                      const int32_t* __restrict__ part_rep,
                                                      int32_t* __restrict__ count,
                                                      int32_t* __restrict__ bin,
                                                      int32_t* __restrict__ rank) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const double X[3] = {x[p], x[N + p], x[2 * N + p]};
  const RepMD& m = md[part_rep[p]];
  if (m.force_model < 2 || !(isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2]))) {
    bin[p] = -1;
    return;
  }
  const int c = m.cell_off + local_cell(X, m);
  bin[p] = c;
  rank[p] = atomicAdd(count + c, 1);
}

// Exclusive scan of the n cell counts in two launches: per-block scans
// (kScanTile cells per block, which also reset the counts) and a single-block
// scan of the tile totals.  The start of cell c is then the in-tile scan plus
// its tile's offset (bin_begin); the total sits at index n.  (Folding the
// second launch into the first with a last-block counter needs a device-wide
// fence in every block, which on this multi-die part costs far more than the
// launch.)
constexpr int kScanTile = 1024;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int incl = sh[t];
  return incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(int32_t* __restrict__ in, int64_t n,
                                                       int32_t* __restrict__ out,
                                                       int32_t* __restrict__ tile_sum) {
  __shared__ int sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
  int v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[q] = base + q < n ? in[base + q] : 0;
    if (base + q < n) in[base + q] = 0;  // counts start from zero at the next binning
  }
  const int tsum = v[0] + v[1] + v[2] + v[3];
  int run = block_exclusive_scan(tsum, sh);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (base + q < n) out[base + q] = run;
    run += v[q];
  }
  if (threadIdx.x == kBlock - 1) tile_sum[blockIdx.x] = run;
}

__global__ __launch_bounds__(kBlock) void k_scan_top(int32_t* __restrict__ tile_sum, int ntiles,
                                                     int32_t* __restrict__ total) {
  __shared__ int sh[kBlock];
  // each thread scans a contiguous chunk, then the chunk sums are scanned
  const int per = (ntiles + kBlock - 1) / kBlock;
  const int lo = threadIdx.x * per, hi = min(lo + per, ntiles);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += tile_sum[i];
  int run = block_exclusive_scan(s, sh);
  for (int i = lo; i < hi; ++i) {
    const int v = tile_sum[i];
    tile_sum[i] = run;
    run += v;
  }
  if (threadIdx.x == kBlock - 1) *total = run;
}

__device__ __forceinline__ int bin_begin(const int32_t* __restrict__ start,
                                         const int32_t* __restrict__ tiles, int64_t n, int c) {
  return c == n ? start[n] : start[c] + tiles[c / kScanTile];
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(const int32_t* __restrict__ bin,
                                                        const int32_t* __restrict__ rank,
                                                        const int32_t* __restrict__ start,
                                                        const int32_t* __restrict__ tiles,
                                                        int64_t n, int64_t N,
                                                        int32_t* __restrict__ sorted) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const int c = bin[p];
  if (c >= 0) sorted[bin_begin(start, tiles, n, c) + rank[p]] = (int32_t)p;
}

// ---------------------------------------------------------------------------
// Forces: each particle sums its own bond and WCA forces (no atomics; every
// pair is evaluated from both sides, so the pair forces cancel up to
// rounding), with minimum-image separations.  Force models 0 and 1 give zero
// or the constant f_ext.
//
// 32 lanes per particle: lanes 0-26 scan one neighbouring cell each (offsets
// -1, 0, +1 per axis; on an axis with fewer than 3 cells, cells 0, 1, 2 of
// that axis instead, so every distinct cell is scanned once), lane 27 adds
// the two chain bonds; the lane sums are a butterfly reduction.  Lane 0
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
  const int32_t* __restrict__ bin;
  const int32_t* __restrict__ start;
  const int32_t* __restrict__ tiles;
  const int32_t* __restrict__ sorted;
  int64_t N;
  int64_t ncells;
};

// Blocks [0, nfb) compute the forces; with AfterST >= 0 (after an MD step,
// not recording) blocks [nfb, nfb + 2 nseg) do the after-step work
// of the MD step just taken (after_step_item), which is independent of the
// forces: it touches J, the claims and the corner cache only.
template <typename T, bool Kick, int AfterST>
__global__ __launch_bounds__(kBlock) void k_forces(ForceArgs<T> a, CoupleArgs<T> ca, int64_t nseg,
                                                   int per, int L, int64_t nfb) {
  if constexpr (AfterST >= 0) {
    if (blockIdx.x >= nfb) {
      after_step_item<T, AfterST, false, false>(ca, (int64_t)blockIdx.x - nfb, nseg, per, L);
      return;
    }
  }
  const int64_t N = a.N;
  // lanes come in whole particles (32 | kBlock), as the shuffles require
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < N * kForceLanes;
       t += nfb * kBlock) {
    const int64_t p = t / kForceLanes;
    const int lane = (int)(t & (kForceLanes - 1));
    const RepMD& m = a.md[a.part_rep[p]];
    double F[3] = {0.0, 0.0, 0.0};
    const int c = m.force_model >= 2 ? a.bin[p] : -1;
    if (c >= 0) {
      const double X[3] = {a.x[p], a.x[N + p], a.x[2 * N + p]};
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
          const int s1 = bin_begin(a.start, a.tiles, a.ncells, cell + 1);
          for (int s = bin_begin(a.start, a.tiles, a.ncells, cell); s < s1; ++s) {
            const int q = a.sorted[s];
            if (q == p) continue;
            double dx[3], r2 = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              dx[d] = min_image(X[d] - a.x[d * N + q], m.L[d]);
              r2 += dx[d] * dx[d];
            }
            if (r2 >= rc2) continue;
            const double sr2 = sig2 / r2;
            const double sr6 = sr2 * sr2 * sr2;
            const double fm = 24.0 * m.wca_eps * (2.0 * sr6 * sr6 - sr6) / r2;
#pragma unroll
            for (int d = 0; d < 3; ++d) F[d] += fm * dx[d];
          }
        }
      } else if (lane == 27) {
        // bonds to the chain neighbours: harmonic (model 2) or FENE (model 3,
        // no finite force at r >= R0)
        const int pos = (int)((p - m.part_off) % m.chain_len);
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          if ((side == 0 && pos == 0) || (side == 1 && pos == m.chain_len - 1)) continue;
          const int64_t q = side == 0 ? p - 1 : p + 1;
          double dx[3], r2 = 0.0;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            dx[d] = min_image(X[d] - a.x[d * N + q], m.L[d]);
            r2 += dx[d] * dx[d];
          }
          double fm;
          if (m.force_model == 2) {
            const double r = sqrt(r2);
            fm = -m.k_bond * (r - m.r0_bond) / r;
          } else {
            const double x2 = r2 / (m.r0_bond * m.r0_bond);
            fm = x2 < 1.0 ? -m.k_bond / (1.0 - x2) : __builtin_nan("");
          }
#pragma unroll
          for (int d = 0; d < 3; ++d) F[d] += fm * dx[d];
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
        if (Kick && m.split_kick) {
          const double vv = a.v[d * N + p];
          if (isfinite(vv)) a.v[d * N + p] = vv + m.h * (F[d] + a.fc_held[d * N + p]);
        }
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
  a.bin = (const int32_t*)at(c, L.bin_of);
  a.start = (const int32_t*)at(c, L.bin_start);
  a.tiles = (const int32_t*)at(c, L.bin_tiles);
  a.sorted = (const int32_t*)at(c, L.bin_sorted);
  a.N = c->plan.Ntot;
  a.ncells = c->plan.Ctot;
  return a;
}

// Bin the particles of bead-spring replicas (models 2, 3) into their cells.
// counted: the coupling kernel of the MD step already filled count, bin
// and rank.
static hipError_t launch_binning(Context* c, bool counted) {
  const int64_t N = c->plan.Ntot;
  const Layout& L = c->plan.lay;
  const int pb = (int)((N + kBlock - 1) / kBlock);
  int32_t* count = (int32_t*)at(c, L.bin_count);
  int32_t* tiles = (int32_t*)at(c, L.bin_tiles);
  int32_t* rank = (int32_t*)at(c, L.bin_rank);
  int32_t* bin = (int32_t*)at(c, L.bin_of);
  int32_t* start = (int32_t*)at(c, L.bin_start);
  const int64_t n = c->plan.Ctot;
  if (!counted)
    hipLaunchKernelGGL(k_bin_count, dim3(pb), dim3(kBlock), 0, c->stream, (const double*)c->x,
                       N, (const RepMD*)at(c, L.rep_md), (const int32_t*)at(c, L.part_rep), count,
                       bin, rank);
  const int ntiles = (int)((n + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kBlock), 0, c->stream, count, n, start,
                     tiles);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, c->stream, tiles, ntiles, start + n);
  hipLaunchKernelGGL(k_bin_scatter, dim3(pb), dim3(kBlock), 0, c->stream, bin, rank, start, tiles,
                     n, N, (int32_t*)at(c, L.bin_sorted));
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
  hipLaunchKernelGGL((k_forces<T, Kick, AfterST>), grid, dim3(kBlock), 0, c->stream, a, ca, nseg,
                     per, L, nfb);
  return hipGetLastError();
}

// Conservative forces at the current positions (all force models).
hipError_t launch_forces(Context* c) {
  if (c->plan.Ntot == 0) return hipSuccess;
  hipError_t e;
  if (c->plan.any_forces2 && (e = launch_binning(c, false)) != hipSuccess) return e;
  return c->plan.prec == 32 ? forces_t<float, false, -1>(c) : forces_t<double, false, -1>(c);
}

// Forces at the bound positions; the corner cache is stale from here on.
hipError_t launch_init_forces(Context* c) {
  hipError_t e = launch_forces(c);
  if (e != hipSuccess) return e;
  return invalidate_corner_cache(c);
}

// After an MD step of replicas with position-dependent forces: binning,
// forces at the new positions, the second half-kick and the step's
// after-step work in the same launch (so the coupling step launches no
// after-step kernel of its own).
template <typename T>
static hipError_t forces_and_kick_t(Context* c, int substep) {
  if (c->rec_part) return forces_t<T, true, -1>(c, substep);
  return c->p[0].stencil == 1 ? forces_t<T, true, 1>(c, substep)
                              : forces_t<T, true, 0>(c, substep);
}

hipError_t launch_forces_and_kick(Context* c, int substep) {
  if (c->plan.Ntot == 0) return hipSuccess;
  hipError_t e = launch_binning(c, !c->rec_part);
  if (e != hipSuccess) return e;
  return c->plan.prec == 32 ? forces_and_kick_t<float>(c, substep)
                            : forces_and_kick_t<double>(c, substep);
}

}  // namespace lbmd_impl
