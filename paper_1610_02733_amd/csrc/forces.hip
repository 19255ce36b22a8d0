// Conservative particle forces F_cons (Eq. 4; they act on the particles
// only) for the bead-spring workload: harmonic bonds between consecutive
// beads of a chain and the purely repulsive WCA potential between all pairs,
// found through a cell list.  Also the counting-sort binning of particles
// into cells (histogram, three-level exclusive scan, scatter).
#include "lbmd_internal.hpp"

namespace lbmd_impl {

// ---------------------------------------------------------------------------
// Binning: cell = floor(x / edge) per axis on each replica's grid of
// nb[0] x nb[1] x nb[2] cells of edge L / nb >= the WCA cut-off; cells of all
// replicas share one global index space (offset cell_off).  Non-finite
// particles go to no cell (they are left out of the force loop).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int local_cell(const double X[3], const RepMD& m) {
  int c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int q = (int)floor(X[d] * m.inv_edge[d]);
    q = q < 0 ? 0 : (q >= m.nb[d] ? m.nb[d] - 1 : q);
    c[d] = q;
  }
  return c[0] + m.nb[0] * (c[1] + m.nb[1] * c[2]);
}

__global__ __launch_bounds__(kBlock) void k_fill_int(int32_t* __restrict__ a, int64_t n, int v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] = v;
}

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
  if (m.force_model != 2 || !(isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2]))) {
    bin[p] = -1;
    return;
  }
  const int c = m.cell_off + local_cell(X, m);
  bin[p] = c;
  rank[p] = atomicAdd(count + c, 1);
}

// Exclusive scan of n ints in three launches: per-block scans (kScanTile
// elements per block), a single-block scan of the tile totals, and the
// add-back.
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

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int32_t* __restrict__ in, int64_t n,
                                                       int32_t* __restrict__ out,
                                                       int32_t* __restrict__ tile_sum) {
  __shared__ int sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
  int v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = base + q < n ? in[base + q] : 0;
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

__global__ __launch_bounds__(kBlock) void k_scan_add(int32_t* __restrict__ out, int64_t n,
                                                     const int32_t* __restrict__ tile_sum) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] += tile_sum[i / kScanTile];
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(const int32_t* __restrict__ bin,
                                                        const int32_t* __restrict__ rank,
                                                        const int32_t* __restrict__ start,
                                                        int64_t N, int32_t* __restrict__ sorted) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const int c = bin[p];
  if (c >= 0) sorted[start[c] + rank[p]] = (int32_t)p;
}

// ---------------------------------------------------------------------------
// Forces: each particle sums its own bond and WCA forces (no atomics; every
// pair is evaluated from both sides, so the pair forces cancel up to
// rounding).  Minimum-image separations.  Force models 0 and 1 give zero or
// the constant f_ext.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double min_image(double d, double L) { return d - L * rint(d / L); }

__global__ __launch_bounds__(kBlock) void k_forces(const double* __restrict__ x,
                                                   double* __restrict__ f, int64_t N,
                                                   const RepMD* __restrict__ md,
                                                   const int32_t* __restrict__ part_rep,
                                                   const int32_t* __restrict__ bin,
                                                   const int32_t* __restrict__ start,
                                                   const int32_t* __restrict__ sorted) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const RepMD& m = md[part_rep[p]];
  double F[3] = {0.0, 0.0, 0.0};
  if (m.force_model == 1) {
    F[0] = m.f_ext[0];
    F[1] = m.f_ext[1];
    F[2] = m.f_ext[2];
  }
  const int c = bin[p];
  if (m.force_model != 2 || c < 0) {
    f[p] = F[0];
    f[N + p] = F[1];
    f[2 * N + p] = F[2];
    return;
  }
  const double X[3] = {x[p], x[N + p], x[2 * N + p]};
  const double rc2 = 1.2599210498948732 * m.wca_sigma * m.wca_sigma;  // (2^(1/6) sigma)^2
  const double sig2 = m.wca_sigma * m.wca_sigma;
  // harmonic bonds to the chain neighbours
  const int pos = (int)((p - m.part_off) % m.chain_len);
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    if ((side == 0 && pos == 0) || (side == 1 && pos == m.chain_len - 1)) continue;
    const int64_t q = side == 0 ? p - 1 : p + 1;
    double dx[3], r2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      dx[d] = min_image(X[d] - x[d * N + q], m.L[d]);
      r2 += dx[d] * dx[d];
    }
    const double r = sqrt(r2);
    const double fm = -m.k_bond * (r - m.r0_bond) / r;
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] += fm * dx[d];
  }
  // WCA over the 27 neighbouring cells (distinct cells only on grids < 3 wide)
  const int lc = c - m.cell_off;
  const int cz = lc / (m.nb[0] * m.nb[1]);
  const int cy = (lc / m.nb[0]) % m.nb[1];
  const int cx = lc % m.nb[0];
  const int wz = m.nb[2] < 3 ? m.nb[2] : 3, wy = m.nb[1] < 3 ? m.nb[1] : 3,
            wx = m.nb[0] < 3 ? m.nb[0] : 3;
  for (int oz = 0; oz < wz; ++oz) {
    int zz = m.nb[2] < 3 ? oz : cz + oz - 1;
    zz = zz < 0 ? zz + m.nb[2] : (zz >= m.nb[2] ? zz - m.nb[2] : zz);
    for (int oy = 0; oy < wy; ++oy) {
      int yy = m.nb[1] < 3 ? oy : cy + oy - 1;
      yy = yy < 0 ? yy + m.nb[1] : (yy >= m.nb[1] ? yy - m.nb[1] : yy);
      for (int ox = 0; ox < wx; ++ox) {
        int xx = m.nb[0] < 3 ? ox : cx + ox - 1;
        xx = xx < 0 ? xx + m.nb[0] : (xx >= m.nb[0] ? xx - m.nb[0] : xx);
        const int cell = m.cell_off + xx + m.nb[0] * (yy + m.nb[1] * zz);
        for (int s = start[cell]; s < start[cell + 1]; ++s) {
          const int q = sorted[s];
          if (q == p) continue;
          double dx[3], r2 = 0.0;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            dx[d] = min_image(X[d] - x[d * N + q], m.L[d]);
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
    }
  }
  f[p] = F[0];
  f[N + p] = F[1];
  f[2 * N + p] = F[2];
}

// Second half-kick of velocity Verlet with the new conservative force and
// the coupling force held over the step (replicas with force model 2).
__global__ __launch_bounds__(kBlock) void k_kick(double* __restrict__ v, const double* __restrict__ f,
                                                 const double* __restrict__ fc, int64_t N,
                                                 const RepMD* __restrict__ md,
                                                 const int32_t* __restrict__ part_rep) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const RepMD& m = md[part_rep[p]];
  if (!m.split_kick) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double vv = v[d * N + p];
    if (isfinite(vv)) v[d * N + p] = vv + m.h * (f[d * N + p] + fc[d * N + p]);
  }
}

int64_t force_cells(const lbmd_params* p) {
  if (p->force_model != 2) return 0;
  const double rc = std::pow(2.0, 1.0 / 6.0) * p->wca_sigma;
  const int L[3] = {p->nx, p->ny, p->nz};
  int64_t n = 1;
  for (int d = 0; d < 3; ++d) {
    int q = (int)std::floor((double)L[d] / rc);
    n *= q < 1 ? 1 : q;
  }
  return n;
}

// Conservative forces at the current positions (all force models).
hipError_t launch_forces(Context* c) {
  const int64_t N = c->plan.Ntot;
  if (N == 0) return hipSuccess;
  const Layout& L = c->plan.lay;
  const int pb = (int)((N + kBlock - 1) / kBlock);
  const RepMD* md = (const RepMD*)at(c, L.rep_md);
  const int32_t* prep = (const int32_t*)at(c, L.part_rep);
  int32_t* bin = (int32_t*)at(c, L.bin_of);
  int32_t* start = (int32_t*)at(c, L.bin_start);
  int32_t* sorted = (int32_t*)at(c, L.bin_sorted);
  hipError_t e;
  if (c->plan.any_forces2) {
    int32_t* count = (int32_t*)at(c, L.bin_count);
    int32_t* tiles = (int32_t*)at(c, L.bin_tiles);
    int32_t* rank = (int32_t*)at(c, L.bin_rank);
    const int64_t n = c->plan.Ctot;
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       c->stream, count, n, 0);
    hipLaunchKernelGGL(k_bin_count, dim3(pb), dim3(kBlock), 0, c->stream, (const double*)c->x, N,
                       md, prep, count, bin, rank);
    const int ntiles = (int)((n + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kBlock), 0, c->stream, count, n, start,
                       tiles);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, c->stream, tiles, ntiles, start + n);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       c->stream, start, n, tiles);
    hipLaunchKernelGGL(k_bin_scatter, dim3(pb), dim3(kBlock), 0, c->stream, bin, rank, start, N,
                       sorted);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_fill_int, dim3(pb), dim3(kBlock), 0, c->stream, bin, N, -1);
  }
  hipLaunchKernelGGL(k_forces, dim3(pb), dim3(kBlock), 0, c->stream, (const double*)c->x,
                     (double*)at(c, L.fcons), N, md, prep, bin, start, sorted);
  return hipGetLastError();
}

// Forces at the bound positions; the corner cache is stale from here on.
hipError_t launch_init_forces(Context* c) {
  hipError_t e = launch_forces(c);
  if (e != hipSuccess) return e;
  return invalidate_corner_cache(c);
}

// Forces at the new positions, then the second half-kick.
hipError_t launch_forces_and_kick(Context* c) {
  hipError_t e = launch_forces(c);
  if (e != hipSuccess) return e;
  const int64_t N = c->plan.Ntot;
  const Layout& L = c->plan.lay;
  hipLaunchKernelGGL(k_kick, dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     c->stream, (double*)c->v, (const double*)at(c, L.fcons),
                     (const double*)at(c, L.fc_held), N, (const RepMD*)at(c, L.rep_md),
                     (const int32_t*)at(c, L.part_rep));
  return hipGetLastError();
}

}  // namespace lbmd_impl
