// Conservative particle forces F_cons (Eq. 4; they act on the particles
// only) for the bead-spring workload: harmonic bonds between consecutive
// beads of a chain and the purely repulsive WCA potential between all pairs,
// found through a cell list.  Also the counting-sort binning of particles
// into cells (histogram, three-level exclusive scan, scatter).
#include "lbmd_internal.hpp"

namespace lbmd_impl {

// ---------------------------------------------------------------------------
// Binning: cell = floor(x / edge) per axis on a grid of nb[0] x nb[1] x nb[2]
// cells of edge L / nb >= the WCA cut-off.  Non-finite particles go to no
// cell (they are left out of the force loop).
// ---------------------------------------------------------------------------
struct BinGeom {
  int nb[3];
  double inv_edge[3];
  int ncell;
};

__device__ __forceinline__ int bin_of(const double X[3], const BinGeom& b) {
  int c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int q = (int)floor(X[d] * b.inv_edge[d]);
    q = q < 0 ? 0 : (q >= b.nb[d] ? b.nb[d] - 1 : q);
    c[d] = q;
  }
  return c[0] + b.nb[0] * (c[1] + b.nb[1] * c[2]);
}

__global__ __launch_bounds__(kBlock) void k_fill_int(int32_t* __restrict__ a, int n, int v) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_bin_count(const double* __restrict__ x, int N, BinGeom b,
                                                      int32_t* __restrict__ count,
                                                      int32_t* __restrict__ bin,
                                                      int32_t* __restrict__ rank) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const double X[3] = {x[p], x[N + p], x[2 * N + p]};
  if (!(isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2]))) {
    bin[p] = -1;
    return;
  }
  const int c = bin_of(X, b);
  bin[p] = c;
  rank[p] = atomicAdd(count + c, 1);
}

// Exclusive scan of n ints in three launches: per-block scans (kScanTile
// elements per block), a single-block scan of the tile totals, and the
// add-back.
constexpr int kScanTile = 1024;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh) {
  // kBlock threads, each holding the sum of 4 consecutive elements
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

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int32_t* __restrict__ in, int n,
                                                       int32_t* __restrict__ out,
                                                       int32_t* __restrict__ tile_sum) {
  __shared__ int sh[kBlock];
  const int base = blockIdx.x * kScanTile + threadIdx.x * 4;
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

__global__ __launch_bounds__(kBlock) void k_scan_add(int32_t* __restrict__ out, int n,
                                                     const int32_t* __restrict__ tile_sum) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] += tile_sum[i / kScanTile];
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(const int32_t* __restrict__ bin,
                                                        const int32_t* __restrict__ rank,
                                                        const int32_t* __restrict__ start, int N,
                                                        int32_t* __restrict__ sorted) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const int c = bin[p];
  if (c >= 0) sorted[start[c] + rank[p]] = p;
}

// ---------------------------------------------------------------------------
// Forces: each particle sums its own bond and WCA forces (no atomics; every
// pair is evaluated from both sides, so the pair forces cancel up to
// rounding).  Minimum-image separations.
// ---------------------------------------------------------------------------
struct ForceArgs {
  const double* __restrict__ x;
  double* __restrict__ f;
  const int32_t* __restrict__ bin;
  const int32_t* __restrict__ start;  // [ncell + 1] (last = particles binned)
  const int32_t* __restrict__ sorted;
  int N, chain_len;
  BinGeom b;
  double L[3];
  double k_bond, r0, eps, sig2, rc2;
};

__device__ __forceinline__ double min_image(double d, double L) { return d - L * rint(d / L); }

__global__ __launch_bounds__(kBlock) void k_forces(ForceArgs a) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= a.N) return;
  const int N = a.N;
  const double X[3] = {a.x[p], a.x[N + p], a.x[2 * N + p]};
  double F[3] = {0.0, 0.0, 0.0};
  const int c = a.bin[p];
  if (c < 0) {
    a.f[p] = a.f[N + p] = a.f[2 * N + p] = 0.0;
    return;
  }
  // harmonic bonds to the chain neighbours
  const int pos = p % a.chain_len;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int q = side == 0 ? p - 1 : p + 1;
    if ((side == 0 && pos == 0) || (side == 1 && pos == a.chain_len - 1)) continue;
    double dx[3], r2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      dx[d] = min_image(X[d] - a.x[d * N + q], a.L[d]);
      r2 += dx[d] * dx[d];
    }
    const double r = sqrt(r2);
    const double fm = -a.k_bond * (r - a.r0) / r;
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] += fm * dx[d];
  }
  // WCA over the 27 neighbouring cells (distinct cells only on grids < 3 wide)
  const int cz = c / (a.b.nb[0] * a.b.nb[1]);
  const int cy = (c / a.b.nb[0]) % a.b.nb[1];
  const int cx = c % a.b.nb[0];
  const int nz = a.b.nb[2] < 3 ? a.b.nb[2] : 3, ny = a.b.nb[1] < 3 ? a.b.nb[1] : 3,
            nx = a.b.nb[0] < 3 ? a.b.nb[0] : 3;
  for (int oz = 0; oz < nz; ++oz) {
    int zz = a.b.nb[2] < 3 ? oz : cz + oz - 1;
    zz = zz < 0 ? zz + a.b.nb[2] : (zz >= a.b.nb[2] ? zz - a.b.nb[2] : zz);
    for (int oy = 0; oy < ny; ++oy) {
      int yy = a.b.nb[1] < 3 ? oy : cy + oy - 1;
      yy = yy < 0 ? yy + a.b.nb[1] : (yy >= a.b.nb[1] ? yy - a.b.nb[1] : yy);
      for (int ox = 0; ox < nx; ++ox) {
        int xx = a.b.nb[0] < 3 ? ox : cx + ox - 1;
        xx = xx < 0 ? xx + a.b.nb[0] : (xx >= a.b.nb[0] ? xx - a.b.nb[0] : xx);
        const int cell = xx + a.b.nb[0] * (yy + a.b.nb[1] * zz);
        for (int s = a.start[cell]; s < a.start[cell + 1]; ++s) {
          const int q = a.sorted[s];
          if (q == p) continue;
          double dx[3], r2 = 0.0;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            dx[d] = min_image(X[d] - a.x[d * N + q], a.L[d]);
            r2 += dx[d] * dx[d];
          }
          if (r2 >= a.rc2) continue;
          const double sr2 = a.sig2 / r2;
          const double sr6 = sr2 * sr2 * sr2;
          const double fm = 24.0 * a.eps * (2.0 * sr6 * sr6 - sr6) / r2;
#pragma unroll
          for (int d = 0; d < 3; ++d) F[d] += fm * dx[d];
        }
      }
    }
  }
  a.f[p] = F[0];
  a.f[N + p] = F[1];
  a.f[2 * N + p] = F[2];
}

// Second half-kick of velocity Verlet with the new conservative force and
// the coupling force held over the step.
__global__ __launch_bounds__(kBlock) void k_kick(double* __restrict__ v, const double* __restrict__ f,
                                                 const double* __restrict__ fc, int N, double h) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double vv = v[d * N + p];
    if (isfinite(vv)) v[d * N + p] = vv + h * (f[d * N + p] + fc[d * N + p]);
  }
}

static BinGeom bin_geom(const Context* c) {
  BinGeom b;
  const double rc = std::pow(2.0, 1.0 / 6.0) * c->p.wca_sigma;
  const int L[3] = {c->p.nx, c->p.ny, c->p.nz};
  b.ncell = 1;
  for (int d = 0; d < 3; ++d) {
    int n = (int)std::floor((double)L[d] / rc);
    n = n < 1 ? 1 : n;
    b.nb[d] = n;
    b.inv_edge[d] = (double)n / (double)L[d];
    b.ncell *= n;
  }
  return b;
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

__global__ void k_const_force(double* __restrict__ f, int N, double fx, double fy, double fz) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  f[p] = fx;
  f[N + p] = fy;
  f[2 * N + p] = fz;
}

// Conservative forces at the current positions (all force models).
hipError_t launch_forces(Context* c) {
  const int N = c->p.n_particles;
  if (N == 0) return hipSuccess;
  const int pb = (N + kBlock - 1) / kBlock;
  double* f = (double*)at(c, c->lay.fcons);
  hipError_t e;
  if (c->p.force_model != 2) {
    const bool cst = c->p.force_model == 1;
    hipLaunchKernelGGL(k_const_force, dim3(pb), dim3(kBlock), 0, c->stream, f, N,
                       cst ? c->p.f_ext[0] : 0.0, cst ? c->p.f_ext[1] : 0.0,
                       cst ? c->p.f_ext[2] : 0.0);
    return hipGetLastError();
  }
  const BinGeom b = bin_geom(c);
  int32_t* count = (int32_t*)at(c, c->lay.bin_count);
  int32_t* start = (int32_t*)at(c, c->lay.bin_start);
  int32_t* tiles = (int32_t*)at(c, c->lay.bin_tiles);
  int32_t* bin = (int32_t*)at(c, c->lay.bin_of);
  int32_t* rank = (int32_t*)at(c, c->lay.bin_rank);
  int32_t* sorted = (int32_t*)at(c, c->lay.bin_sorted);
  const int n = b.ncell;
  hipLaunchKernelGGL(k_fill_int, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, c->stream,
                     count, n, 0);
  hipLaunchKernelGGL(k_bin_count, dim3(pb), dim3(kBlock), 0, c->stream, (const double*)c->x, N,
                     b, count, bin, rank);
  const int ntiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kBlock), 0, c->stream, count, n, start, tiles);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, c->stream, tiles, ntiles, start + n);
  hipLaunchKernelGGL(k_scan_add, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, c->stream,
                     start, n, tiles);
  hipLaunchKernelGGL(k_bin_scatter, dim3(pb), dim3(kBlock), 0, c->stream, bin, rank, start, N,
                     sorted);
  ForceArgs a;
  a.x = (const double*)c->x;
  a.f = f;
  a.bin = bin;
  a.start = start;
  a.sorted = sorted;
  a.N = N;
  a.chain_len = c->p.chain_len;
  a.b = b;
  a.L[0] = c->p.nx;
  a.L[1] = c->p.ny;
  a.L[2] = c->p.nz;
  a.k_bond = c->p.k_bond;
  a.r0 = c->p.r0_bond;
  a.eps = c->p.wca_eps;
  a.sig2 = c->p.wca_sigma * c->p.wca_sigma;
  a.rc2 = std::pow(2.0, 1.0 / 3.0) * a.sig2;
  hipLaunchKernelGGL(k_forces, dim3(pb), dim3(kBlock), 0, c->stream, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipSuccess;
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
  const int N = c->p.n_particles;
  const double h = 1.0 / c->p.n_sub / (2.0 * c->p.particle_mass);
  hipLaunchKernelGGL(k_kick, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, c->stream,
                     (double*)c->v, (const double*)at(c, c->lay.fcons),
                     (const double*)at(c, c->lay.fc_held), N, h);
  return hipGetLastError();
}

}  // namespace lbmd_impl
