// Spatial reordering of the bound particles.
//
// The particle kernels touch, per particle, the populations around its
// stencil (refill), the transfer field at its stencil sites (coupling and
// spreading) and its own state.  With particles stored in random spatial
// order, neighbouring lanes touch unrelated cache lines; stored along a
// space-filling curve, particles that share lines (and rows of lines)
// are processed by the same wavefronts at the same time.  The key is the
// Morton (Z-order) index of the particle's 4 x 4 x 4-site tile below its
// replica index, sorted stably by a device radix sort, so replicas keep
// their particle ranges and equal keys keep their order (the permutation is
// deterministic).  Non-finite particles go to the end of their replica.
// Each slot carries the identity of its particle (its index at binding),
// which the particle noise counter uses: a reordered run draws the same
// noise per particle as one that was never reordered.
#include <hipcub/hipcub.hpp>

#include "particle_geom.hpp"

namespace lbmd_impl {

constexpr int kTileShift = 2;   // 4-site tiles
constexpr int kMortonBits = 12;  // per axis: up to 4096 tiles
constexpr int kKeyBits = 3 * kMortonBits;

__device__ __forceinline__ uint64_t spread_bits3(uint32_t v) {
  uint64_t x = v & 0xFFFu;  // 12 bits -> every third of 36
  x = (x | (x << 16)) & 0x0000FF0000FFull;
  x = (x | (x << 8)) & 0x00F00F00F00Full;
  x = (x | (x << 4)) & 0x0C30C30C30C3ull;
  x = (x | (x << 2)) & 0x249249249249ull;
  return x;
}

__global__ __launch_bounds__(kBlock) void k_sort_keys(const double* __restrict__ x, int64_t N,
                                                      const RepMD* __restrict__ md,
                                                      const int32_t* __restrict__ part_rep,
                                                      uint64_t* __restrict__ keys,
                                                      int32_t* __restrict__ idx) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const uint64_t rep = (uint64_t)part_rep[p];
  uint64_t key = (rep << kKeyBits) | ((1ull << kKeyBits) - 1ull);
  const double X[3] = {x[p], x[N + p], x[2 * N + p]};
  if (isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2])) {
    const RepMD& m = md[rep];
    const int n3[3] = {m.g.nx, m.g.ny, m.g.nz};
    uint32_t t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) t[d] = (uint32_t)(cell_of((int)floor(X[d]), n3[d]) >> kTileShift);
    key = (rep << kKeyBits) | spread_bits3(t[0]) | (spread_bits3(t[1]) << 1) |
          (spread_bits3(t[2]) << 2);
  }
  keys[p] = key;
  idx[p] = (int32_t)p;
}

// New order t takes old particle perm[t]: gather into scratch.
__global__ __launch_bounds__(kBlock) void k_permute_gather(const int32_t* __restrict__ perm,
                                                           int64_t N,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ v,
                                                           const int32_t* __restrict__ img,
                                                           const int32_t* __restrict__ pid,
                                                           double* __restrict__ xs,
                                                           double* __restrict__ vs,
                                                           int32_t* __restrict__ is,
                                                           int32_t* __restrict__ ps) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= N) return;
  const int64_t p = perm[t];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xs[d * N + t] = x[d * N + p];
    vs[d * N + t] = v[d * N + p];
    is[d * N + t] = img[d * N + p];
  }
  ps[t] = pid[p];
}

// Particle identities at binding: the replica-local index.
__global__ __launch_bounds__(kBlock) void k_init_pid(int64_t N, const RepMD* __restrict__ md,
                                                     const int32_t* __restrict__ part_rep,
                                                     int32_t* __restrict__ pid) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p < N) pid[p] = (int32_t)(p - md[part_rep[p]].part_off);
}

hipError_t launch_init_pid(Context* c) {
  const int64_t N = c->plan.Ntot;
  if (N == 0) return hipSuccess;
  const Layout& L = c->plan.lay;
  hipLaunchKernelGGL(k_init_pid, dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     c->stream, N, (const RepMD*)at(c, L.rep_md),
                     (const int32_t*)at(c, L.part_rep), (int32_t*)at(c, L.pid));
  return hipGetLastError();
}

static int sort_end_bit(int R) {
  int b = 0;
  while ((1 << b) < R) ++b;
  return kKeyBits + b;
}

size_t sort_temp_bytes(int64_t N) {
  // generous bound for the radix sort's temporary storage; the exact need is
  // checked against it when the sort runs
  return (size_t)N * 24 + ((size_t)8 << 20);
}

hipError_t launch_sort_particles(Context* c, int32_t* d_perm, bool* too_small) {
  const int64_t N = c->plan.Ntot;
  *too_small = false;
  if (N == 0) return hipSuccess;
  const Layout& L = c->plan.lay;
  uint64_t* keys = (uint64_t*)at(c, L.sort_keys);
  int32_t* vals = (int32_t*)at(c, L.sort_vals);
  const int blocks = (int)((N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_sort_keys, dim3(blocks), dim3(kBlock), 0, c->stream, (const double*)c->x,
                     N, (const RepMD*)at(c, L.rep_md), (const int32_t*)at(c, L.part_rep), keys,
                     vals);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int end_bit = sort_end_bit(c->plan.R);
  size_t need = 0;
  e = hipcub::DeviceRadixSort::SortPairs(nullptr, need, keys, keys + N, vals, vals + N, (int)N, 0,
                                         end_bit, c->stream);
  if (e != hipSuccess) return e;
  if (need > sort_temp_bytes(N)) {
    *too_small = true;
    return hipSuccess;
  }
  e = hipcub::DeviceRadixSort::SortPairs(at(c, L.sort_temp), need, keys, keys + N, vals,
                                         vals + N, (int)N, 0, end_bit, c->stream);
  if (e != hipSuccess) return e;
  const int32_t* perm = vals + N;
  double* xs = (double*)at(c, L.sort_x);
  double* vs = (double*)at(c, L.sort_v);
  int32_t* is = (int32_t*)at(c, L.sort_img);
  int32_t* ps = (int32_t*)keys;  // the sort keys are no longer needed
  int32_t* pid = (int32_t*)at(c, L.pid);
  hipLaunchKernelGGL(k_permute_gather, dim3(blocks), dim3(kBlock), 0, c->stream, perm, N,
                     (const double*)c->x, (const double*)c->v, (const int32_t*)c->img,
                     (const int32_t*)pid, xs, vs, is, ps);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t nd = 3 * (size_t)N;
  if ((e = hipMemcpyAsync(c->x, xs, nd * 8, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(c->v, vs, nd * 8, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(c->img, is, nd * 4, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(pid, ps, (size_t)N * 4, hipMemcpyDeviceToDevice, c->stream)) !=
          hipSuccess)
    return e;
  if (d_perm &&
      (e = hipMemcpyAsync(d_perm, perm, (size_t)N * 4, hipMemcpyDeviceToDevice, c->stream)) !=
          hipSuccess)
    return e;
  // forces at the reordered positions; the corner cache refills at the next MD step
  return launch_init_forces(c);
}

}  // namespace lbmd_impl
