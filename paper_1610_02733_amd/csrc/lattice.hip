// Lattice kernels: the fused pull collide-and-stream step (Eq. 3 with the
// MRT collision, fluid noise and Guo forcing of Sec. 2-3), the FP64 moment
// reductions (Eq. 1-2) and population / transfer copies.
#include "lbmd_internal.hpp"

namespace lbmd_impl {
using namespace lbmd_dev;

// ---------------------------------------------------------------------------
// Fused collide-and-stream, one thread per site, pull scheme.
//
// The source buffer holds post-collision deviations at the site that produced
// them; the thread at site r gathers buffer[i][r - c_i] (the post-stream
// state), adds the pending momentum transfer J(r) as the force density of
// this LB step, collides and writes its 19 results at r in the other buffer
// (coalesced).  J is only read where the site's bit in `mark` is set (the
// coupling sets it when it transfers momentum there), and is cleared with it,
// so the untouched bulk of the lattice costs no transfer traffic.  Threads
// map linearly onto sites, so one wavefront owns exactly one 64-bit mark word.
// ---------------------------------------------------------------------------
template <typename T>
struct StreamArgs {
  const T* __restrict__ src;
  T* __restrict__ dst;
  Vec4<T>* __restrict__ J;
  unsigned long long* __restrict__ mark;
  Geom g;
  uint32_t key0, key1, step_lo, step_hi, tag0, tag1;
  CollideConsts<T> k;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_collide_stream(StreamArgs<T> a) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= a.g.S) return;
  const unsigned long long word = a.mark[r >> 6];
  int x, y, z;
  site_coords(a.g, r, x, y, z);
  int src[19];
  pull_sources(a.g, x, y, z, src);
  const size_t S = (size_t)a.g.S;
  // every population is read once per step: non-temporal loads keep the
  // stream from evicting the transfer field and the mark words
  T d[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) d[i] = __builtin_nontemporal_load(a.src + (size_t)i * S + src[i]);

  T Fx = a.k.g[0], Fy = a.k.g[1], Fz = a.k.g[2];
  if ((word >> (r & 63)) & 1ull) {
    const Vec4<T> jv = a.J[r];
    Fx += jv.x;
    Fy += jv.y;
    Fz += jv.z;
    a.J[r] = Vec4<T>{T(0), T(0), T(0), T(0)};
  }
  uint32_t hw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (a.k.noise) {
    const Words4 o0 = philox10(Words4{(uint32_t)r, a.step_lo, a.tag0, a.step_hi}, a.key0, a.key1);
    const Words4 o1 = philox10(Words4{(uint32_t)r, a.step_lo, a.tag1, a.step_hi}, a.key0, a.key1);
    hw[0] = o0.w0; hw[1] = o0.w1; hw[2] = o0.w2; hw[3] = o0.w3;
    hw[4] = o1.w0; hw[5] = o1.w1; hw[6] = o1.w2; hw[7] = o1.w3;
  }
  collide_deviation<T>(d, Fx, Fy, Fz, hw, a.k);
  // every population is written once per step: stream the stores past the
  // caches (non-temporal hint)
#pragma unroll
  for (int i = 0; i < 19; ++i) __builtin_nontemporal_store(d[i], a.dst + (size_t)i * S + r);
  if ((r & 63) == 0 && word) a.mark[r >> 6] = 0ull;
}

template <typename T>
static CollideConsts<T> make_consts(const Context* c) {
  CollideConsts<T> k;
  k.rho0 = (T)c->p.rho0;
  k.gs = (T)c->gs;
  k.gb = (T)c->gb;
  k.gg = (T)c->gg;
  k.hs = (T)(0.5 * (1.0 + c->gs));
  k.hb = (T)(0.5 * (1.0 + c->gb));
  k.mu = (T)c->mu;
  for (int v = 0; v < 15; ++v) k.ns[v] = (T)c->ns[v];
  for (int d = 0; d < 3; ++d) k.g[d] = (T)c->p.body_force[d];
  k.noise = c->p.kT > 0.0 ? 1 : 0;
  return k;
}

template <typename T>
static hipError_t collide_stream_t(Context* c) {
  StreamArgs<T> a;
  a.src = (const T*)at(c, c->lay.pop[c->cur]);
  a.dst = (T*)at(c, c->lay.pop[1 - c->cur]);
  a.J = (Vec4<T>*)at(c, c->lay.transfer);
  a.mark = (unsigned long long*)at(c, c->lay.mark);
  a.g = c->geom;
  a.key0 = (uint32_t)(c->p.seed & 0xFFFFFFFFu);
  a.key1 = (uint32_t)(c->p.seed >> 32);
  a.step_lo = (uint32_t)((uint64_t)c->t_lb & 0xFFFFFFFFu);
  a.step_hi = (uint32_t)((uint64_t)c->t_lb >> 32);
  a.tag0 = noise_tag(kPurposeFluid, c->p.replica, 0);
  a.tag1 = noise_tag(kPurposeFluid, c->p.replica, 1);
  a.k = make_consts<T>(c);
  const int blocks = (int)((c->S + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_collide_stream<T>, dim3(blocks), dim3(kBlock), 0, c->stream, a);
  return hipGetLastError();
}

hipError_t launch_collide_stream(Context* c) {
  return c->p.precision == 32 ? collide_stream_t<float>(c) : collide_stream_t<double>(c);
}

// ---------------------------------------------------------------------------
// Block reduction of kRedWidth doubles per thread into partials[blockIdx].
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_reduce_store(double acc[kRedWidth], double* out) {
  __shared__ double sh[kBlock / 64][kRedWidth];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kRedWidth; ++q) {
    double s = acc[q];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) sh[wv][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < kRedWidth) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += sh[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// Columns: 0 sum drho, 1-3 sum j, 4-6 sum J, 7 sum |j/rho|^2, 8-10 sum v,
// 11 sum |v|^2 (mass applied on the host).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_moments(const T* __restrict__ pop,
                                                    const Vec4<T>* __restrict__ J, Geom g, T rho0,
                                                    T* __restrict__ rho_out, T* __restrict__ u_out,
                                                    const double* __restrict__ v, int N,
                                                    double* __restrict__ partials) {
  double acc[kRedWidth];
#pragma unroll
  for (int q = 0; q < kRedWidth; ++q) acc[q] = 0.0;
  const size_t S = (size_t)g.S;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < g.S; r += gridDim.x * kBlock) {
    int x, y, z, src[19];
    site_coords(g, r, x, y, z);
    pull_sources(g, x, y, z, src);
    T d[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = pop[(size_t)i * S + src[i]];
    T drho, jx, jy, jz;
    moments_deviation<T>(d, drho, jx, jy, jz);
    const T rho = rho0 + drho;
    const T ux = jx / rho, uy = jy / rho, uz = jz / rho;
    if (rho_out) rho_out[r] = rho;
    if (u_out) {
      u_out[r] = ux;
      u_out[S + r] = uy;
      u_out[2 * S + r] = uz;
    }
    const Vec4<T> jv = J[r];
    acc[0] += (double)drho;
    acc[1] += (double)jx;
    acc[2] += (double)jy;
    acc[3] += (double)jz;
    acc[4] += (double)jv.x;
    acc[5] += (double)jv.y;
    acc[6] += (double)jv.z;
    const double dux = (double)jx / (double)rho, duy = (double)jy / (double)rho,
                 duz = (double)jz / (double)rho;
    acc[7] += dux * dux + duy * duy + duz * duz;
  }
  if (v) {
    for (int p = blockIdx.x * kBlock + threadIdx.x; p < N; p += gridDim.x * kBlock) {
      const double a = v[p], b = v[N + p], cc = v[2 * N + p];
      acc[8] += a;
      acc[9] += b;
      acc[10] += cc;
      acc[11] += a * a + b * b + cc * cc;
    }
  }
  block_reduce_store(acc, partials + (size_t)blockIdx.x * kRedWidth);
}

__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ partials,
                                                     int nblocks, double* __restrict__ totals) {
  double acc[kRedWidth];
#pragma unroll
  for (int q = 0; q < kRedWidth; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock)
#pragma unroll
    for (int q = 0; q < kRedWidth; ++q) acc[q] += partials[(size_t)b * kRedWidth + q];
  block_reduce_store(acc, totals);
}

template <typename T>
static hipError_t moments_t(Context* c, void* d_rho, void* d_u, double* d_totals) {
  const int blocks = (int)std::min<int64_t>(kRedBlocks, (c->S + kBlock - 1) / kBlock);
  double* partials = (double*)at(c, c->lay.partials);
  hipLaunchKernelGGL(k_moments<T>, dim3(blocks), dim3(kBlock), 0, c->stream,
                     (const T*)at(c, c->lay.pop[c->cur]), (const Vec4<T>*)at(c, c->lay.transfer),
                     c->geom, (T)c->p.rho0, (T*)d_rho, (T*)d_u,
                     (const double*)(c->bound ? c->v : nullptr), c->p.n_particles, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !d_totals) return e;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, c->stream, partials, blocks, d_totals);
  return hipGetLastError();
}

hipError_t launch_moments(Context* c, void* d_rho, void* d_u, double* d_totals) {
  return c->p.precision == 32 ? moments_t<float>(c, d_rho, d_u, d_totals)
                              : moments_t<double>(c, d_rho, d_u, d_totals);
}

// ---------------------------------------------------------------------------
// Copies between pull storage and the plain post-stream layout.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_get_pop(const T* __restrict__ pop, Geom g,
                                                    T* __restrict__ out) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= g.S) return;
  int x, y, z, src[19];
  site_coords(g, r, x, y, z);
  pull_sources(g, x, y, z, src);
  const size_t S = (size_t)g.S;
#pragma unroll
  for (int i = 0; i < 19; ++i) out[(size_t)i * S + r] = pop[(size_t)i * S + src[i]];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_pop(T* __restrict__ pop, Geom g,
                                                    const T* __restrict__ in) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= g.S) return;
  int x, y, z, src[19];
  site_coords(g, r, x, y, z);
  pull_sources(g, x, y, z, src);
  const size_t S = (size_t)g.S;
#pragma unroll
  for (int i = 0; i < 19; ++i) pop[(size_t)i * S + src[i]] = in[(size_t)i * S + r];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_get_transfer(const Vec4<T>* __restrict__ J, int S,
                                                         T* __restrict__ out) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= S) return;
  const Vec4<T> jv = J[r];
  out[r] = jv.x;
  out[(size_t)S + r] = jv.y;
  out[2 * (size_t)S + r] = jv.z;
}

template <typename T>
static hipError_t copy_t(Context* c, void* dst, const void* src, int what) {
  const int blocks = (int)((c->S + kBlock - 1) / kBlock);
  T* pop = (T*)at(c, c->lay.pop[c->cur]);
  if (what == 0)
    hipLaunchKernelGGL(k_get_pop<T>, dim3(blocks), dim3(kBlock), 0, c->stream, pop, c->geom,
                       (T*)dst);
  else if (what == 1)
    hipLaunchKernelGGL(k_set_pop<T>, dim3(blocks), dim3(kBlock), 0, c->stream, pop, c->geom,
                       (const T*)src);
  else
    hipLaunchKernelGGL(k_get_transfer<T>, dim3(blocks), dim3(kBlock), 0, c->stream,
                       (const Vec4<T>*)at(c, c->lay.transfer), c->geom.S, (T*)dst);
  return hipGetLastError();
}

hipError_t launch_get_populations(Context* c, void* dst) {
  return c->p.precision == 32 ? copy_t<float>(c, dst, nullptr, 0) : copy_t<double>(c, dst, nullptr, 0);
}
hipError_t launch_set_populations(Context* c, const void* src) {
  return c->p.precision == 32 ? copy_t<float>(c, nullptr, src, 1) : copy_t<double>(c, nullptr, src, 1);
}
hipError_t launch_get_transfer(Context* c, void* dst) {
  return c->p.precision == 32 ? copy_t<float>(c, dst, nullptr, 2) : copy_t<double>(c, dst, nullptr, 2);
}

}  // namespace lbmd_impl
