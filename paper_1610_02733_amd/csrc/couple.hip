// Particle coupling kernels (Sec. 3, Eq. 4-8): fluid velocity at the
// particle by interpolation over the 8 sites of its cube, friction plus
// noise, velocity Verlet, and transfer of -dP to the same 8 sites with the
// same weights.
#include "lbmd_internal.hpp"

namespace lbmd_impl {
using namespace lbmd_dev;

template <typename T>
struct CoupleArgs {
  T* __restrict__ x;
  T* __restrict__ v;
  int32_t* __restrict__ img;
  const T* __restrict__ fcons;
  const T* __restrict__ pop;
  Vec4<T>* __restrict__ J;
  unsigned long long* __restrict__ mark;
  int32_t* __restrict__ rec_cell;
  T* __restrict__ rec_frac;
  T* __restrict__ rec_dp;
  int32_t* __restrict__ flags;
  Geom g;
  int N;
  T rho0, gamma, amp, tau, h;  // h = tau / (2 m)
  T L[3];
  uint32_t key0, key1, step_lo, step_hi, tag;
  int variant;
  int noise;
};

// Periodic wrap with image counting; a value that lands on exactly L after
// adding L stays at 0 in its old image.
template <typename T>
__device__ __forceinline__ void wrap_coord(T& x, int32_t& im, T L) {
  if (x >= L) {
    x -= L;
    im += 1;
  } else if (x < T(0)) {
    x += L;
    im -= 1;
    if (x >= L) {
      x -= L;
      im += 1;
    }
  }
}

// Integer cube corner from a coordinate, kept inside [0, n) whatever the
// input (the coupling always addresses valid sites).
__device__ __forceinline__ int cell_of(int c, int n) {
  c %= n;
  return c < 0 ? c + n : c;
}

template <typename T>
__device__ __forceinline__ void corner_weights(const T s[3], T w[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const T a = (k & 1) ? s[0] : T(1) - s[0];
    const T b = (k & 2) ? s[1] : T(1) - s[1];
    const T cc = (k & 4) ? s[2] : T(1) - s[2];
    w[k] = a * b * cc;
  }
}

__device__ __forceinline__ void corner_sites(const Geom& g, const int base[3], int site[8],
                                             int cx[8], int cy[8], int cz[8]) {
  const int x1 = base[0] + 1 == g.nx ? 0 : base[0] + 1;
  const int y1 = base[1] + 1 == g.ny ? 0 : base[1] + 1;
  const int z1 = base[2] + 1 == g.nz ? 0 : base[2] + 1;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    cx[k] = (k & 1) ? x1 : base[0];
    cy[k] = (k & 2) ? y1 : base[1];
    cz[k] = (k & 4) ? z1 : base[2];
    site[k] = cx[k] + g.nx * (cy[k] + g.ny * cz[k]);
  }
}

template <typename T>
__device__ __forceinline__ void transfer(const CoupleArgs<T>& a, const int site[8], const T w[8],
                                         const T dp[3]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    Vec4<T>* q = a.J + site[k];
    atomicAdd(&q->x, -w[k] * dp[0]);
    atomicAdd(&q->y, -w[k] * dp[1]);
    atomicAdd(&q->z, -w[k] * dp[2]);
  }
}

template <typename T>
__device__ __forceinline__ void mark_sites(const CoupleArgs<T>& a, const int site[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k)
    atomicOr(a.mark + (site[k] >> 6), 1ull << (site[k] & 63));
}

// One MD step for one particle.  Variant 1 transfers its momentum right
// away (nothing in this MD step reads J); variant 2 stores (cube, weights
// source, dP) for the spreading kernel, because every particle must first
// read the velocities as of the end of the previous MD step.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_couple(CoupleArgs<T> a) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= a.N) return;
  const int N = a.N;
  T X[3], V[3];
  bool finite = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    X[d] = a.x[d * N + p];
    V[d] = a.v[d * N + p];
    finite = finite && isfinite(X[d]) && isfinite(V[d]);
  }
  if (!finite) {
    a.flags[0] = 1;
    if (a.variant == 2) a.rec_cell[p] = -1;
    return;
  }
  int base[3];
  T s[3];
  const int n3[3] = {a.g.nx, a.g.ny, a.g.nz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T fl = floor(X[d]);
    s[d] = X[d] - fl;
    base[d] = cell_of((int)fl, n3[d]);
  }
  int site[8], cx[8], cy[8], cz[8];
  corner_sites(a.g, base, site, cx, cy, cz);
  T w[8];
  corner_weights<T>(s, w);

  // fluid velocity at the particle (Eq. 5) from the post-stream state
  const size_t S = (size_t)a.g.S;
  T u[3] = {T(0), T(0), T(0)};
#pragma unroll 1
  for (int k = 0; k < 8; ++k) {
    int src[19];
    pull_sources(a.g, cx[k], cy[k], cz[k], src);
    T d[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = a.pop[(size_t)i * S + src[i]];
    T drho, jx, jy, jz;
    moments_deviation<T>(d, drho, jx, jy, jz);
    if (a.variant == 2) {
      const Vec4<T> jv = a.J[site[k]];
      jx += jv.x;
      jy += jv.y;
      jz += jv.z;
    }
    const T inv = T(1) / (a.rho0 + drho);
    u[0] += w[k] * (jx * inv);
    u[1] += w[k] * (jy * inv);
    u[2] += w[k] * (jz * inv);
  }

  // friction + noise (Eq. 4), momentum change over the MD step (Eq. 6)
  T xi[3] = {T(0), T(0), T(0)};
  if (a.noise) {
    const Words4 o = philox10(Words4{(uint32_t)p, a.step_lo, a.tag, a.step_hi}, a.key0, a.key1);
    const uint32_t ws[3] = {o.w0, o.w1, o.w2};
#pragma unroll
    for (int d = 0; d < 3; ++d)
      xi[d] = T(3.4641016151377546) *
              (((T)(int)(ws[d] >> 8) + T(0.5)) * T(5.9604644775390625e-08) - T(0.5));
  }
  T Fc[3], dp[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    Fc[d] = -a.gamma * (V[d] - u[d]) + a.amp * xi[d];
    dp[d] = a.tau * Fc[d];
  }

  // velocity Verlet with the coupling force held over the step; the
  // conservative force of force models 0/1 does not depend on position
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T fc = a.fcons[d * N + p];
    int32_t im = a.img[d * N + p];
    V[d] += a.h * (fc + Fc[d]);
    X[d] += a.tau * V[d];
    wrap_coord<T>(X[d], im, a.L[d]);
    V[d] += a.h * (fc + Fc[d]);
    a.x[d * N + p] = X[d];
    a.v[d * N + p] = V[d];
    a.img[d * N + p] = im;
  }

  // momentum transfer to the fluid (Eq. 7-8)
  mark_sites<T>(a, site);
  if (a.variant == 1) {
    transfer<T>(a, site, w, dp);
  } else {
    a.rec_cell[p] = base[0];
    a.rec_cell[N + p] = base[1];
    a.rec_cell[2 * N + p] = base[2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      a.rec_frac[d * N + p] = s[d];
      a.rec_dp[d * N + p] = dp[d];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_spread(CoupleArgs<T> a) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= a.N) return;
  const int N = a.N;
  const int base[3] = {a.rec_cell[p], a.rec_cell[N + p], a.rec_cell[2 * N + p]};
  if (base[0] < 0) return;
  T s[3], dp[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    s[d] = a.rec_frac[d * N + p];
    dp[d] = a.rec_dp[d * N + p];
  }
  int site[8], cx[8], cy[8], cz[8];
  corner_sites(a.g, base, site, cx, cy, cz);
  T w[8];
  corner_weights<T>(s, w);
  transfer<T>(a, site, w, dp);
}

template <typename T>
static CoupleArgs<T> couple_args(Context* c) {
  CoupleArgs<T> a;
  const int N = c->p.n_particles;
  a.x = (T*)c->x;
  a.v = (T*)c->v;
  a.img = c->img;
  a.fcons = (const T*)at(c, c->lay.fcons);
  a.pop = (const T*)at(c, c->lay.pop[c->cur]);
  a.J = (Vec4<T>*)at(c, c->lay.transfer);
  a.mark = (unsigned long long*)at(c, c->lay.mark);
  a.rec_cell = (int32_t*)at(c, c->lay.rec_cell);
  a.rec_frac = (T*)at(c, c->lay.rec_frac);
  a.rec_dp = (T*)at(c, c->lay.rec_dp);
  a.flags = (int32_t*)at(c, c->lay.flags);
  a.g = c->geom;
  a.N = N;
  const double tau = 1.0 / c->p.n_sub;
  a.rho0 = (T)c->p.rho0;
  a.gamma = (T)c->p.friction;
  a.amp = (T)std::sqrt(2.0 * c->p.friction * c->p.kT / tau);
  a.tau = (T)tau;
  a.h = (T)(tau / (2.0 * c->p.particle_mass));
  a.L[0] = (T)c->p.nx;
  a.L[1] = (T)c->p.ny;
  a.L[2] = (T)c->p.nz;
  a.key0 = (uint32_t)(c->p.seed & 0xFFFFFFFFu);
  a.key1 = (uint32_t)(c->p.seed >> 32);
  a.step_lo = (uint32_t)((uint64_t)c->t_md & 0xFFFFFFFFu);
  a.step_hi = (uint32_t)((uint64_t)c->t_md >> 32);
  a.tag = noise_tag(kPurposeParticle, c->p.replica, 0);
  a.variant = c->p.variant;
  a.noise = (c->p.kT > 0.0 && c->p.friction > 0.0) ? 1 : 0;
  return a;
}

template <typename T>
static hipError_t couple_t(Context* c) {
  CoupleArgs<T> a = couple_args<T>(c);
  const int blocks = (a.N + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_couple<T>, dim3(blocks), dim3(kBlock), 0, c->stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.variant == 1) return e;
  hipLaunchKernelGGL(k_spread<T>, dim3(blocks), dim3(kBlock), 0, c->stream, a);
  return hipGetLastError();
}

hipError_t launch_couple(Context* c) {
  if (c->p.n_particles == 0) return hipSuccess;
  return c->p.precision == 32 ? couple_t<float>(c) : couple_t<double>(c);
}

// Conservative forces at the bound positions (force models 0 and 1).
template <typename T>
__global__ void k_const_force(T* __restrict__ f, int N, T fx, T fy, T fz) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  f[p] = fx;
  f[N + p] = fy;
  f[2 * N + p] = fz;
}

template <typename T>
static hipError_t init_forces_t(Context* c) {
  const int N = c->p.n_particles;
  const bool cst = c->p.force_model == 1;
  const int blocks = (N + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_const_force<T>, dim3(blocks), dim3(kBlock), 0, c->stream,
                     (T*)at(c, c->lay.fcons), N, (T)(cst ? c->p.f_ext[0] : 0.0),
                     (T)(cst ? c->p.f_ext[1] : 0.0), (T)(cst ? c->p.f_ext[2] : 0.0));
  return hipGetLastError();
}

hipError_t launch_init_forces(Context* c) {
  if (c->p.n_particles == 0) return hipSuccess;
  return c->p.precision == 32 ? init_forces_t<float>(c) : init_forces_t<double>(c);
}

}  // namespace lbmd_impl
