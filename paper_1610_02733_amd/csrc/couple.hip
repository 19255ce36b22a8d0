// Particle coupling kernels (Sec. 3, Eq. 4-8): fluid velocity at the
// particle by interpolation over the sites of its stencil (the 8 sites of
// its cube, or 27 with the three-point kernel), friction plus noise,
// velocity Verlet, and transfer of -dP to the same sites with the same
// weights.  Particles of all replicas in one launch; each particle reads its
// replica's constants.  Kernels are templated on the stencil (ST, see
// particle_geom.hpp); the adjoint exists for the trilinear one only.
#include <algorithm>

#include "particle_geom.hpp"

namespace lbmd_impl {
using namespace lbmd_dev;

// T is the lattice precision (populations, transfer field, corner cache);
// particle state and all particle arithmetic are FP64 in both precisions.
template <typename T>
struct CoupleArgs {
  double* __restrict__ x;
  double* __restrict__ v;
  int32_t* __restrict__ img;
  const double* __restrict__ fcons;
  T* pop[2];
  Vec4<T>* __restrict__ J;
  unsigned long long* __restrict__ mark;
  int32_t* __restrict__ rec_cell;
  double* __restrict__ rec_frac;
  double* __restrict__ rec_dp;
  double* __restrict__ fc_held;  // coupling force of the step (split kick)
  T* __restrict__ cc;
  int32_t* __restrict__ cc_cell;
  int32_t* __restrict__ cc_stamp;
  unsigned long long* __restrict__ shared_site;  // sites claimed more than once this interval
  int32_t* __restrict__ flags;
  const RepMD* __restrict__ md;
  const int32_t* __restrict__ part_rep;
  const int32_t* __restrict__ pid;  // particle identity of each slot (noise counter)
  const Clock* __restrict__ clock;
  double* __restrict__ rec;  // recording: [kAdjRec][N] state and corner velocities of the step
  size_t P;     // population stride
  int64_t N;    // particles over all replicas
  int substep;  // MD step inside the LB interval
  int variant;
  int single;   // one replica: its constants are uniform across the grid
};

// Cache entry k of particle p: (jx, jy, jz, 1/rho) of stencil site k.
template <int ST = 0, typename T>
__device__ __forceinline__ Vec4<T>* cache_entry(const CoupleArgs<T>& a, int64_t p, int k) {
  return reinterpret_cast<Vec4<T>*>(a.cc) + (size_t)p * Stencil<ST>::kSites + k;
}

__device__ __forceinline__ int cache_stamp(const Clock* clk) {
  return (int)(((unsigned long long)clk->t_lb & 0x3FFFFFFFull) + 1);
}

// Mark a site as a receiver of momentum transfer in this LB interval; a site
// claimed again (by another particle, or by one that changed cubes) is
// flagged as shared.
template <typename T>
__device__ __forceinline__ void claim_site(const CoupleArgs<T>& a, int gs) {
  const unsigned long long bit = 1ull << (gs & 63);
  if (atomicOr(a.mark + (gs >> 6), bit) & bit) atomicOr(a.shared_site + (gs >> 6), bit);
}

// ---------------------------------------------------------------------------
// Corner-cache refill, once per LB interval (before its first MD step):
// (j, 1/rho) of the post-stream state at the 8 corners of every particle's
// cube.  32 lanes per particle, 4 per corner, which split the corner's 19
// pulled populations; the state does not change until the next LB step, so
// the MD steps of the interval read 8 contiguous vectors per particle instead
// of 8 x 19 scattered populations.  Also marks the 8 sites as receivers of
// momentum transfer for the LB step.
// ---------------------------------------------------------------------------
constexpr int kRefillLanes = 32;

template <typename T>
__device__ __forceinline__ T quad_sum(T v) {  // over the 4 lanes of a corner
  v += __shfl_xor(v, 1, kRefillLanes);
  v += __shfl_xor(v, 2, kRefillLanes);
  return v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_refill(CoupleArgs<T> a) {
  const T* __restrict__ pop = a.pop[a.clock->cur];
  const int stamp = cache_stamp(a.clock);
  const int64_t lanes = a.N * kRefillLanes;
  // lanes come in whole particles (32 | kBlock), so a particle's lanes stay
  // together in every iteration
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < lanes;
       t += (int64_t)gridDim.x * kBlock) {
    const int64_t p = t / kRefillLanes;
    const int sl = threadIdx.x & (kRefillLanes - 1);
    const int k = sl >> 2, c = sl & 3;
    const RepMD& m = a.md[a.single ? 0 : a.part_rep[p]];
    const int64_t N = a.N;
    double X[3];
    bool finite = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      X[d] = a.x[d * N + p];
      finite = finite && isfinite(X[d]);
    }
    if (!finite) continue;
    Cube q;
    cube_of(X, m.g, q);
    int cx, cy, cz, site;
    double w;
    corner_of(q, m.g, k, cx, cy, cz, site, w);
    T drho = T(0), qx = T(0), qy = T(0), qz = T(0);
#pragma unroll
    for (int mm = 0; mm < 5; ++mm) {
      const int i = c + 4 * mm;
      if (i < 19) {
        const int ex = kVel[i][0], ey = kVel[i][1], ez = kVel[i][2];
        int sx = cx - ex, sy = cy - ey, sz = cz - ez;
        sx = sx < 0 ? sx + m.g.nx : (sx >= m.g.nx ? sx - m.g.nx : sx);
        sy = sy < 0 ? sy + m.g.ny : (sy >= m.g.ny ? sy - m.g.ny : sy);
        sz = sz < 0 ? sz + m.g.nz : (sz >= m.g.nz ? sz - m.g.nz : sz);
        const T d = pop[(size_t)i * a.P + m.site_off + sx + m.g.nx * (sy + m.g.ny * sz)];
        drho += d;
        qx += (T)ex * d;
        qy += (T)ey * d;
        qz += (T)ez * d;
      }
    }
    drho = quad_sum(drho);
    qx = quad_sum(qx);
    qy = quad_sum(qy);
    qz = quad_sum(qz);
    const T mine = c == 0 ? qx : (c == 1 ? qy : (c == 2 ? qz : T(1) / ((T)m.rho0 + drho)));
    a.cc[(size_t)p * 32 + sl] = mine;
    if (sl == 0) {
      a.cc_cell[p] = q.base[0] + m.g.nx * (q.base[1] + m.g.ny * q.base[2]);
      a.cc_stamp[p] = stamp;
    }
    if (c == 0) claim_site(a, m.site_off + site);
  }
}

// The same refill for the three-point stencil: 32 lanes per particle, lane k
// < 27 gathers the 19 pulled populations of stencil site k itself.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_refill3(CoupleArgs<T> a) {
  const T* __restrict__ pop = a.pop[a.clock->cur];
  const int stamp = cache_stamp(a.clock);
  const int64_t lanes = a.N * 32;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < lanes;
       t += (int64_t)gridDim.x * kBlock) {
    const int64_t p = t / 32;
    const int k = (int)(t & 31);
    if (k >= Stencil<1>::kSites) continue;
    const RepMD& m = a.md[a.single ? 0 : a.part_rep[p]];
    const int64_t N = a.N;
    double X[3];
    bool finite = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      X[d] = a.x[d * N + p];
      finite = finite && isfinite(X[d]);
    }
    if (!finite) continue;
    Cube q;
    Stencil<1>::locate(X, m.g, q);
    int cx, cy, cz, site;
    double w;
    Stencil<1>::site(q, m.g, k, cx, cy, cz, site, w);
    int sidx[19];
    pull_sources(m.g, cx, cy, cz, sidx);
    T d[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = pop[(size_t)i * a.P + m.site_off + sidx[i]];
    T drho, jx, jy, jz;
    moments_deviation<T>(d, drho, jx, jy, jz);
    *cache_entry<1>(a, p, k) = Vec4<T>{jx, jy, jz, T(1) / ((T)m.rho0 + drho)};
    if (k == 0) {
      a.cc_cell[p] = q.base[0] + m.g.nx * (q.base[1] + m.g.ny * q.base[2]);
      a.cc_stamp[p] = stamp;
    }
    claim_site(a, m.site_off + site);
  }
}

// ---------------------------------------------------------------------------
// One MD step (Sec. 3, Eq. 4-8), L lanes per particle, each with
// ceil(sites / L) sites of its stencil (cube: L = 8 in variant 1, where
// every lane has one corner, and L = 4 with two corners each in variants 2
// and 3; three-point stencil: L = 32, one site each).
//
// Each lane fetches its sites' cached moments (a particle that left its
// cube since the refill gathers the new sites itself) and, in variants 2 and
// 3, the sites' pending transfer; the interpolated fluid velocity (Eq. 5)
// is the sum over the lanes (butterfly shuffles, the same order on every
// lane).  Friction + noise (Eq. 4, 6) and velocity Verlet are evaluated on
// all lanes alike; lane 0 stores the particle.  Variant 1 then transfers
// the momentum right away (Eq. 7-8): the (site, component) adds of a
// particle are spread over its lanes in rounds, so the lanes of one atomic
// instruction share a few sites rather than touching 64 unrelated cache
// lines (eight lanes measured faster here than four).  Variants 2 and 3
// store (cube, dP) for the spreading kernel instead, because every particle
// must first read the velocities as of the end of the previous MD step
// (variant 3 sees the same velocities as variant 2 inside an interval; its
// transfer differs only in how the LB step applies it); there four lanes
// with two corners each halve the redundant per-particle arithmetic.
//
// With Rec, the particle's position and velocity before the step and the
// corner velocities (j [+ J]) and inverse densities it interpolated are
// recorded for the reverse sweep (position NaN: particle skipped).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pick3(const double v[3], int c) {
  return c == 0 ? v[0] : (c == 1 ? v[1] : v[2]);
}

// Lanes of the coupling kernel per particle: L lanes with ceil(sites / L)
// stencil sites each (8 for the cube in variant 1, whose in-kernel transfer
// spreads its atomics over the lanes; fewer in variants 2 and 3; 32 for the
// three-point stencil).
template <int L>
struct CoupleShape {
  static constexpr int kLanes = L;
  __device__ static __forceinline__ double sum(double v) {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) v += __shfl_xor(v, o, L);
    return v;
  }
};

// Transfer -w_k dP of one particle (Eq. 7-8) from its lanes: pair index
// kLanes r + lane = 3 site + component, over as many rounds as needed.
template <typename T, int ST, int L>
__device__ __forceinline__ void transfer_from_lanes(Vec4<T>* __restrict__ J, const RepMD& m,
                                                    const Cube& q, int lane, const double dp[3]) {
  constexpr int kL = L, kPairs = 3 * Stencil<ST>::kSites;
#pragma unroll
  for (int rnd = 0; rnd < (kPairs + kL - 1) / kL; ++rnd) {
    const int pair = rnd * kL + lane;
    if (pair >= kPairs) break;
    const int kc = pair / 3, c = pair - 3 * kc;
    int cx, cy, cz, site;
    double w;
    Stencil<ST>::site(q, m.g, kc, cx, cy, cz, site, w);
    atomicAdd(((T*)(J + m.site_off + site)) + c, (T)(-w * pick3(dp, c)));
  }
}

template <typename T, bool Rec, int ST, int L>
__global__ __launch_bounds__(kBlock) void k_couple(CoupleArgs<T> a) {
  using St = Stencil<ST>;
  using Sh = CoupleShape<L>;
  constexpr int kPer = (St::kSites + L - 1) / L;
  static_assert(!Rec || ST == 0, "recording (adjoint) exists for the trilinear stencil only");
  const T* __restrict__ pop = a.pop[a.clock->cur];
  const int stamp = cache_stamp(a.clock);
  const unsigned long long t_md = (unsigned long long)(a.clock->t_md + a.substep);
  const uint32_t step_lo = (uint32_t)(t_md & 0xFFFFFFFFull), step_hi = (uint32_t)(t_md >> 32);
  const int64_t N = a.N;
  const int64_t lanes = N * Sh::kLanes;
  // lanes come in whole particles (kLanes | kBlock): the lanes of a particle
  // are always active together, as the shuffles require
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < lanes;
       t += (int64_t)gridDim.x * kBlock) {
    const int64_t p = t / Sh::kLanes;
    const int k0 = (int)(t & (Sh::kLanes - 1));
    const int rr = a.single ? 0 : a.part_rep[p];
    double X[3], V[3];
    bool live = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      X[d] = a.x[d * N + p];
      V[d] = a.v[d * N + p];
      live = live && isfinite(X[d]) && isfinite(V[d]);
    }
    if (!live) {
      if (k0 == 0) {
        a.flags[0] = 1;
        if (a.variant >= 2) a.rec_cell[p] = -1;
        if (Rec) a.rec[p] = __builtin_nan("");
      }
      continue;
    }
    const RepMD& m = a.md[rr];
    Cube q;
    St::locate(X, m.g, q);
    const int cell = q.base[0] + m.g.nx * (q.base[1] + m.g.ny * q.base[2]);
    const bool hit = a.cc_stamp[p] == stamp && a.cc_cell[p] == cell;
    double ux = 0.0, uy = 0.0, uz = 0.0;
#pragma unroll
    for (int jj = 0; jj < kPer; ++jj) {
      const int k = k0 + jj * Sh::kLanes;
      if (k >= St::kSites) break;
      int cx, cy, cz, site;
      double w;
      St::site(q, m.g, k, cx, cy, cz, site, w);
      Vec4<T> cv;
      if (hit) {
        cv = *cache_entry<ST>(a, p, k);
      } else {
        // left the cube of the refill: this lane gathers its site
        int sidx[19];
        pull_sources(m.g, cx, cy, cz, sidx);
        T d[19];
#pragma unroll
        for (int i = 0; i < 19; ++i) d[i] = pop[(size_t)i * a.P + m.site_off + sidx[i]];
        T drho, jx, jy, jz;
        moments_deviation<T>(d, drho, jx, jy, jz);
        cv = Vec4<T>{jx, jy, jz, T(1) / ((T)m.rho0 + drho)};
        *cache_entry<ST>(a, p, k) = cv;
        claim_site(a, m.site_off + site);
        if (k == 0) {
          a.cc_cell[p] = cell;
          a.cc_stamp[p] = stamp;
        }
      }
      // fluid velocity at the particle (Eq. 5)
      double jx = (double)cv.x, jy = (double)cv.y, jz = (double)cv.z;
      if (a.variant >= 2) {
        const Vec4<T> jv = a.J[m.site_off + site];
        jx += (double)jv.x;
        jy += (double)jv.y;
        jz += (double)jv.z;
      }
      if (Rec) {
        a.rec[(6 + 3 * k) * N + p] = jx;
        a.rec[(7 + 3 * k) * N + p] = jy;
        a.rec[(8 + 3 * k) * N + p] = jz;
        a.rec[(30 + k) * N + p] = (double)cv.w;
      }
      const double wi = w * (double)cv.w;
      ux += wi * jx;
      uy += wi * jy;
      uz += wi * jz;
    }
    if (Rec && k0 == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        a.rec[d * N + p] = X[d];
        a.rec[(3 + d) * N + p] = V[d];
      }
    }
    const double u[3] = {Sh::sum(ux), Sh::sum(uy), Sh::sum(uz)};
    // friction + noise (Eq. 4), momentum change over the MD step (Eq. 6)
    double xi[3] = {0.0, 0.0, 0.0};
    if (m.noise) {
      const uint32_t lp = (uint32_t)a.pid[p];
      const Words4 o = philox10(Words4{lp, step_lo, m.tag, step_hi}, m.key0, m.key1);
      const uint32_t ws[3] = {o.w0, o.w1, o.w2};
#pragma unroll
      for (int d = 0; d < 3; ++d)
        xi[d] = 3.4641016151377546 * (((double)(ws[d] >> 8) + 0.5) * 5.9604644775390625e-08 - 0.5);
    }
    // velocity Verlet with the coupling force held over the step; with
    // position-dependent conservative forces the second half-kick waits
    // for the forces at the new positions (k_kick)
    double dp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double Fc = -m.gamma * (V[d] - u[d]) + m.amp * xi[d];
      dp[d] = m.tau * Fc;
      if (k0 == 0) {
        const double fc = a.fcons[d * N + p];
        int32_t im = a.img[d * N + p];
        double v1 = V[d] + m.h * (fc + Fc);
        double x1 = X[d] + m.tau * v1;
        wrap_coord(x1, im, m.L[d]);
        if (m.split_kick)
          a.fc_held[d * N + p] = Fc;
        else
          v1 += m.h * (fc + Fc);
        a.x[d * N + p] = x1;
        a.v[d * N + p] = v1;
        a.img[d * N + p] = im;
        if (a.variant >= 2) {
          a.rec_cell[d * N + p] = q.base[d];
          a.rec_frac[d * N + p] = q.s[d];
          a.rec_dp[d * N + p] = dp[d];
        }
      }
    }
    if (a.variant == 1) transfer_from_lanes<T, ST, L>(a.J, m, q, k0, dp);
  }
}

// Variant-2 momentum transfer of the MD step just taken, one lane per
// stencil site (see spread_corner).  With position-dependent forces the same
// transfer runs inside the force kernel instead.
template <typename T, int ST>
__global__ __launch_bounds__(kBlock) void k_spread(CoupleArgs<T> a) {
  using St = Stencil<ST>;
  const int64_t N = a.N;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < N * St::kLanes;
       t += (int64_t)gridDim.x * kBlock) {
    const int64_t p = t / St::kLanes;
    const int k = (int)(t & (St::kLanes - 1));
    if (k >= St::kSites) continue;
    Cube q;
    q.base[0] = a.rec_cell[p];
    if (q.base[0] < 0) continue;
    const RepMD& m = a.md[a.single ? 0 : a.part_rep[p]];
    q.base[1] = a.rec_cell[N + p];
    q.base[2] = a.rec_cell[2 * N + p];
    double dp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      q.s[d] = a.rec_frac[d * N + p];
      dp[d] = a.rec_dp[d * N + p];
    }
    spread_corner<T, ST>(a.J, a.shared_site, m, q, k, dp);
  }
}

template <typename T>
static CoupleArgs<T> couple_args(Context* c, int substep) {
  CoupleArgs<T> a;
  const Layout& L = c->plan.lay;
  a.x = (double*)c->x;
  a.v = (double*)c->v;
  a.img = c->img;
  a.fcons = (const double*)at(c, L.fcons);
  a.pop[0] = (T*)c->popv[0];
  a.pop[1] = (T*)c->popv[1];
  a.J = (Vec4<T>*)at(c, L.transfer);
  a.mark = (unsigned long long*)at(c, L.mark);
  a.rec_cell = (int32_t*)at(c, L.rec_cell);
  a.rec_frac = (double*)at(c, L.rec_frac);
  a.rec_dp = (double*)at(c, L.rec_dp);
  a.fc_held = (double*)at(c, L.fc_held);
  a.cc = (T*)at(c, L.cc);
  a.cc_cell = (int32_t*)at(c, L.cc_cell);
  a.cc_stamp = (int32_t*)at(c, L.cc_stamp);
  a.shared_site = (unsigned long long*)at(c, L.shared_site);
  a.flags = (int32_t*)at(c, L.flags);
  a.md = (const RepMD*)at(c, L.rep_md);
  a.part_rep = (const int32_t*)at(c, L.part_rep);
  a.pid = (const int32_t*)at(c, L.pid);
  a.clock = (const Clock*)at(c, L.clock);
  a.rec = c->rec_part ? c->rec_part + (size_t)substep * kAdjRec * (size_t)c->plan.Ntot : nullptr;
  a.P = (size_t)c->plan.Stot;
  a.N = c->plan.Ntot;
  a.substep = substep;
  a.variant = c->p[0].variant;
  a.single = c->plan.R == 1 ? 1 : 0;
  return a;
}

static int grid_for(int64_t work_blocks, int tuned) {
  const int64_t g = tuned > 0 ? std::min<int64_t>(tuned, work_blocks) : work_blocks;
  return (int)std::max<int64_t>(g, 1);
}

template <typename T, int ST>
static hipError_t launch_refill_st(Context* c, const CoupleArgs<T>& a) {
  const dim3 grid(grid_for((a.N * 32 + kBlock - 1) / kBlock, c->tune.part_blocks));
  if (ST == 0)
    hipLaunchKernelGGL(k_refill<T>, grid, dim3(kBlock), 0, c->stream, a);
  else
    hipLaunchKernelGGL(k_refill3<T>, grid, dim3(kBlock), 0, c->stream, a);
  return hipGetLastError();
}

template <typename T, int ST>
static hipError_t couple_st(Context* c, int substep) {
  using St = Stencil<ST>;
  CoupleArgs<T> a = couple_args<T>(c, substep);
  hipError_t e;
  const int64_t N = a.N;
  if (substep == 0 && (e = launch_refill_st<T, ST>(c, a)) != hipSuccess) return e;
  // lanes per particle of the coupling kernel
  constexpr int kL1 = ST == 0 ? 8 : 32, kL2 = ST == 0 ? 4 : 32;
  const int L = (a.variant == 1 || a.rec) ? kL1 : kL2;
  const dim3 cgrid(grid_for((N * L + kBlock - 1) / kBlock, c->tune.part_blocks));
  if (ST == 0 && a.rec)
    hipLaunchKernelGGL((k_couple<T, true, 0, 8>), cgrid, dim3(kBlock), 0, c->stream, a);
  else if (L == kL1)
    hipLaunchKernelGGL((k_couple<T, false, ST, kL1>), cgrid, dim3(kBlock), 0, c->stream, a);
  else
    hipLaunchKernelGGL((k_couple<T, false, ST, kL2>), cgrid, dim3(kBlock), 0, c->stream, a);
  // variants 2 and 3: the transfer waits until every particle has read J;
  // with position-dependent forces it runs inside the force kernel
  if ((e = hipGetLastError()) != hipSuccess || a.variant == 1 || c->plan.any_forces2) return e;
  const dim3 sgrid(grid_for((N * St::kLanes + kBlock - 1) / kBlock, c->tune.part_blocks));
  hipLaunchKernelGGL((k_spread<T, ST>), sgrid, dim3(kBlock), 0, c->stream, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t couple_t(Context* c, int substep) {
  return c->p[0].stencil == 1 ? couple_st<T, 1>(c, substep) : couple_st<T, 0>(c, substep);
}

hipError_t launch_couple(Context* c, int substep) {
  if (c->plan.Ntot == 0) return hipSuccess;
  return c->plan.prec == 32 ? couple_t<float>(c, substep) : couple_t<double>(c, substep);
}

template <typename T>
static hipError_t refill_t(Context* c) {
  CoupleArgs<T> a = couple_args<T>(c, 0);
  return c->p[0].stencil == 1 ? launch_refill_st<T, 1>(c, a) : launch_refill_st<T, 0>(c, a);
}

// The corner-cache refill alone (reads particle positions, writes only the
// cache and the marks of this LB interval): used to time launch shapes.
hipError_t launch_couple_refill_only(Context* c) {
  if (c->plan.Ntot == 0) return hipSuccess;
  return c->plan.prec == 32 ? refill_t<float>(c) : refill_t<double>(c);
}

// Forget cached corner moments (after the populations or counters were
// replaced from outside).
hipError_t invalidate_corner_cache(Context* c) {
  if (c->plan.Ntot == 0) return hipSuccess;
  return hipMemsetAsync(at(c, c->plan.lay.cc_stamp), 0, sizeof(int32_t) * c->plan.Ntot,
                        c->stream);
}

}  // namespace lbmd_impl
