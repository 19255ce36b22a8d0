// Device helpers shared by the particle kernels and their adjoints: periodic
// wrap with image counting, the cube of lattice sites around a particle and
// the trilinear weights of its corners (Eq. 5).
#pragma once

#include "lbmd_internal.hpp"

namespace lbmd_impl {
using namespace lbmd_dev;

// Periodic wrap into [0, L) with image counting for any displacement
// (x -= k L, k = floor(x / L)); a value that rounds to exactly L after the
// shift moves to 0 in the next image.
__device__ __forceinline__ void wrap_coord(double& x, int32_t& im, double L) {
  if (x >= 0.0 && x < L) return;
  double k = floor(x / L);
  if (fabs(k) > 1e9) k = copysign(1e9, k);  // keep the image count in range
  x -= k * L;
  im += (int32_t)k;
  if (x >= L) {
    x -= L;
    im += 1;
  } else if (x < 0.0) {
    x += L;
    im -= 1;
  }
}

// Integer cube corner from a coordinate, kept inside [0, n) whatever the
// input (the coupling always addresses valid sites).
__device__ __forceinline__ int cell_of(int c, int n) {
  c %= n;
  return c < 0 ? c + n : c;
}

// Force cell of a position on its replica's cell grid (clamped to the grid).
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

// D3Q19 velocities in the library's order (opposite pairs adjacent).
static __device__ const int8_t kVel[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

struct Cube {
  int base[3];
  double s[3];
};

__device__ __forceinline__ void cube_of(const double X[3], const Geom& g, Cube& q) {
  const int n3[3] = {g.nx, g.ny, g.nz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double fl = floor(X[d]);
    q.s[d] = X[d] - fl;
    q.base[d] = cell_of((int)fl, n3[d]);
  }
}

// Site (replica-local) and trilinear weight (Eq. 5) of corner k of the cube.
__device__ __forceinline__ void corner_of(const Cube& q, const Geom& g, int k, int& cx, int& cy,
                                          int& cz, int& site, double& w) {
  cx = q.base[0] + (k & 1);
  cy = q.base[1] + ((k >> 1) & 1);
  cz = q.base[2] + ((k >> 2) & 1);
  cx = cx == g.nx ? 0 : cx;
  cy = cy == g.ny ? 0 : cy;
  cz = cz == g.nz ? 0 : cz;
  site = cx + g.nx * (cy + g.ny * cz);
  w = ((k & 1) ? q.s[0] : 1.0 - q.s[0]) * ((k & 2) ? q.s[1] : 1.0 - q.s[1]) *
      ((k & 4) ? q.s[2] : 1.0 - q.s[2]);
}

// Particle noise amplitude for the stencil weights' squared sum S: the
// random force balances the dissipation of the explicit MD step (Eq. 4, 6).
// The step damps the relative velocity w of the particle and the fluid at its
// stencil (the fluid takes -dP there at once: an effective mass rho0 / S) as
// w <- (1 - a) w + (1/m + S/rho0) dP_rand, a = gamma tau (1/m + S/rho0),
// whose equilibrium variance is kT (1/m + S/rho0) when <dP_rand^2> =
// 2 gamma kT tau (1 - a/2): F_rand = sqrt(2 gamma kT / tau) sqrt(1 - a/2) xi.
// Zero for a >= 2 (beyond the explicit step's stability bound).
__device__ __forceinline__ double noise_balance(const RepMD& m, double S) {
  return 1.0 - 0.5 * (m.gamma * m.tau * (m.inv_m + S / m.rho0));
}
__device__ __forceinline__ double noise_amplitude(const RepMD& m, double S) {
  const double bal = noise_balance(m, S);
  return bal > 0.0 ? m.amp * sqrt(bal) : 0.0;
}

// Kernels that give a particle one lane per corner of its cube (8 | kBlock,
// so the lanes of a particle are always active together).
constexpr int kCornerLanes = 8;

__device__ __forceinline__ double oct_sum(double v) {  // over the 8 lanes of a particle
  v += __shfl_xor(v, 1, kCornerLanes);
  v += __shfl_xor(v, 2, kCornerLanes);
  v += __shfl_xor(v, 4, kCornerLanes);
  return v;
}

// ---------------------------------------------------------------------------
// Interpolation / spreading stencils (Eq. 5 and Eq. 7 use the same one).
// A particle's stencil is described by a Cube: the lowest site index per
// axis (wrapped) and the offset s of the particle from a reference site.
//   ST = 0, trilinear: the 8 corners of the cube with lower corner floor(X),
//     s = X - floor(X).
//   ST = 1, three-point kernel per axis (Roma, Peskin and Berger 1999; the
//     higher-order scheme the paper mentions, Sec. 4): the 3 sites nearest
//     along each axis, c - 1, c, c + 1 with c = floor(X + 1/2), s = X - c;
//     the axis weight of a site at distance r from the particle is
//       (1 + sqrt(1 - 3 r^2)) / 3                for |r| <= 1/2,
//       (5 - 3|r| - sqrt(1 - 3 (1 - |r|)^2)) / 6 for 1/2 <= |r| <= 3/2;
//     27 sites.
// kLanes is the lane count per particle of the kernels that gather a
// stencil's sites one lane each (refill, re-gather after a cube change):
// 8, or 32 with lanes 27-31 idle.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double kernel3(double r) {
  const double a = fabs(r);
  if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) * (1.0 / 3.0);
  const double b = 1.0 - a;  // |r| < 3/2 always holds for the three nearest sites
  return (5.0 - 3.0 * a - sqrt(1.0 - 3.0 * b * b)) * (1.0 / 6.0);
}

template <int ST>
struct Stencil;

template <>
struct Stencil<0> {
  static constexpr int kSites = 8, kLanes = 8;
  __device__ static __forceinline__ void locate(const double X[3], const Geom& g, Cube& q) {
    cube_of(X, g, q);
  }
  __device__ static __forceinline__ void site(const Cube& q, const Geom& g, int k, int& cx,
                                              int& cy, int& cz, int& s, double& w) {
    corner_of(q, g, k, cx, cy, cz, s, w);
  }
};

template <>
struct Stencil<1> {
  static constexpr int kSites = 27, kLanes = 32;
  __device__ static __forceinline__ void locate(const double X[3], const Geom& g, Cube& q) {
    const int n3[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double c = floor(X[d] + 0.5);
      q.s[d] = X[d] - c;
      q.base[d] = cell_of((int)c - 1, n3[d]);
    }
  }
  __device__ static __forceinline__ void site(const Cube& q, const Geom& g, int k, int& cx,
                                              int& cy, int& cz, int& s, double& w) {
    const int ox = k % 3, oy = (k / 3) % 3, oz = k / 9;
    cx = q.base[0] + ox;
    cy = q.base[1] + oy;
    cz = q.base[2] + oz;
    cx = cx >= g.nx ? cx - g.nx : cx;
    cy = cy >= g.ny ? cy - g.ny : cy;
    cz = cz >= g.nz ? cz - g.nz : cz;
    s = cx + g.nx * (cy + g.ny * cz);
    w = kernel3(q.s[0] - (double)(ox - 1)) * kernel3(q.s[1] - (double)(oy - 1)) *
        kernel3(q.s[2] - (double)(oz - 1));
  }
};

}  // namespace lbmd_impl
