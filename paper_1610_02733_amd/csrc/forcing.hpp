// The forcing part of the collision operator on its own: the paper's variant
// C update of a site after an MD step (Sec. 3).  A site that receives the
// momentum dJ in an MD step, with current momentum j and density rho, takes
//   dm_{1,2,3} = dJ,   dm_k = (1 + gamma_k)/2 q_k(u, dJ)  (stress modes 4..9),
// u = (j + dJ/2) / rho, mass and kinetic modes unchanged; q_k are the mode
// images of u dJ + dJ u (the Guo source of the LB step).
//
// Nothing reads a site's populations inside an LB interval except through
// rho and j (the particles' interpolation and the next update's u), so the
// library keeps the increments per site -- the momentum in the transfer field
// J, the six stress-mode increments in a stress field -- and adds them to the
// pulled populations when the LB step (or a copy of the state) reads the
// site.  In exact arithmetic this is the same as changing the populations at
// every MD step.
#pragma once

#include "lbmd_device.hpp"

namespace lbmd_impl {
using namespace lbmd_dev;

// Stress-mode increments (mode units, k = 4..9) of one variant-C update:
// j0 and irho are the site's momentum and inverse density at the start of
// the LB interval, J the momentum it received earlier in the interval, dJ
// the transfer of this MD step.
template <typename T>
__device__ __forceinline__ void stress_increment(T j0x, T j0y, T j0z, T irho, T Jx, T Jy, T Jz,
                                                 T dx, T dy, T dz, T hb, T hs, T s[6]) {
  const T ux = (j0x + Jx + T(0.5) * dx) * irho;
  const T uy = (j0y + Jy + T(0.5) * dy) * irho;
  const T uz = (j0z + Jz + T(0.5) * dz) * irho;
  const T fx = ux * dx, fy = uy * dy, fz = uz * dz;
  s[0] = hb * T(2) * (fx + fy + fz);
  s[1] = hs * T(2) * (T(2) * fx - fy - fz);
  s[2] = hs * T(2) * (fy - fz);
  s[3] = hs * (ux * dy + uy * dx);
  s[4] = hs * (uy * dz + uz * dy);
  s[5] = hs * (ux * dz + uz * dx);
}

// Population-deviation increments dd_i = w_i sum_k e_k(c_i) dm_k / b_k for
// momentum increments J and stress increments s (density and kinetic
// increments zero).
template <typename T>
__device__ __forceinline__ void mode_increments_to_pops(T Jx, T Jy, T Jz, const T s[6], T dd[19]) {
  const T M1 = T(3) * Jx, M2 = T(3) * Jy, M3 = T(3) * Jz;
  const T M4 = T(1.5) * s[0], M5 = T(0.75) * s[1], M6 = T(2.25) * s[2];
  const T M7 = T(9) * s[3], M8 = T(9) * s[4], M9 = T(9) * s[5];
  const T w1 = T(1) / T(18), w2 = T(1) / T(36);
  dd[0] = -M4 * (T(1) / T(3));
  const T Ex = T(2) * M5, Ey = M6 - M5, Ez = -M5 - M6;
  dd[1] = (Ex + M1) * w1;
  dd[2] = (Ex - M1) * w1;
  dd[3] = (Ey + M2) * w1;
  dd[4] = (Ey - M2) * w1;
  dd[5] = (Ez + M3) * w1;
  dd[6] = (Ez - M3) * w1;
  const T Dxy = M4 + M5 + M6, Dxz = M4 + M5 - M6, Dyz = M4 - T(2) * M5;
  dd[7] = (Dxy + M7 + M1 + M2) * w2;
  dd[8] = (Dxy + M7 - M1 - M2) * w2;
  dd[9] = (Dxy - M7 + M1 - M2) * w2;
  dd[10] = (Dxy - M7 - M1 + M2) * w2;
  dd[11] = (Dxz + M9 + M1 + M3) * w2;
  dd[12] = (Dxz + M9 - M1 - M3) * w2;
  dd[13] = (Dxz - M9 + M1 - M3) * w2;
  dd[14] = (Dxz - M9 - M1 + M3) * w2;
  dd[15] = (Dyz + M8 + M2 + M3) * w2;
  dd[16] = (Dyz + M8 - M2 - M3) * w2;
  dd[17] = (Dyz - M8 + M2 - M3) * w2;
  dd[18] = (Dyz - M8 - M2 + M3) * w2;
}

// Stress accumulator of a site: (s4, s5, s6, s7) and (s8, s9, -, -).
template <typename T>
struct Stress8 {
  Vec4<T> a, b;
};

}  // namespace lbmd_impl
