// The paper's variant C (Sec. 3) in closed form.
//
// In variant C every MD step k puts its transfer dJ_k into the populations
// of each receiving site through the forcing part of the collision alone:
// momentum + dJ_k, stress modes + (1 + gamma)/2 times the mode image of
// u_k dJ_k + dJ_k u_k with u_k = (j_k + dJ_k/2)/rho, mass and kinetic modes
// unchanged.  With j_k = j0 + J_k (J_k: what the site received before step
// k; rho does not change) the stress sources of an interval telescope:
//   sum_k (u_k dJ_k + dJ_k u_k) = (j0 J + J j0 + J J) / rho,
// J = sum_k dJ_k, because (J_k + dJ_k/2) dJ_k + dJ_k (J_k + dJ_k/2)
// = J_{k+1} J_{k+1} - J_k J_k.  The state after the interval's MD steps is
// therefore a function of the interval-start populations and the total
// transfer J alone, and the velocity (j0 + J)/rho the particles read inside
// the interval is the one variant B reads.  The library accumulates J as in
// variant B and applies these increments where the state is read: in the
// collide-stream kernel and in population copies.
#pragma once

#include "lbmd_device.hpp"

namespace lbmd_impl {
using namespace lbmd_dev;

// Stress-mode increments s[0..5] (modes 4..9, mode units) of an interval
// that moved the momentum J into a site with interval-start momentum j0 and
// inverse density irho.
template <typename T>
__device__ __forceinline__ void varc_stress(T j0x, T j0y, T j0z, T irho, T Jx, T Jy, T Jz, T hb,
                                            T hs, T s[6]) {
  const T qxx = (T(2) * j0x + Jx) * Jx * irho;
  const T qyy = (T(2) * j0y + Jy) * Jy * irho;
  const T qzz = (T(2) * j0z + Jz) * Jz * irho;
  const T qxy = (j0x * Jy + Jx * j0y + Jx * Jy) * irho;
  const T qyz = (j0y * Jz + Jy * j0z + Jy * Jz) * irho;
  const T qxz = (j0x * Jz + Jx * j0z + Jx * Jz) * irho;
  s[0] = hb * (qxx + qyy + qzz);
  s[1] = hs * (T(2) * qxx - qyy - qzz);
  s[2] = hs * (qyy - qzz);
  s[3] = hs * qxy;
  s[4] = hs * qyz;
  s[5] = hs * qxz;
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

}  // namespace lbmd_impl
