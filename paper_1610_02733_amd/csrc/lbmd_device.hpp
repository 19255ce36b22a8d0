// Device-side building blocks of the fluctuating D3Q19 LB / MD coupling:
// counter-based noise, the moment-space collision on population deviations
// and the lattice index helpers.  Host-callable too (no device intrinsics in
// the arithmetic), so the same code can be checked on the CPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmd_dev {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64-bit products; the two key words advance by the Weyl increments
// between rounds.
// ---------------------------------------------------------------------------
struct Words4 {
  uint32_t w0, w1, w2, w3;
};

__host__ __device__ __forceinline__ Words4 philox10(Words4 c, uint32_t ka, uint32_t kb) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t prodA = (uint64_t)0xD2511F53u * (uint64_t)c.w0;
    const uint64_t prodB = (uint64_t)0xCD9E8D57u * (uint64_t)c.w2;
    Words4 n;
    n.w0 = (uint32_t)(prodB >> 32) ^ c.w1 ^ ka;
    n.w1 = (uint32_t)prodB;
    n.w2 = (uint32_t)(prodA >> 32) ^ c.w3 ^ kb;
    n.w3 = (uint32_t)prodA;
    c = n;
    ka += 0x9E3779B9u;
    kb += 0xBB67AE85u;
  }
  return c;
}

// Noise-stream counter: (index, step low word, purpose<<28 | replica<<8 |
// call, step high word); key = the two words of the 64-bit seed.
enum : uint32_t { kPurposeFluid = 1u, kPurposeParticle = 2u };

__host__ __device__ __forceinline__ uint32_t noise_tag(uint32_t purpose, uint32_t replica,
                                                       uint32_t call) {
  return (purpose << 28) | ((replica & 0xFFFFFu) << 8) | (call & 0xFFu);
}

// ---------------------------------------------------------------------------
// Real-type helpers
// ---------------------------------------------------------------------------
template <typename T>
struct Vec4 {
  T x, y, z, w;
};

template <typename T>
__host__ __device__ __forceinline__ T tsqrt(T a);
template <>
__host__ __device__ __forceinline__ float tsqrt<float>(float a) { return sqrtf(a); }
template <>
__host__ __device__ __forceinline__ double tsqrt<double>(double a) { return sqrt(a); }

// ---------------------------------------------------------------------------
// Collision constants (per context, passed by value to the kernels).
// Relaxation factors g_s (shear), g_b (bulk), g_g (kinetic modes); h = (1+g)/2
// multiplies the Guo stress source; ns[k-4] = sqrt(b_k (1 - g_k^2)) *
// sqrt(12) / 2^16 turns a centred 16-bit integer into phi_k r_k / sqrt(mu rho).
// ---------------------------------------------------------------------------
template <typename T>
struct CollideConsts {
  T rho0;
  T gs, gb, gg;
  T hs, hb;
  T mu;  // 3 kT
  T ns[15];
  T g[3];  // uniform body-force density
  int noise;
};

// Collision of one site, in place on the 19 population deviations
// d_i = f_i - w_i rho0 (post-stream, pre-collision in; post-collision out).
// F: force density acting over the LB step (pending transfer + body force).
// hw: the eight Philox words of this site and step (used when k.noise).
//
// Mode basis: weighted-orthogonal D3Q19 polynomials 1, c, (c^2-1),
// (3cx^2-c^2), (cy^2-cz^2), cxcy, cycz, cxcz, (3c^2-5)c, (cy^2-cz^2)cx,
// (cz^2-cx^2)cy, (cx^2-cy^2)cz, 3c^4-6c^2+1, (2c^2-3)(3cx^2-c^2),
// (2c^2-3)(cy^2-cz^2), evaluated here through sums (s) and differences (a) of
// opposite populations.  Equilibrium stress moments are the images of
// rho c_s^2 I + rho u u with u = (j + F/2)/rho; the kinetic modes have zero
// equilibrium; the Guo source adds (1+g)/2 times the image of u F + F u.
//
// VarC: the site also holds the momentum J that the MD steps of the interval
// moved into it in the paper's variant C.  Its state is then the pulled one
// plus momentum J and the stress increments (1+g)/2 times the image of
// (j J + J j + J J)/rho (j: the pulled momentum), which are added in mode
// space before the relaxation (F then carries the body force alone).
template <typename T, bool VarC = false>
__host__ __device__ __forceinline__ void collide_deviation(T d[19], T Fx, T Fy, T Fz,
                                                           const uint32_t hw[8],
                                                           const CollideConsts<T>& k,
                                                           T Jx = T(0), T Jy = T(0),
                                                           T Jz = T(0)) {
  const T s12 = d[1] + d[2], a12 = d[1] - d[2];
  const T s34 = d[3] + d[4], a34 = d[3] - d[4];
  const T s56 = d[5] + d[6], a56 = d[5] - d[6];
  const T s78 = d[7] + d[8], a78 = d[7] - d[8];
  const T s9a = d[9] + d[10], a9a = d[9] - d[10];
  const T sbc = d[11] + d[12], abc = d[11] - d[12];
  const T sde = d[13] + d[14], ade = d[13] - d[14];
  const T sfg = d[15] + d[16], afg = d[15] - d[16];
  const T shi = d[17] + d[18], ahi = d[17] - d[18];
  const T sxy = s78 + s9a, sxz = sbc + sde, syz = sfg + shi;
  const T sdiag = sxy + sxz + syz;
  const T saxis = s12 + s34 + s56;

  const T drho = d[0] + saxis + sdiag;
  T jx = a12 + a78 + a9a + abc + ade;
  T jy = a34 + a78 - a9a + afg + ahi;
  T jz = a56 + abc - ade + afg - ahi;
  const T rho = k.rho0 + drho;
  const T irho = T(1) / rho;
  T i4 = T(0), i5 = T(0), i6 = T(0), i7 = T(0), i8 = T(0), i9 = T(0);
  if (VarC) {
    const T qxx = (T(2) * jx + Jx) * Jx * irho;
    const T qyy = (T(2) * jy + Jy) * Jy * irho;
    const T qzz = (T(2) * jz + Jz) * Jz * irho;
    i4 = k.hb * (qxx + qyy + qzz);
    i5 = k.hs * (T(2) * qxx - qyy - qzz);
    i6 = k.hs * (qyy - qzz);
    i7 = k.hs * (jx * Jy + Jx * jy + Jx * Jy) * irho;
    i8 = k.hs * (jy * Jz + Jy * jz + Jy * Jz) * irho;
    i9 = k.hs * (jx * Jz + Jx * jz + Jx * Jz) * irho;
    jx += Jx;
    jy += Jy;
    jz += Jz;
  }
  const T ux = (jx + T(0.5) * Fx) * irho;
  const T uy = (jy + T(0.5) * Fy) * irho;
  const T uz = (jz + T(0.5) * Fz) * irho;

  // stress modes
  T m4 = sdiag - d[0];
  T m5 = T(2) * s12 - s34 - s56 + sxy + sxz - T(2) * syz;
  T m6 = s34 - s56 + sxy - sxz;
  T m7 = s78 - s9a;
  T m8 = sfg - shi;
  T m9 = sbc - sde;
  if (VarC) {
    m4 += i4;
    m5 += i5;
    m6 += i6;
    m7 += i7;
    m8 += i8;
    m9 += i9;
  }
  // kinetic modes
  const T m10 = a78 + a9a + abc + ade - T(2) * a12;
  const T m11 = a78 - a9a + afg + ahi - T(2) * a34;
  const T m12 = abc - ade + afg - ahi - T(2) * a56;
  const T m13 = a78 + a9a - abc - ade;
  const T m14 = a9a - a78 + afg + ahi;
  const T m15 = abc - ade - afg + ahi;
  const T m16 = d[0] - T(2) * saxis + sdiag;
  const T m17 = s34 + s56 - T(2) * s12 + sxy + sxz - T(2) * syz;
  const T m18 = s56 - s34 + sxy - sxz;

  // equilibrium stress moments and Guo source
  const T xx = ux * ux, yy = uy * uy, zz = uz * uz;
  const T e4 = rho * (xx + yy + zz);
  const T e5 = rho * (T(2) * xx - yy - zz);
  const T e6 = rho * (yy - zz);
  const T e7 = rho * ux * uy;
  const T e8 = rho * uy * uz;
  const T e9 = rho * ux * uz;
  const T fx = ux * Fx, fy = uy * Fy, fz = uz * Fz;
  const T q4 = T(2) * (fx + fy + fz);
  const T q5 = T(2) * (T(2) * fx - fy - fz);
  const T q6 = T(2) * (fy - fz);
  const T q7 = ux * Fy + uy * Fx;
  const T q8 = uy * Fz + uz * Fy;
  const T q9 = ux * Fz + uz * Fx;

  T p[15];
  p[0] = e4 + k.gb * (m4 - e4) + k.hb * q4;
  p[1] = e5 + k.gs * (m5 - e5) + k.hs * q5;
  p[2] = e6 + k.gs * (m6 - e6) + k.hs * q6;
  p[3] = e7 + k.gs * (m7 - e7) + k.hs * q7;
  p[4] = e8 + k.gs * (m8 - e8) + k.hs * q8;
  p[5] = e9 + k.gs * (m9 - e9) + k.hs * q9;
  p[6] = k.gg * m10;
  p[7] = k.gg * m11;
  p[8] = k.gg * m12;
  p[9] = k.gg * m13;
  p[10] = k.gg * m14;
  p[11] = k.gg * m15;
  p[12] = k.gg * m16;
  p[13] = k.gg * m17;
  p[14] = k.gg * m18;
  if (k.noise) {
    const T amp = tsqrt<T>(k.mu * rho);
#pragma unroll
    for (int v = 0; v < 15; ++v) {
      const uint32_t w = hw[v >> 1];
      const uint32_t h = (v & 1) ? (w >> 16) : (w & 0xFFFFu);
      p[v] += amp * k.ns[v] * ((T)(int)h - T(32767.5));
    }
  }

  // back transform: d_i = w_i sum_k e_k(c_i) m*_k / b_k
  const T M0 = drho;
  const T M1 = T(3) * (jx + Fx), M2 = T(3) * (jy + Fy), M3 = T(3) * (jz + Fz);
  const T M4 = T(1.5) * p[0], M5 = T(0.75) * p[1], M6 = T(2.25) * p[2];
  const T M7 = T(9) * p[3], M8 = T(9) * p[4], M9 = T(9) * p[5];
  const T M10 = T(1.5) * p[6], M11 = T(1.5) * p[7], M12 = T(1.5) * p[8];
  const T M13 = T(4.5) * p[9], M14 = T(4.5) * p[10], M15 = T(4.5) * p[11];
  const T M16 = T(0.5) * p[12], M17 = T(0.75) * p[13], M18 = T(2.25) * p[14];

  const T w1 = T(1) / T(18), w2 = T(1) / T(36);
  d[0] = (M0 - M4 + M16) * (T(1) / T(3));
  const T Eax = M0 - T(2) * M16 + M17;  // shared by the three axis pairs
  const T Ex = M0 + T(2) * M5 - T(2) * M16 - T(2) * M17, Ox = M1 - T(2) * M10;
  const T Ey = Eax - M5 + M6 - M18, Oy = M2 - T(2) * M11;
  const T Ez = Eax - M5 - M6 + M18, Oz = M3 - T(2) * M12;
  d[1] = (Ex + Ox) * w1;
  d[2] = (Ex - Ox) * w1;
  d[3] = (Ey + Oy) * w1;
  d[4] = (Ey - Oy) * w1;
  d[5] = (Ez + Oz) * w1;
  d[6] = (Ez - Oz) * w1;
  const T D = M0 + M4 + M16;
  const T Dxy = D + M5 + M6 + M17 + M18;
  const T Dxz = D + M5 - M6 + M17 - M18;
  const T Dyz = D - T(2) * M5 - T(2) * M17;
  const T E78 = Dxy + M7, O78 = M1 + M2 + M10 + M11 + M13 - M14;
  const T E9a = Dxy - M7, O9a = M1 - M2 + M10 - M11 + M13 + M14;
  const T Ebc = Dxz + M9, Obc = M1 + M3 + M10 + M12 - M13 + M15;
  const T Ede = Dxz - M9, Ode = M1 - M3 + M10 - M12 - M13 - M15;
  const T Efg = Dyz + M8, Ofg = M2 + M3 + M11 + M12 + M14 - M15;
  const T Ehi = Dyz - M8, Ohi = M2 - M3 + M11 - M12 + M14 + M15;
  d[7] = (E78 + O78) * w2;
  d[8] = (E78 - O78) * w2;
  d[9] = (E9a + O9a) * w2;
  d[10] = (E9a - O9a) * w2;
  d[11] = (Ebc + Obc) * w2;
  d[12] = (Ebc - Obc) * w2;
  d[13] = (Ede + Ode) * w2;
  d[14] = (Ede - Ode) * w2;
  d[15] = (Efg + Ofg) * w2;
  d[16] = (Efg - Ofg) * w2;
  d[17] = (Ehi + Ohi) * w2;
  d[18] = (Ehi - Ohi) * w2;
}

// All 19 modes m_k = sum_i e_k(c_i) d_i of a population vector.
template <typename T>
__host__ __device__ __forceinline__ void modes19(const T d[19], T m[19]) {
  const T s12 = d[1] + d[2], a12 = d[1] - d[2];
  const T s34 = d[3] + d[4], a34 = d[3] - d[4];
  const T s56 = d[5] + d[6], a56 = d[5] - d[6];
  const T s78 = d[7] + d[8], a78 = d[7] - d[8];
  const T s9a = d[9] + d[10], a9a = d[9] - d[10];
  const T sbc = d[11] + d[12], abc = d[11] - d[12];
  const T sde = d[13] + d[14], ade = d[13] - d[14];
  const T sfg = d[15] + d[16], afg = d[15] - d[16];
  const T shi = d[17] + d[18], ahi = d[17] - d[18];
  const T sxy = s78 + s9a, sxz = sbc + sde, syz = sfg + shi;
  const T sdiag = sxy + sxz + syz, saxis = s12 + s34 + s56;
  m[0] = d[0] + saxis + sdiag;
  m[1] = a12 + a78 + a9a + abc + ade;
  m[2] = a34 + a78 - a9a + afg + ahi;
  m[3] = a56 + abc - ade + afg - ahi;
  m[4] = sdiag - d[0];
  m[5] = T(2) * s12 - s34 - s56 + sxy + sxz - T(2) * syz;
  m[6] = s34 - s56 + sxy - sxz;
  m[7] = s78 - s9a;
  m[8] = sfg - shi;
  m[9] = sbc - sde;
  m[10] = a78 + a9a + abc + ade - T(2) * a12;
  m[11] = a78 - a9a + afg + ahi - T(2) * a34;
  m[12] = abc - ade + afg - ahi - T(2) * a56;
  m[13] = a78 + a9a - abc - ade;
  m[14] = a9a - a78 + afg + ahi;
  m[15] = abc - ade - afg + ahi;
  m[16] = d[0] - T(2) * saxis + sdiag;
  m[17] = s34 + s56 - T(2) * s12 + sxy + sxz - T(2) * syz;
  m[18] = s56 - s34 + sxy - sxz;
}

// Transpose of the mode map: d_i = sum_k e_k(c_i) m_k.
template <typename T>
__host__ __device__ __forceinline__ void modes19_transpose(const T m[19], T d[19]) {
  d[0] = m[0] - m[4] + m[16];
  const T Eax = m[0] - T(2) * m[16] + m[17];
  const T Ex = m[0] + T(2) * m[5] - T(2) * m[16] - T(2) * m[17], Ox = m[1] - T(2) * m[10];
  const T Ey = Eax - m[5] + m[6] - m[18], Oy = m[2] - T(2) * m[11];
  const T Ez = Eax - m[5] - m[6] + m[18], Oz = m[3] - T(2) * m[12];
  d[1] = Ex + Ox;
  d[2] = Ex - Ox;
  d[3] = Ey + Oy;
  d[4] = Ey - Oy;
  d[5] = Ez + Oz;
  d[6] = Ez - Oz;
  const T D = m[0] + m[4] + m[16];
  const T Dxy = D + m[5] + m[6] + m[17] + m[18];
  const T Dxz = D + m[5] - m[6] + m[17] - m[18];
  const T Dyz = D - T(2) * m[5] - T(2) * m[17];
  const T E78 = Dxy + m[7], O78 = m[1] + m[2] + m[10] + m[11] + m[13] - m[14];
  const T E9a = Dxy - m[7], O9a = m[1] - m[2] + m[10] - m[11] + m[13] + m[14];
  const T Ebc = Dxz + m[9], Obc = m[1] + m[3] + m[10] + m[12] - m[13] + m[15];
  const T Ede = Dxz - m[9], Ode = m[1] - m[3] + m[10] - m[12] - m[13] - m[15];
  const T Efg = Dyz + m[8], Ofg = m[2] + m[3] + m[11] + m[12] + m[14] - m[15];
  const T Ehi = Dyz - m[8], Ohi = m[2] - m[3] + m[11] - m[12] + m[14] + m[15];
  d[7] = E78 + O78;
  d[8] = E78 - O78;
  d[9] = E9a + O9a;
  d[10] = E9a - O9a;
  d[11] = Ebc + Obc;
  d[12] = Ebc - Obc;
  d[13] = Ede + Ode;
  d[14] = Ede - Ode;
  d[15] = Efg + Ofg;
  d[16] = Efg - Ofg;
  d[17] = Ehi + Ohi;
  d[18] = Ehi - Ohi;
}

// Reverse mode of collide_deviation.  Inputs: the collision's inputs (d, F,
// noise words) and the adjoint of its outputs (dbar_out).  Outputs: the
// adjoint of the input deviations (dbar_in), of the force density (Fb), and
// the derivatives of the result with respect to the relaxation factors of
// the bulk, shear and kinetic modes (gbar[0..2]).  The noise enters through
// its amplitude sqrt(mu rho b_k (1 - g_k^2)); the variates themselves are
// fixed numbers of the counter-based stream.
template <typename T>
__host__ __device__ __forceinline__ void collide_deviation_adjoint(
    const T d[19], T Fx, T Fy, T Fz, const uint32_t hw[8], const CollideConsts<T>& k,
    const T dbar_out[19], T dbar_in[19], T& Fbx, T& Fby, T& Fbz, T gbar[3]) {
  // forward intermediates
  T m[19];
  modes19<T>(d, m);
  const T rho = k.rho0 + m[0];
  const T irho = T(1) / rho;
  const T ux = (m[1] + T(0.5) * Fx) * irho;
  const T uy = (m[2] + T(0.5) * Fy) * irho;
  const T uz = (m[3] + T(0.5) * Fz) * irho;
  const T xx = ux * ux, yy = uy * uy, zz = uz * uz;
  const T e[6] = {rho * (xx + yy + zz), rho * (T(2) * xx - yy - zz), rho * (yy - zz),
                  rho * ux * uy,        rho * uy * uz,                rho * ux * uz};
  const T fx = ux * Fx, fy = uy * Fy, fz = uz * Fz;
  const T q[6] = {T(2) * (fx + fy + fz), T(2) * (T(2) * fx - fy - fz), T(2) * (fy - fz),
                  ux * Fy + uy * Fx,     uy * Fz + uz * Fy,            ux * Fz + uz * Fx};
  // back transform: d_out = W E^T (m* / b)  ->  Mbar = E (W dbar_out)
  const T w0 = T(1) / T(3), w1 = T(1) / T(18), w2 = T(1) / T(36);
  T y[19];
  y[0] = w0 * dbar_out[0];
#pragma unroll
  for (int i = 1; i < 7; ++i) y[i] = w1 * dbar_out[i];
#pragma unroll
  for (int i = 7; i < 19; ++i) y[i] = w2 * dbar_out[i];
  T Mb[19];
  modes19<T>(y, Mb);
  // m*_k = b_k M_k: the adjoint of m*_k is Mbar_k / b_k
  const T ib[19] = {T(1),   T(3),   T(3),   T(3),   T(1.5), T(0.75), T(2.25),
                    T(9),   T(9),   T(9),   T(1.5), T(1.5), T(1.5),  T(4.5),
                    T(4.5), T(4.5), T(0.5), T(0.75), T(2.25)};
  T ps[19];
#pragma unroll
  for (int kk = 0; kk < 19; ++kk) ps[kk] = Mb[kk] * ib[kk];
  // m*_0 = rho - rho0 (deviation), m*_{1..3} = j + F
  T mb[19];
  T rhob = T(0);
  mb[0] = ps[0];
  mb[1] = ps[1];
  mb[2] = ps[2];
  mb[3] = ps[3];
  Fbx = ps[1];
  Fby = ps[2];
  Fbz = ps[3];
  gbar[0] = gbar[1] = gbar[2] = T(0);
  // noise on modes 4..18
  if (k.noise) {
    const T amp = tsqrt<T>(k.mu * rho);
    const T damp = amp > T(0) ? T(0.5) * k.mu / amp : T(0);
#pragma unroll
    for (int v = 0; v < 15; ++v) {
      const uint32_t w = hw[v >> 1];
      const uint32_t h = (v & 1) ? (w >> 16) : (w & 0xFFFFu);
      const T cv = (T)(int)h - T(32767.5);
      const T pb = ps[v + 4];
      rhob += pb * k.ns[v] * cv * damp;
      // ns = K sqrt(1 - g^2): d ns / d g = -ns g / (1 - g^2)
      const int cls = v == 0 ? 0 : (v <= 5 ? 1 : 2);
      const T g = cls == 0 ? k.gb : (cls == 1 ? k.gs : k.gg);
      gbar[cls] += pb * amp * cv * (-k.ns[v] * g / (T(1) - g * g));
    }
  }
  // relaxation of the stress modes (k = 4..9) and Guo source
  T eb[6], qb[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const T g = s == 0 ? k.gb : k.gs;
    const T h = s == 0 ? k.hb : k.hs;
    const T pb = ps[4 + s];
    eb[s] = (T(1) - g) * pb;
    mb[4 + s] = g * pb;
    qb[s] = h * pb;
    gbar[s == 0 ? 0 : 1] += pb * (m[4 + s] - e[s]) + T(0.5) * pb * q[s];
  }
  // kinetic modes relax to zero
#pragma unroll
  for (int kk = 10; kk < 19; ++kk) {
    mb[kk] = k.gg * ps[kk];
    gbar[2] += ps[kk] * m[kk];
  }
  // equilibrium e(rho, u)
  rhob += eb[0] * (xx + yy + zz) + eb[1] * (T(2) * xx - yy - zz) + eb[2] * (yy - zz) +
          eb[3] * ux * uy + eb[4] * uy * uz + eb[5] * ux * uz;
  T ubx = rho * (eb[0] * T(2) * ux + eb[1] * T(4) * ux + eb[3] * uy + eb[5] * uz);
  T uby = rho * (eb[0] * T(2) * uy - eb[1] * T(2) * uy + eb[2] * T(2) * uy + eb[3] * ux +
                 eb[4] * uz);
  T ubz = rho * (eb[0] * T(2) * uz - eb[1] * T(2) * uz - eb[2] * T(2) * uz + eb[4] * uy +
                 eb[5] * ux);
  // Guo source q(u, F)
  ubx += T(2) * qb[0] * Fx + T(4) * qb[1] * Fx + qb[3] * Fy + qb[5] * Fz;
  uby += T(2) * qb[0] * Fy - T(2) * qb[1] * Fy + T(2) * qb[2] * Fy + qb[3] * Fx + qb[4] * Fz;
  ubz += T(2) * qb[0] * Fz - T(2) * qb[1] * Fz - T(2) * qb[2] * Fz + qb[4] * Fy + qb[5] * Fx;
  Fbx += T(2) * qb[0] * ux + T(4) * qb[1] * ux + qb[3] * uy + qb[5] * uz;
  Fby += T(2) * qb[0] * uy - T(2) * qb[1] * uy + T(2) * qb[2] * uy + qb[3] * ux + qb[4] * uz;
  Fbz += T(2) * qb[0] * uz - T(2) * qb[1] * uz - T(2) * qb[2] * uz + qb[4] * uy + qb[5] * ux;
  // u = (j + F/2) / rho
  mb[1] += ubx * irho;
  mb[2] += uby * irho;
  mb[3] += ubz * irho;
  Fbx += T(0.5) * ubx * irho;
  Fby += T(0.5) * uby * irho;
  Fbz += T(0.5) * ubz * irho;
  rhob -= (ubx * ux + uby * uy + ubz * uz) * irho;
  // rho = rho0 + m_0
  mb[0] += rhob;
  modes19_transpose<T>(mb, dbar_in);
}

// Density deviation and momentum of 19 population deviations.
template <typename T>
__host__ __device__ __forceinline__ void moments_deviation(const T d[19], T& drho, T& jx, T& jy,
                                                           T& jz) {
  const T a12 = d[1] - d[2], a34 = d[3] - d[4], a56 = d[5] - d[6];
  const T a78 = d[7] - d[8], a9a = d[9] - d[10], abc = d[11] - d[12];
  const T ade = d[13] - d[14], afg = d[15] - d[16], ahi = d[17] - d[18];
  T s = d[0];
#pragma unroll
  for (int i = 1; i < 19; ++i) s += d[i];
  drho = s;
  jx = a12 + a78 + a9a + abc + ade;
  jy = a34 + a78 - a9a + afg + ahi;
  jz = a56 + abc - ade + afg - ahi;
}

// ---------------------------------------------------------------------------
// Lattice geometry and population storage.  Site index r = x + nx*(y + ny*z).
//
// Populations are stored per replica in z-planes: for each z the 19
// population planes of nx*ny values follow one another, x fastest, so
// population i of site (x, y, z) sits at offset ((z*19 + i)*ny + y)*nx + x
// from the replica's base (19 * its first global site).  A wavefront that
// streams a row of one population touches one contiguous run, and the 19
// planes of a z-slab lie within 19*nx*ny values: on MI355X this plane
// interleave streamed faster than 19 separate arrays (measured: 78% against
// 73-74% of the HBM peak for the bare collide-stream access pattern at
// 256^3).
//
// "Pull" storage: the entry of population i at site s holds the
// post-collision value produced at s, so the post-stream value at r is the
// entry of population i at r - c_i.
// ---------------------------------------------------------------------------
struct Geom {
  int nx, ny, nz;
  int S;          // nx*ny*nz
  int A;          // nx*ny, one population plane
  double inv_nx;  // 1/nx, 1/ny for the division helpers
  double inv_ny;
};

// n / d for 0 <= n < 2^31 via a double reciprocal and one correction step.
__host__ __device__ __forceinline__ int div_fast(int n, int d, double inv_d, int& rem) {
  int q = (int)((double)n * inv_d);
  int r = n - q * d;
  if (r < 0) {
    q -= 1;
    r += d;
  } else if (r >= d) {
    q += 1;
    r -= d;
  }
  rem = r;
  return q;
}

__host__ __device__ __forceinline__ void site_coords(const Geom& g, int r, int& x, int& y, int& z) {
  int row = div_fast(r, g.nx, g.inv_nx, x);
  z = div_fast(row, g.ny, g.inv_ny, y);
}

// Offset of population i of site (x, y, z) from the replica's base.
__host__ __device__ __forceinline__ size_t pop_offset(const Geom& g, int i, int x, int y, int z) {
  return ((size_t)z * 19 + (size_t)i) * (size_t)g.A + (size_t)(y * g.nx + x);
}

// Offsets of the pull sources of the 19 populations at site (x, y, z): the
// entry of population i at r - c_i (periodic).
__host__ __device__ __forceinline__ void pull_offsets(const Geom& g, int x, int y, int z,
                                                      size_t off[19]) {
  const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
  const size_t A = (size_t)g.A;
  // plane bases z*19*A (population 0) and row starts y*nx
  const size_t b0 = (size_t)z * 19 * A, bm = (size_t)zm * 19 * A, bp = (size_t)zp * 19 * A;
  const int r0 = y * g.nx, rm = ym * g.nx, rp = yp * g.nx;
  off[0] = b0 + (size_t)(r0 + x);
  off[1] = b0 + A + (size_t)(r0 + xm);          // +x came from x-1
  off[2] = b0 + 2 * A + (size_t)(r0 + xp);      // -x
  off[3] = b0 + 3 * A + (size_t)(rm + x);       // +y
  off[4] = b0 + 4 * A + (size_t)(rp + x);       // -y
  off[5] = bm + 5 * A + (size_t)(r0 + x);       // +z
  off[6] = bp + 6 * A + (size_t)(r0 + x);       // -z
  off[7] = b0 + 7 * A + (size_t)(rm + xm);      // (1,1,0)
  off[8] = b0 + 8 * A + (size_t)(rp + xp);      // (-1,-1,0)
  off[9] = b0 + 9 * A + (size_t)(rp + xm);      // (1,-1,0)
  off[10] = b0 + 10 * A + (size_t)(rm + xp);    // (-1,1,0)
  off[11] = bm + 11 * A + (size_t)(r0 + xm);    // (1,0,1)
  off[12] = bp + 12 * A + (size_t)(r0 + xp);    // (-1,0,-1)
  off[13] = bp + 13 * A + (size_t)(r0 + xm);    // (1,0,-1)
  off[14] = bm + 14 * A + (size_t)(r0 + xp);    // (-1,0,1)
  off[15] = bm + 15 * A + (size_t)(rm + x);     // (0,1,1)
  off[16] = bp + 16 * A + (size_t)(rp + x);     // (0,-1,-1)
  off[17] = bp + 17 * A + (size_t)(rm + x);     // (0,1,-1)
  off[18] = bm + 18 * A + (size_t)(rp + x);     // (0,-1,1)
}

}  // namespace lbmd_dev
