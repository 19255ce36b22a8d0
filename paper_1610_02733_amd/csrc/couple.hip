// Particle coupling kernels (Sec. 3, Eq. 4-8): fluid velocity at the
// particle by interpolation over the sites of its stencil (the 8 sites of
// its cube, or 27 with the three-point kernel), friction plus noise,
// velocity Verlet, and transfer of -dP to the same sites with the same
// weights.  Particles of all replicas in one launch; each particle reads its
// replica's constants.  Kernels are templated on the stencil (ST, see
// particle_geom.hpp); the adjoint exists for the trilinear one only.
#include <algorithm>

#include "couple_state.hpp"

namespace lbmd_impl {
using namespace lbmd_dev;

// ---------------------------------------------------------------------------
// Corner-cache refill, once per LB interval (before its first MD step):
// (j, 1/rho) of the post-stream state at the 8 corners of every particle's
// cube.  32 lanes per particle, 4 per corner, which split the corner's 19
// pulled populations; the state does not change until the next LB step, so
// the MD steps of the interval read 8 contiguous vectors per particle instead
// of 8 x 19 scattered populations.  Also marks the 8 sites as receivers of
// momentum transfer for the LB step and records the particle at its cube's
// base (owner_of_shared).
// ---------------------------------------------------------------------------
constexpr int kRefillLanes = 32;

// Workgroups go to the chip's 8 XCDs in turn (workgroup b to XCD b mod 8),
// and every XCD has an L2 of its own.  Particles stored next to each other
// in the spatial order pull many of the same population lines, and with
// blocks renumbered so that XCD x takes the x-th contiguous eighth of them,
// neighbours share one L2.  That cuts the L2 misses of the refill by a fifth
// but not its DRAM lines (without it the repeated lines are hits in the
// memory-side cache shared by all XCDs), and spreading the XCDs over eight
// regions of the lattice at once costs more than it saves for the cube
// (175 against 169 us per 1e5 particles); the three-point refill, with 27
// sites per particle, gains about 1% and uses it.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_contiguous_block() {
  const int64_t G = gridDim.x, b = blockIdx.x;
  const int64_t q = G / kXcds, r = G % kXcds, x = b % kXcds;
  return x * q + (x < r ? x : r) + b / kXcds;
}

template <typename T>
__device__ __forceinline__ T quad_sum(T v) {  // over the 4 lanes of a corner
  v += __shfl_xor(v, 1, kRefillLanes);
  v += __shfl_xor(v, 2, kRefillLanes);
  return v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_refill(CoupleArgs<T> a) {
  const T* __restrict__ pop = a.pop[a.clock->cur];
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
        const T d = pop[19 * (size_t)m.site_off + pop_offset(m.g, i, sx, sy, sz)];
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
    // claims (claim_site): corners k and k ^ 1 (4 lanes apart) lie in one
    // row, most often in one 64-bit mark word, and then one atomic sets both
    // bits; each corner reads its own bit's old value (a corner that
    // coincides with its partner, on an axis of one site, is claimed twice)
    const int gs = m.site_off + site;
    const int gs_pair = __shfl_xor(gs, 4, kRefillLanes);
    const bool same_word = (gs >> 6) == (gs_pair >> 6);
    const bool lead = (k & 1) == 0 || !same_word;
    unsigned long long old = 0;
    if (c == 0 && lead) {
      unsigned long long bits = 1ull << (gs & 63);
      if (same_word) bits |= 1ull << (gs_pair & 63);
      old = atomicOr(a.mark + (gs >> 6), bits);
    }
    const unsigned long long old_pair = __shfl_xor(old, 4, kRefillLanes);
    if (c == 0 && (((lead ? old : old_pair) >> (gs & 63)) & 1ull || gs == gs_pair))
      reinterpret_cast<T*>(a.J + gs)[3] = T(1);
    if (sl == 0 && a.own_on) a.owner[gs] = (int32_t)p;  // corner 0: the cube's base
  }
}

// The same refill for the three-point stencil: 32 lanes per particle, lane k
// < 27 gathers the 19 pulled populations of stencil site k itself.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_refill3(CoupleArgs<T> a) {
  const T* __restrict__ pop = a.pop[a.clock->cur];
  const int64_t lanes = a.N * 32;
  for (int64_t t = xcd_contiguous_block() * kBlock + threadIdx.x; t < lanes;
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
    size_t off[19];
    pull_offsets(m.g, cx, cy, cz, off);
    const T* __restrict__ base = pop + 19 * (size_t)m.site_off;
    T d[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = base[off[i]];
    T drho, jx, jy, jz;
    moments_deviation<T>(d, drho, jx, jy, jz);
    *cache_entry<1>(a, p, k) = Vec4<T>{jx, jy, jz, T(1) / ((T)m.rho0 + drho)};
    // claims (claim_site): the three sites of a row (lanes k - ox .. k - ox
    // + 2) most often share a 64-bit mark word, and then the row's first
    // lane sets their bits with one atomic; each site reads its own bit's
    // old value (sites that coincide, on an axis shorter than the stencil,
    // are claimed more than once)
    const int gs = m.site_off + site;
    const int ox = k % 3, lead = (int)(t & 31) - ox;
    const int g0 = __shfl(gs, lead, 32), g1 = __shfl(gs, lead + 1, 32),
              g2 = __shfl(gs, lead + 2, 32);
    const bool covered = ox > 0 && (gs >> 6) == (g0 >> 6);
    unsigned long long old = 0;
    if (!covered) {
      unsigned long long bits = 1ull << (gs & 63);
      if (ox == 0) {
        if ((g1 >> 6) == (gs >> 6)) bits |= 1ull << (g1 & 63);
        if ((g2 >> 6) == (gs >> 6)) bits |= 1ull << (g2 & 63);
      }
      old = atomicOr(a.mark + (gs >> 6), bits);
    }
    const unsigned long long old_lead = __shfl(old, lead, 32);
    const bool dup = (gs == g0) + (gs == g1) + (gs == g2) > 1;
    if ((((covered ? old_lead : old) >> (gs & 63)) & 1ull) || dup)
      reinterpret_cast<T*>(a.J + gs)[3] = T(1);
    if (k == 0 && a.own_on) a.owner[gs] = (int32_t)p;  // the stencil's base
  }
}

// ---------------------------------------------------------------------------
// One MD step (Sec. 3, Eq. 4-8), L lanes per particle, each with
// ceil(sites / L) sites of its stencil (cube: two lanes with four corners
// each, which cuts the redundant per-particle arithmetic, or eight while
// recording; three-point stencil: eight lanes with up to four sites each).
//
// Each lane fetches its sites' cached moments (the refill, or for a particle
// that changed cubes the after-step work of the previous step, filled them)
// and the sites' pending transfer: the particle's own entry at sites it
// claimed alone, J at shared ones (couple_state.hpp, own transfers); the
// interpolated fluid velocity (Eq. 5) is the sum over the lanes (butterfly
// shuffles, the same order on every lane) and includes the pending transfer
// in variants 2 and 3 (variant 3 sees the same velocities as variant 2
// inside an interval; its transfer differs only in how the LB step applies
// it).  Friction + noise (Eq. 4, 6) and velocity Verlet are evaluated on all
// lanes alike; lane 0 stores the particle.  The transfer -w_k dP (Eq. 7-8)
// is then added at once at sites only this particle claimed in the interval,
// which no other particle reads or writes (to its own entry, and to J when
// it leaves the site or the interval ends), and listed for the after-step
// work (after_step_item) at shared sites, because in variants 2 and 3 every
// particle must first read J as of the end of the previous MD step.
//
// With Rec, the particle's position and velocity before the step and the
// corner velocities (j [+ J]) and inverse densities it interpolated are
// recorded for the reverse sweep (position NaN: particle skipped).  With Bin
// (position-dependent forces follow), lane 0 also counts the particle into
// its force cell at the new position.
// ---------------------------------------------------------------------------
// Lanes of the coupling kernel per particle: L lanes with ceil(sites / L)
// stencil sites each.
template <int L>
struct CoupleShape {
  static constexpr int kLanes = L;
  __device__ static __forceinline__ double sum(double v) {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) v += __shfl_xor(v, o, L);
    return v;
  }
};

// Retag: the launch takes every site's sharing from J (the first MD step
// after a refill), so the own-transfer entries are written but not read.
template <typename T, bool Rec, int ST, int L, bool Bin, bool One, bool Retag = false>
__global__ __launch_bounds__(kBlock) void k_couple(CoupleArgs<T> a) {
  using St = Stencil<ST>;
  using Sh = CoupleShape<L>;
  constexpr int kPer = (St::kSites + L - 1) / L;
  static_assert(!Rec || ST == 0, "recording (adjoint) exists for the trilinear stencil only");
  const unsigned long long t_md = (unsigned long long)(a.clock->t_md + a.substep);
  const uint32_t step_lo = (uint32_t)(t_md & 0xFFFFFFFFull), step_hi = (uint32_t)(t_md >> 32);
  const int64_t N = a.N;
  const int64_t lanes = N * Sh::kLanes;
  // One (a single replica): the replica's constants are the same for every
  // particle, read once before any store (uniform, scalar loads); otherwise
  // each particle reads its replica's entry
  RepMD m1;
  if constexpr (One) m1 = a.md[0];
  // entries of this block's segment in the two lists, counted in LDS
  __shared__ int s_l, s_m;
  // Bin: the overflow length of the other half, for the binning after this one
  if (Bin && blockIdx.x == 0 && threadIdx.x == 0) a.bin_count[2 * a.ncells + (int)(t_md & 1)] = 0;
  // lanes come in whole particles (kLanes | kBlock): the lanes of a particle
  // are always active together, as the shuffles require; every thread of a
  // block runs the loop the same number of times (block barriers)
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t t0 = (int64_t)blockIdx.x * kBlock; t0 < lanes; t0 += stride) {
    const int64_t t = t0 + threadIdx.x;
    const int64_t seg = t0 / kBlock;
    if (threadIdx.x == 0) s_l = s_m = 0;
    __syncthreads();
    bool moved = false, leave = false;
    int new_cell = 0, old_cell = 0;
    int gs_[kPer];
    double w_[kPer];
    Vec4<T> jv_[kPer];
    bool sh_[kPer], dec_[kPer];
    double dp[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int jj = 0; jj < kPer; ++jj) {
      gs_[jj] = -1;
      sh_[jj] = dec_[jj] = false;
    }
    const int64_t p = t / Sh::kLanes;
    const int k0 = (int)(t & (Sh::kLanes - 1));
    double X[3], V[3];
    // everything the step reads of the particle and its stencil entries,
    // loaded together (J, which needs the stencil's sites, follows)
    double fc[3] = {0.0, 0.0, 0.0};
    uint32_t lp = 0;
    Vec4<T> cv_[kPer];
    int old_bin = -1;  // Bin: the particle's count entry of the previous binning
    int rep_p = 0;     // the particle's replica (several replicas)
    RepMD mr;
    bool live = t < lanes;
    if (live) {
      if (Bin && k0 == 0) old_bin = a.bin[p];
      if constexpr (!One) rep_p = a.part_rep[p];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        X[d] = a.x[d * N + p];
        V[d] = a.v[d * N + p];
      }
      // conservative forces: none in force model 0 (known here for a single
      // replica; otherwise the zeros are read)
      if (!One || m1.force_model != 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) fc[d] = a.fcons[d * N + p];
      }
      lp = (uint32_t)a.pid[p];
#pragma unroll
      for (int jj = 0; jj < kPer; ++jj) {
        const int k = k0 + jj * Sh::kLanes;
        if (k < St::kSites) {
          cv_[jj] = *cache_entry<ST>(a, p, k);
          // (Bin: position-dependent forces, so no own transfers are kept;
          // every MD step takes the sharing and the transfer from J; Retag:
          // this step does)
          if constexpr (Bin || Retag)
            jv_[jj] = Vec4<T>{T(0), T(0), T(0), T(0)};
          else
            jv_[jj] = *own_entry<ST>(a, p, k);
        }
      }
      // the replica's constants as soon as its index is in (several replicas)
      if constexpr (!One) mr = a.md[rep_p];
#pragma unroll
      for (int d = 0; d < 3; ++d) live = live && isfinite(X[d]) && isfinite(V[d]);
      if (!live && k0 == 0) {
        a.flags[0] = 1;
        if (Rec) a.rec[p] = __builtin_nan("");
        if (Bin) {
          if (old_bin >= 0) a.bin_count[old_bin] = 0;
          a.bin[p] = -1;
        }
      }
    }
    if (live) {
      const RepMD& m = One ? m1 : mr;
      Cube q;
      St::locate(X, m.g, q);
      // the sites' pending transfer: the particle's own one where it claimed
      // the site alone, else J (all loads issued before use); after a refill
      // the w word of J tells which (claim_site), and so it does for a site
      // claimed after a stencil change (own w = 2)
#pragma unroll
      for (int jj = 0; jj < kPer; ++jj) {
        const int k = k0 + jj * Sh::kLanes;
        if (k < St::kSites) {
          int cx, cy, cz, site;
          double w;
          St::site(q, m.g, k, cx, cy, cz, site, w);
          gs_[jj] = m.site_off + site;
          w_[jj] = w;
        }
      }
      // (one load per site, from J or again from the own entry, which no
      // other thread writes: no branch, so the loads issue back to back)
      const bool retag = a.retag != 0;
      const Vec4<T>* src_[kPer];
#pragma unroll
      for (int jj = 0; jj < kPer; ++jj) {
        const T ow = jv_[jj].w;
        dec_[jj] = retag | (ow == T(2));
        const bool use_j = (retag | (ow != T(0))) & (gs_[jj] >= 0);
        // (a slot past the stencil's last site reads the first own entry)
        src_[jj] = use_j ? a.J + gs_[jj]
                         : own_entry<ST>(a, p, gs_[jj] >= 0 ? k0 + jj * Sh::kLanes : 0);
      }
#pragma unroll
      for (int jj = 0; jj < kPer; ++jj) jv_[jj] = *src_[jj];
      double ux = 0.0, uy = 0.0, uz = 0.0;
#pragma unroll
      for (int jj = 0; jj < kPer; ++jj) {
        if (gs_[jj] < 0) continue;
        const int k = k0 + jj * Sh::kLanes;
        const Vec4<T> cv = cv_[jj];
        sh_[jj] = jv_[jj].w != T(0);
        // fluid velocity at the particle (Eq. 5)
        double jx = (double)cv.x, jy = (double)cv.y, jz = (double)cv.z;
        if (a.variant >= 2) {  // the fluid velocity includes the pending transfer
          jx += (double)jv_[jj].x;
          jy += (double)jv_[jj].y;
          jz += (double)jv_[jj].z;
        }
        if (Rec) {
          a.rec[(6 + 3 * k) * N + p] = jx;
          a.rec[(7 + 3 * k) * N + p] = jy;
          a.rec[(8 + 3 * k) * N + p] = jz;
          a.rec[(30 + k) * N + p] = (double)cv.w;
        }
        const double wi = w_[jj] * (double)cv.w;
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
      // noise amplitude from the stencil's squared weights (noise_amplitude)
      double s2 = 0.0;
#pragma unroll
      for (int jj = 0; jj < kPer; ++jj)
        if (gs_[jj] >= 0) s2 += w_[jj] * w_[jj];
      const double amp = m.noise ? noise_amplitude(m, Sh::sum(s2)) : 0.0;
      // friction + noise (Eq. 4), momentum change over the MD step (Eq. 6)
      double xi[3] = {0.0, 0.0, 0.0};
      if (m.noise) {
        const Words4 o = philox10(Words4{lp, step_lo, m.tag, step_hi}, m.key0, m.key1);
        const uint32_t ws[3] = {o.w0, o.w1, o.w2};
#pragma unroll
        for (int d = 0; d < 3; ++d)
          xi[d] = 3.4641016151377546 * (((double)(ws[d] >> 8) + 0.5) * 5.9604644775390625e-08 - 0.5);
      }
      // velocity Verlet with the coupling force held over the step; with
      // position-dependent conservative forces the second half-kick waits
      // for the forces at the new positions (k_forces)
      double Xn[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double Fc = -m.gamma * (V[d] - u[d]) + amp * xi[d];
        dp[d] = m.tau * Fc;
        double v1 = V[d] + m.h * (fc[d] + Fc);
        double x1 = X[d] + m.tau * v1;
        int32_t dim = 0;  // periodic images crossed in this step (rare)
        wrap_coord(x1, dim, m.L[d]);
        Xn[d] = x1;
        if (k0 == 0) {
          if (m.split_kick)
            a.fc_held[d * N + p] = Fc;
          else
            v1 += m.h * (fc[d] + Fc);
          a.x[d * N + p] = x1;
          a.v[d * N + p] = v1;
          if (dim != 0) a.img[d * N + p] += dim;
        }
      }
      if (Bin && k0 == 0) {
        // force cell at the new position (MD step t_md + 1), for the force
        // kernel that follows; the count entry of the previous binning (the
        // other half) is cleared for the binning after this one
        if (old_bin >= 0) a.bin_count[old_bin] = 0;
        const int half = (int)((t_md + 1) & 1);
        if (m.force_model >= 2 && isfinite(Xn[0]) && isfinite(Xn[1]) && isfinite(Xn[2])) {
          const int cb = m.cell_off + local_cell(Xn, m);
          a.bin[p] = (int32_t)(half * a.ncells + cb);
          cell_insert(a.bin_count + half * a.ncells, a.bin_slot, a.bin_ovf,
                      a.bin_count + 2 * a.ncells + half, a.cell_cap, cb, (int)p);
        } else {
          a.bin[p] = -1;
        }
      }
      // the next MD step needs other sites if the stencil moved (a
      // non-finite new position is caught by that step); every lane of the
      // particle sees the same new position
      const bool fin = isfinite(Xn[0]) && isfinite(Xn[1]) && isfinite(Xn[2]);
      if (fin) {
        Cube qn;
        St::locate(Xn, m.g, qn);
        moved = qn.base[0] != q.base[0] || qn.base[1] != q.base[1] || qn.base[2] != q.base[2];
        new_cell = qn.base[0] + m.g.nx * (qn.base[1] + m.g.ny * qn.base[2]);
      }
      // the particle's own transfers go to J when it leaves its sites (a
      // non-finite particle is skipped from the next step on) and at the
      // interval's last MD step
      leave = a.last || moved || !fin;
      if (moved && k0 == 0) a.moved_at[p] = (long long)t_md;
      old_cell = q.base[0] + m.g.nx * (q.base[1] + m.g.ny * q.base[2]);
      // the record of the stencil it leaves (owner_of_shared)
      if ((moved || !fin) && k0 == 0 && a.own_on) a.owner[m.site_off + old_cell] = -1;
    }
    // transfer -w_k dP (Eq. 7-8): a site only this particle claimed in the
    // interval has no other reader or writer, so it takes the new value right
    // away; transfers to shared sites wait in the step's list until every
    // particle has read J (after_step_item)
#pragma unroll
    for (int jj = 0; jj < kPer; ++jj) {
      const int gs = gs_[jj];
      const double ww = gs >= 0 ? w_[jj] : 0.0;
      const T ax = (T)(-ww * dp[0]), ay = (T)(-ww * dp[1]), az = (T)(-ww * dp[2]);
      if (gs >= 0 && !sh_[jj]) {
        const Vec4<T> nv{jv_[jj].x + ax, jv_[jj].y + ay, jv_[jj].z + az, T(0)};
        if (!Bin && !a.final_step) *own_entry<ST>(a, p, k0 + jj * Sh::kLanes) = nv;
        if (leave) a.J[gs] = nv;
      }
      if (gs >= 0 && sh_[jj]) {
        const int64_t e = seg * (kBlock * kPer) + atomicAdd(&s_l, 1);
        a.lsite[e] = gs;
        a.ldelta[e] = Vec4<T>{ax, ay, az, T(0)};
        if (!Bin && dec_[jj] && !a.final_step)
          *own_entry<ST>(a, p, k0 + jj * Sh::kLanes) = Vec4<T>{T(0), T(0), T(0), T(1)};
      }
    }
    // (after the interval's last MD step the next refill gathers and claims
    // every particle's stencil: moved particles need no after-step work)
    if (moved && k0 == 0 && !a.final_step)
      reinterpret_cast<int4*>(a.mlist)[seg * (kBlock / L) + atomicAdd(&s_m, 1)] =
          make_int4((int)p, new_cell, old_cell, rep_p);
    __syncthreads();
    if (threadIdx.x == 0) {
      a.lseg[seg] = s_l;
      a.mseg[seg] = s_m;
    }
  }
}

// After an MD step without a force kernel: the after-step work
// (after_step_item) as a launch of its own.
// With Reduce, the shared-site transfers of each segment are summed per site
// in LDS first (reduce_segment_transfers; dynamic shared memory of
// kSiteTable * (4 + 3 sizeof(T)) bytes).
template <typename T, int ST, bool Reduce, bool One>
__global__ __launch_bounds__(kBlock) void k_after_step(CoupleArgs<T> a, int64_t nseg, int per,
                                                      int L) {
  extern __shared__ int site_table_mem[];
  SiteTable<T> tab{nullptr, nullptr};
  if (Reduce) {
    tab.key = site_table_mem;
    tab.val = reinterpret_cast<T*>(site_table_mem + kSiteTable);
  }
  for (int64_t it = blockIdx.x; it < 2 * nseg; it += gridDim.x)
    after_step_item<T, ST, One, true>(a, it, nseg, per, L, tab);
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

int couple_lane_candidates(int stencil, int out[4]) {
  if (stencil == 1) {
    out[0] = 8;
    out[1] = 16;
    return 2;
  }
  out[0] = 2;
  out[1] = 4;
  out[2] = 8;
  return 3;
}

template <typename T, int ST, int L>
static void launch_couple_lanes(Context* c, const CoupleArgs<T>& a, bool bin, dim3 grid) {
  if (bin && a.single)
    hipLaunchKernelGGL((k_couple<T, false, ST, L, true, true>), grid, dim3(kBlock), 0, c->stream,
                       a);
  else if (bin)
    hipLaunchKernelGGL((k_couple<T, false, ST, L, true, false>), grid, dim3(kBlock), 0, c->stream,
                       a);
  else if (a.single && a.retag)
    hipLaunchKernelGGL((k_couple<T, false, ST, L, false, true, true>), grid, dim3(kBlock), 0,
                       c->stream, a);
  else if (a.single)
    hipLaunchKernelGGL((k_couple<T, false, ST, L, false, true>), grid, dim3(kBlock), 0, c->stream,
                       a);
  else if (a.retag)
    hipLaunchKernelGGL((k_couple<T, false, ST, L, false, false, true>), grid, dim3(kBlock), 0,
                       c->stream, a);
  else
    hipLaunchKernelGGL((k_couple<T, false, ST, L, false, false>), grid, dim3(kBlock), 0, c->stream,
                       a);
}

template <typename T, int ST>
static hipError_t couple_st(Context* c, int substep) {
  using St = Stencil<ST>;
  CoupleArgs<T> a = couple_args<T>(c, substep);
  hipError_t e;
  const int64_t N = a.N;
  // the whole cache is refilled at the first MD step of an interval, and
  // after it was invalidated from outside (new populations, counters or
  // particles): the coupling kernel relies on it covering every stencil
  if (substep == 0 || c->cache_dirty) {
    if ((e = launch_refill_st<T, ST>(c, a)) != hipSuccess) return e;
    c->cache_dirty = false;
    c->retag = true;
  }
  // the first coupling step after a refill takes the sharing of the sites
  // from J's w words and sets up the own-transfer entries
  a.retag = (c->retag || !a.own_on) ? 1 : 0;
  c->retag = false;
  // lanes per particle of the coupling kernel: eight while recording, else
  // the tuned count or the default
  const int L = a.rec ? 8 : (c->tune.couple_lanes > 0 ? c->tune.couple_lanes
                                                        : DirectShape<ST>::kLanes);
  const dim3 cgrid(grid_for((N * L + kBlock - 1) / kBlock, c->tune.part_blocks));
  // with position-dependent forces (never recorded) the kernel also bins
  const bool bin = c->plan.any_forces2 && !a.rec;
  if (ST == 0 && a.rec) {
    hipLaunchKernelGGL((k_couple<T, true, 0, 8, false, false>), cgrid, dim3(kBlock), 0, c->stream,
                       a);
  } else if constexpr (ST == 0) {
    if (L == 2)
      launch_couple_lanes<T, 0, 2>(c, a, bin, cgrid);
    else if (L == 4)
      launch_couple_lanes<T, 0, 4>(c, a, bin, cgrid);
    else
      launch_couple_lanes<T, 0, 8>(c, a, bin, cgrid);
  } else {
    if (L == 16)
      launch_couple_lanes<T, 1, 16>(c, a, bin, cgrid);
    else
      launch_couple_lanes<T, 1, 8>(c, a, bin, cgrid);
  }
  // transfers to shared sites wait until every particle has read J; with
  // position-dependent forces that work rides in extra blocks of the force
  // kernel's launch, which follows anyway
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (c->plan.any_forces2 && !a.rec) return hipSuccess;
  const int64_t nseg = (N * L + kBlock - 1) / kBlock;
  const dim3 agrid(grid_for(2 * nseg, c->tune.part_blocks));
  const int per = (St::kSites + L - 1) / L;
  // (27-site stencils overlap densely: pre-reduce per segment)
  constexpr bool Reduce = ST == 1;
  const size_t lds = Reduce ? kSiteTable * (4 + 3 * sizeof(T)) : 0;
  if (a.single)
    hipLaunchKernelGGL((k_after_step<T, ST, Reduce, true>), agrid, dim3(kBlock), lds, c->stream, a,
                       nseg, per, L);
  else
    hipLaunchKernelGGL((k_after_step<T, ST, Reduce, false>), agrid, dim3(kBlock), lds, c->stream,
                       a, nseg, per, L);
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

// ---------------------------------------------------------------------------
// Own transfers into J (couple_state.hpp): between two MD steps of an
// interval, J lacks the transfers particles keep in their own entries at
// sites they claimed alone.  This writes them there (J = the particle's own
// transfer, the whole transfer of such a site), for calls that read or
// replace J, the populations or the cache in mid-interval.  The entries are
// those of each particle's current stencil (the after-step work rebuilt
// them if it moved); a particle that became non-finite left its transfers
// in J at that step.  32 lanes per particle, one per stencil site.
// ---------------------------------------------------------------------------
template <typename T, int ST>
__global__ __launch_bounds__(kBlock) void k_leave_transfers(CoupleArgs<T> a) {
  using St = Stencil<ST>;
  const int64_t N = a.N;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < N * 32;
       t += (int64_t)gridDim.x * kBlock) {
    const int64_t p = t / 32;
    const int k = (int)(t & 31);
    if (k >= St::kSites) continue;
    const double X[3] = {a.x[p], a.x[N + p], a.x[2 * N + p]};
    if (!(isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2]))) continue;
    const Vec4<T> e = *own_entry<ST>(a, p, k);
    if (e.w != T(0)) continue;
    const RepMD& m = a.md[a.single ? 0 : a.part_rep[p]];
    Cube q;
    St::locate(X, m.g, q);
    int cx, cy, cz, site;
    double w;
    St::site(q, m.g, k, cx, cy, cz, site, w);
    T* j = reinterpret_cast<T*>(a.J + m.site_off + site);
    j[0] = e.x;
    j[1] = e.y;
    j[2] = e.z;
  }
}

template <typename T>
static hipError_t leave_t(Context* c) {
  const CoupleArgs<T> a = couple_args<T>(c, c->subs);
  const dim3 grid(grid_for((a.N * 32 + kBlock - 1) / kBlock, c->tune.part_blocks));
  if (c->p[0].stencil == 1)
    hipLaunchKernelGGL((k_leave_transfers<T, 1>), grid, dim3(kBlock), 0, c->stream, a);
  else
    hipLaunchKernelGGL((k_leave_transfers<T, 0>), grid, dim3(kBlock), 0, c->stream, a);
  return hipGetLastError();
}

// J complete between two MD steps of an interval (nothing to do at an
// LB-step boundary, nor after the interval's last MD step, which left every
// transfer in J).
hipError_t launch_leave_transfers(Context* c) {
  // the entries are valid from the coupling step after a refill until the
  // cache is invalidated (which callers do after leaving the transfers)
  if (c->plan.Ntot == 0 || !c->bound || c->subs <= 0 || c->subs >= c->plan.n_sub ||
      c->retag || c->cache_dirty || c->plan.any_forces2)  // (no own transfers: J is complete)
    return hipSuccess;
  return c->plan.prec == 32 ? leave_t<float>(c) : leave_t<double>(c);
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
  c->retag = true;
  return c->plan.prec == 32 ? refill_t<float>(c) : refill_t<double>(c);
}

// Forget cached corner moments (after the populations, counters or
// particles were replaced from outside): the next MD step refills the cache.
hipError_t invalidate_corner_cache(Context* c) {
  if (c->plan.Ntot > 0) c->cache_dirty = true;
  return hipSuccess;
}

}  // namespace lbmd_impl
