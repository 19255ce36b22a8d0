// State of the particle coupling shared by the coupling kernels and the
// force kernel: the kernel arguments, the corner cache, site claims, the
// moments of a site from its pulled populations, and the work that follows
// an MD step (the direct transfer: plain writes at sites one particle
// claimed, lists for the shared ones).
#pragma once

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
  double* __restrict__ fc_held;  // coupling force of the step (split kick)
  T* __restrict__ cc;
  int32_t* __restrict__ flags;
  const RepMD* __restrict__ md;
  const int32_t* __restrict__ part_rep;
  const int32_t* __restrict__ pid;  // particle identity of each slot (noise counter)
  const Clock* __restrict__ clock;
  double* __restrict__ rec;  // recording: [kAdjRec][N] state and corner velocities of the step
  // per segment (one block-sized stretch of coupling lanes):
  int32_t* __restrict__ lsite;   // transfers of the MD step to shared sites: global site,
  Vec4<T>* __restrict__ ldelta;  //   momentum (x, y, z, -),
  int32_t* __restrict__ lseg;    //   entries in the segment
  int32_t* __restrict__ mlist;   // particles whose stencil moved in the MD step (int2:
                                 //   slot, replica-local index of the new stencil base),
  int32_t* __restrict__ mseg;    //   their number in the segment
  // force cells (position-dependent forces): the coupling kernel bins the
  // particles at their new positions for the force kernel
  int32_t* __restrict__ bin_count;  // [cells] particles per cell (zero on entry)
  int32_t* __restrict__ bin;        // [N] cell of each particle (-1: none)
  int32_t* __restrict__ bin_rank;   // [N] slot inside the cell
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

// Mark a site as a receiver of momentum transfer in this LB interval; a site
// claimed again (by another particle, or by one that changed stencils) is
// flagged as shared in the w word of its transfer entry, which the coupling
// kernel reads together with the transfer itself.  The flag is written only
// by claims (refill, after-step work: never while a coupling kernel runs) and
// cleared with the entry by the LB step; the after-step atomics touch only
// the x, y, z words.  (Recording the claiming particle instead, so that a
// particle re-claiming its own sites keeps them unshared, measured slower:
// the refill's extra compare-and-swap per site cost more than it saved.)
template <typename T>
__device__ __forceinline__ void claim_site(const CoupleArgs<T>& a, int gs) {
  const unsigned long long bit = 1ull << (gs & 63);
  if (atomicOr(a.mark + (gs >> 6), bit) & bit) reinterpret_cast<T*>(a.J + gs)[3] = T(1);
}

// (j, 1/rho) of the post-stream state at site (cx, cy, cz): the 19 pulled
// populations (for a particle whose cached stencil is out of date).
template <typename T>
__device__ __forceinline__ Vec4<T> gather_site_moments(const T* __restrict__ pop, int site_off,
                                                      const Geom& g, int cx, int cy, int cz,
                                                      T rho0) {
  size_t off[19];
  pull_offsets(g, cx, cy, cz, off);
  const T* __restrict__ base = pop + 19 * (size_t)site_off;
  T d[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) d[i] = base[off[i]];
  T drho, jx, jy, jz;
  moments_deviation<T>(d, drho, jx, jy, jz);
  return Vec4<T>{jx, jy, jz, T(1) / (rho0 + drho)};
}

// After every MD step, once every particle has read J: the particles whose
// stencil moved gather the moments of their new sites and claim them, one
// lane per site, before the next step reads them; and the step's transfers
// to shared sites are applied (atomic adds from the segment lists).  The
// two jobs are
// independent (a claim changes no J, the list was fixed by the coupling
// kernel), so each segment of the coupling kernel (kBlock * per entries and
// kBlock / L particles at most) gets one block per job: items [0, nseg)
// take the moved particles, whose dependent loads form the longer chain,
// and items [nseg, 2 nseg) the transfers.  One block runs one item; the
// work runs as a launch of its own (k_after_step) or in extra blocks of
// the force kernel's launch.
// Lanes per particle of the coupling kernel (outside recording): two with
// four corners each for the cube, eight with up to four sites each for the
// three-point stencil.  Fewer lanes repeat less per-particle arithmetic (72
// against 91 us per MD step with one lane per site of the three-point
// stencil) until registers limit the waves in flight.
template <int ST>
struct DirectShape {
  static constexpr int kLanes = ST == 0 ? 2 : 8;
  static constexpr int kPer = (Stencil<ST>::kSites + kLanes - 1) / kLanes;
};

// Pre-reduction of a segment's shared-site transfers in LDS (the launch of
// k_after_step provides the table; the force kernel's extra blocks pass
// none): the entries are summed per distinct site in an open-addressing
// hash table (LDS atomics), then each distinct site receives one device
// atomic per component instead of one per entry.  Pays where stencils
// overlap densely (the 27 sites of the three-point kernel).
// The table holds up to kSiteTable / 2 entries at a time (a longer list is
// taken in chunks); its 16 bytes per slot are dynamic LDS of every block of
// the after-step launch, so its size bounds the blocks resident per CU.
constexpr int kSiteTable = 512;

template <typename T>
struct SiteTable {
  int* key;  // [kSiteTable] global site, -1 = empty
  T* val;    // [3][kSiteTable]
};

template <typename T>
__device__ __forceinline__ void reduce_chunk(const CoupleArgs<T>& a, int64_t base, int n,
                                             SiteTable<T> tab) {
  // table size: the smallest power of two >= 2 n (block-uniform)
  int H = 64, lg = 6;
  while (H < 2 * n) {
    H <<= 1;
    ++lg;
  }
  for (int h = threadIdx.x; h < H; h += kBlock) {
    tab.key[h] = -1;
    tab.val[h] = tab.val[kSiteTable + h] = tab.val[2 * kSiteTable + h] = T(0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += kBlock) {
    const int site = a.lsite[base + e];
    const Vec4<T> dv = a.ldelta[base + e];
    int h = (int)(((uint32_t)site * 2654435761u) >> (32 - lg));
    for (;;) {  // linear probing; the table is at most half full
      const int old = atomicCAS(tab.key + h, -1, site);
      if (old == -1 || old == site) break;
      h = (h + 1) & (H - 1);
    }
    atomicAdd(tab.val + h, dv.x);
    atomicAdd(tab.val + kSiteTable + h, dv.y);
    atomicAdd(tab.val + 2 * kSiteTable + h, dv.z);
  }
  __syncthreads();
  // one lane per (slot, component): the three adds to a site in neighbouring
  // lanes of one instruction
  for (int u = threadIdx.x; u < 3 * H; u += kBlock) {
    const int h = u / 3, comp = u - 3 * h;
    const int site = tab.key[h];
    if (site >= 0) atomicAdd(reinterpret_cast<T*>(a.J + site) + comp, tab.val[comp * kSiteTable + h]);
  }
  __syncthreads();  // the block's next item reuses the table
}

template <typename T>
__device__ __forceinline__ void reduce_segment_transfers(const CoupleArgs<T>& a, int64_t base,
                                                         int n, SiteTable<T> tab) {
  for (int c0 = 0; c0 < n; c0 += kSiteTable / 2)
    reduce_chunk(a, base + c0, n - c0 < kSiteTable / 2 ? n - c0 : kSiteTable / 2, tab);
}

template <typename T, int ST>
__device__ __forceinline__ void after_step_item(const CoupleArgs<T>& a, int64_t it, int64_t nseg,
                                                int per, int L,
                                                SiteTable<T> tab = SiteTable<T>{nullptr, nullptr}) {
  using St = Stencil<ST>;
  if (it < nseg) {
    const int64_t seg = it;
    const int nm = a.mseg[seg] * St::kLanes;
    if (nm == 0) return;
    const T* __restrict__ pop = a.pop[a.clock->cur];
    const int2* __restrict__ ml = reinterpret_cast<const int2*>(a.mlist) + seg * (kBlock / L);
    for (int u = threadIdx.x; u < nm; u += kBlock) {
      const int k = u % St::kLanes;
      if (k >= St::kSites) continue;
      // (particle, replica-local index of its new stencil base)
      const int2 ent = ml[u / St::kLanes];
      const int64_t p = ent.x;
      const RepMD& m = a.md[a.single ? 0 : a.part_rep[p]];
      Cube q;
      q.base[0] = ent.y % m.g.nx;
      q.base[1] = (ent.y / m.g.nx) % m.g.ny;
      q.base[2] = ent.y / (m.g.nx * m.g.ny);
      q.s[0] = q.s[1] = q.s[2] = 0.0;
      int cx, cy, cz, site;
      double w;
      St::site(q, m.g, k, cx, cy, cz, site, w);
      *cache_entry<ST>(a, p, k) =
          gather_site_moments<T>(pop, m.site_off, m.g, cx, cy, cz, (T)m.rho0);
      claim_site(a, m.site_off + site);
    }
  } else {
    const int64_t seg = it - nseg;
    const int n = a.lseg[seg];
    const int64_t base = seg * (int64_t)(kBlock * per);
    if (tab.key && n > 1) {
      reduce_segment_transfers(a, base, n, tab);
      return;
    }
    // one lane per (entry, component): the three adds to one site sit in
    // neighbouring lanes of one instruction and reach the memory side as one
    // request instead of three
    for (int u = threadIdx.x; u < 3 * n; u += kBlock) {
      const int e = u / 3, comp = u - 3 * e;
      const T d = reinterpret_cast<const T*>(a.ldelta + base + e)[comp];
      atomicAdd(reinterpret_cast<T*>(a.J + a.lsite[base + e]) + comp, d);
    }
  }
}

template <typename T>
inline CoupleArgs<T> couple_args(Context* c, int substep) {
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
  a.fc_held = (double*)at(c, L.fc_held);
  a.cc = (T*)at(c, L.cc);
  a.flags = (int32_t*)at(c, L.flags);
  a.md = (const RepMD*)at(c, L.rep_md);
  a.part_rep = (const int32_t*)at(c, L.part_rep);
  a.pid = (const int32_t*)at(c, L.pid);
  a.clock = (const Clock*)at(c, L.clock);
  a.rec = c->rec_part ? c->rec_part + (size_t)substep * kAdjRec * (size_t)c->plan.Ntot : nullptr;
  a.lsite = (int32_t*)at(c, L.slist_site);
  a.ldelta = (Vec4<T>*)at(c, L.slist_delta);
  a.lseg = (int32_t*)at(c, L.seg_count);
  a.mlist = (int32_t*)at(c, L.mlist);
  a.mseg = (int32_t*)at(c, L.seg_count) + c->plan.nseg;
  a.bin_count = (int32_t*)at(c, L.bin_count);
  a.bin = (int32_t*)at(c, L.bin_of);
  a.bin_rank = (int32_t*)at(c, L.bin_rank);
  a.N = c->plan.Ntot;
  a.substep = substep;
  a.variant = c->p[0].variant;
  a.single = c->plan.R == 1 ? 1 : 0;
  return a;
}

}  // namespace lbmd_impl
