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
  // the particle's own transfer at each site of its stencil in this LB
  // interval (x, y, z) and, in w, whether the site is shared (non-zero: the
  // transfer of the site is read from and added to J), [N][sites per stencil]
  Vec4<T>* __restrict__ own;
  int32_t* __restrict__ owner;     // [Stot] at a stencil's lowest site: its particle (owner_of_shared)
  long long* __restrict__ moved_at;  // [N] MD step (global count) of the last stencil change
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
  int32_t* __restrict__ mlist;   // particles whose stencil moved in the MD step (int4:
                                 //   slot, replica-local indices of the new and old
                                 //   stencil bases, replica),
  int32_t* __restrict__ mseg;    //   their number in the segment
  // force cells (position-dependent forces): the coupling kernel bins the
  // particles at their new positions for the force kernel (cell_insert)
  int32_t* __restrict__ bin_count;  // [2][cells] particles per cell, then [2] overflow
                                    //   lengths; the half of the step's parity is zero
                                    //   on entry
  int32_t* __restrict__ bin;        // [N] count entry of each particle: half * cells + cell
                                    //   (-1: none)
  int32_t* __restrict__ bin_slot;   // [cells][cell_cap] particles of each cell
  int32_t* __restrict__ bin_ovf;    // [N] particles past their cell's capacity
  int64_t ncells;
  int cell_cap;
  int64_t N;    // particles over all replicas
  int substep;  // MD step inside the LB interval
  int retag;    // the cache was refilled for this step: sharing comes from the w words of J
  int last;     // the interval's last MD step: every transfer is left in J
  int own_on;   // own transfers in use (else every step reads J and leaves its transfers there)
  int final_step;  // the interval's last MD step: the own entries and the cache of a
                   // particle that changes stencils are not needed after it (the next
                   // interval starts with a refill)
  int variant;
  int single;   // one replica: its constants are uniform across the grid
};

// Cache entry k of particle p: (jx, jy, jz, 1/rho) of stencil site k.
// Force cells.  Positions at MD step t (global count) are binned into the
// half t mod 2 of the double-buffered counts, and each particle's bin entry
// is its index in the counts (half * cells + cell), so the force kernel
// needs no step count.  The coupling kernel of MD step t, which bins into
// one half, clears the other at each particle's previous entry (the half
// the force kernel of the step before has read), so a half is zero again
// before the next binning into it, with no pass over all cells.
__device__ __forceinline__ int bin_parity(const Clock* clk, int pos_step) {
  return (int)((clk->t_md + pos_step) & 1);
}

// Particle p into cell cb: the first cap particles of a cell take its slots,
// later ones go to the overflow list (its length at ovf_n), which the force
// kernel scans in full, so no capacity bounds the result.
__device__ __forceinline__ void cell_insert(int32_t* __restrict__ cnt, int32_t* __restrict__ slot,
                                            int32_t* __restrict__ ovf, int32_t* __restrict__ ovf_n,
                                            int cap, int cb, int p) {
  const int r = atomicAdd(cnt + cb, 1);
  if (r < cap)
    slot[(int64_t)cb * cap + r] = p;
  else
    ovf[atomicAdd(ovf_n, 1)] = p;
}

template <int ST = 0, typename T>
__device__ __forceinline__ Vec4<T>* cache_entry(const CoupleArgs<T>& a, int64_t p, int k) {
  return reinterpret_cast<Vec4<T>*>(a.cc) + (size_t)p * Stencil<ST>::kSites + k;
}

// Own-transfer entry k of particle p (see CoupleArgs::own).
template <int ST = 0, typename T>
__device__ __forceinline__ Vec4<T>* own_entry(const CoupleArgs<T>& a, int64_t p, int k) {
  return a.own + (size_t)p * Stencil<ST>::kSites + k;
}

// Mark a site as a receiver of momentum transfer in this LB interval; a site
// claimed again (by another particle, or by one that changed stencils) is
// flagged as shared in the w word of its transfer entry.  The flag is
// written only by claims (refill, after-step work: never while a coupling
// kernel runs) and cleared with the entry by the LB step; the after-step
// atomics touch only the x, y, z words.  Returns whether the site was
// claimed before.  (Recording the claimant with a compare-and-swap in the w
// word instead measured slower.)
template <typename T>
__device__ __forceinline__ bool claim_site(const CoupleArgs<T>& a, int gs) {
  const unsigned long long bit = 1ull << (gs & 63);
  if (atomicOr(a.mark + (gs >> 6), bit) & bit) {
    reinterpret_cast<T*>(a.J + gs)[3] = T(1);
    return true;
  }
  return false;
}

// Own transfers (CoupleArgs::own).  A site that a particle claimed alone in
// the refill has that particle as its only reader and writer until another
// particle claims it, so the particle keeps its transfer there in its own
// entry (read and written with its cache, contiguous) instead of J
// (scattered lines), and leaves it in J only when it leaves the site, at the
// interval's last MD step, or when the library needs J complete in between
// (launch_leave_transfers).  For sites claimed after a stencil change, the
// particle's next MD step takes the decision from J, as after a refill.
//
// Finding the particle that holds a site alone: every particle records
// itself at the lowest site of its stencil (the refill, and the after-step
// work when its stencil moved; a plain store, last writer wins), and the
// coupling kernel clears the record of a stencil its particle leaves.  A
// particle q that holds site s alone is the only one whose stencil held s in
// this interval, so no other particle wrote or cleared the records of the
// W^3 stencil bases that contain s, and q wrote its own base's record: that
// record names q.  (A cleared or overwritten record belonged to a stencil
// two particles held in the interval, which holds no site alone.)  Records
// are -1 where no particle has been; any other record naming a particle
// whose current stencil does not start there (an earlier binding, a
// particle that stopped) is stale and skipped.
//
// owner_of_shared runs when particle p's claim found site gs claimed before,
// in the after-step work between coupling kernels: the holder q's transfer
// so far goes to J and q's entry is marked shared, so that from the next MD
// step on both read and add to J.  A q that left its stencil in this very
// step has left its transfers in J already; an undecided entry takes its
// flag from J.
// The records of the W^3 stencil bases that contain site (sx, sy, sz) of a
// replica (owner_of_shared), loaded together.
template <int ST>
struct BaseRecords {
  static constexpr int W = ST == 0 ? 2 : 3;  // sites per axis
  int bx[W], by[W], bz[W];                   // the bases per axis (wrapped)
  int32_t rec[W * W * W];                    // base (ox, oy, oz) at ox + W (oy + W oz)
};

template <int ST, typename T>
__device__ __forceinline__ void load_base_records(const CoupleArgs<T>& a, const RepMD& m, int sx,
                                                  int sy, int sz, BaseRecords<ST>& r) {
  constexpr int W = BaseRecords<ST>::W;
#pragma unroll
  for (int o = 0; o < W; ++o) {
    r.bx[o] = cell_of(sx - o, m.g.nx);
    r.by[o] = cell_of(sy - o, m.g.ny);
    r.bz[o] = cell_of(sz - o, m.g.nz);
  }
#pragma unroll
  for (int d = 0; d < W * W * W; ++d)
    r.rec[d] = a.owner[m.site_off + r.bx[d % W] +
                       m.g.nx * (r.by[(d / W) % W] + m.g.ny * r.bz[d / (W * W)])];
}

// Candidate q (the record of the stencil base (bx, by, bz), the site at
// offset (ox, oy, oz) from it): if q's current stencil starts there and q
// holds the site alone, its transfer so far goes to J and its entry turns
// shared.
template <typename T, int ST>
__device__ __forceinline__ void notify_holder(const CoupleArgs<T>& a, const RepMD& m, int rep,
                                              int gs, int64_t p, int64_t q, int ox, int oy,
                                              int oz, int bx, int by, int bz, long long now) {
  using St = Stencil<ST>;
  constexpr int W = BaseRecords<ST>::W;
  const int64_t N = a.N;
  if (q == p || q < 0 || q >= N) return;
  Vec4<T>* e = own_entry<ST>(a, q, ox + W * (oy + W * oz));
  // everything that decides, in one round of loads
  const int rq = a.single ? 0 : a.part_rep[q];
  const long long mv = a.moved_at[q];
  const double X[3] = {a.x[q], a.x[N + q], a.x[2 * N + q]};
  const Vec4<T> ev = *e;
  if (rq != rep || mv == now || ev.w != T(0)) return;  // (undecided: the flag is in J)
  if (!(isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2]))) return;
  Cube c;
  St::locate(X, m.g, c);
  if (c.base[0] != bx || c.base[1] != by || c.base[2] != bz) return;
  T* j = reinterpret_cast<T*>(a.J + gs);
  j[0] = ev.x;
  j[1] = ev.y;
  j[2] = ev.z;
  e->w = T(1);
}

// All W^3 records loaded beforehand (the cube: 8).
template <typename T, int ST>
__device__ __forceinline__ void owner_of_shared(const CoupleArgs<T>& a, const RepMD& m, int rep,
                                                int gs, int64_t p, const BaseRecords<ST>& r) {
  constexpr int W = BaseRecords<ST>::W;
  const long long now = (long long)(a.clock->t_md + a.substep);
#pragma unroll
  for (int d = 0; d < W * W * W; ++d) {
    const int ox = d % W, oy = (d / W) % W, oz = d / (W * W);
    notify_holder<T, ST>(a, m, rep, gs, p, r.rec[d], ox, oy, oz, r.bx[ox], r.by[oy], r.bz[oz],
                         now);
  }
}

// The same one plane of W^2 records at a time (the three-point stencil's 27
// records would hold too many registers at once), for site (sx, sy, sz).
template <typename T, int ST>
__device__ __forceinline__ void owner_of_shared_planes(const CoupleArgs<T>& a, const RepMD& m,
                                                       int rep, int gs, int64_t p, int sx, int sy,
                                                       int sz) {
  constexpr int W = BaseRecords<ST>::W;
  const long long now = (long long)(a.clock->t_md + a.substep);
  int bx[W], by[W];
#pragma unroll
  for (int o = 0; o < W; ++o) {
    bx[o] = cell_of(sx - o, m.g.nx);
    by[o] = cell_of(sy - o, m.g.ny);
  }
#pragma unroll 1
  for (int oz = 0; oz < W; ++oz) {
    const int bz = cell_of(sz - oz, m.g.nz);
    int32_t rec[W * W];
#pragma unroll
    for (int d = 0; d < W * W; ++d)
      rec[d] = a.owner[m.site_off + bx[d % W] + m.g.nx * (by[d / W] + m.g.ny * bz)];
#pragma unroll
    for (int d = 0; d < W * W; ++d)
      notify_holder<T, ST>(a, m, rep, gs, p, rec[d], d % W, d / W, oz, bx[d % W], by[d / W], bz,
                           now);
  }
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

// The after-step work of one coupling segment (kBlock coupling lanes), in
// two parts: the particles of the segment whose stencil moved (the new
// stencil's cache entries, claims and records) and the segment's transfers
// to shared sites.
// Own: own transfers in use (CoupleArgs::own_on; the standalone after-step
// launch always, the force kernel's extra blocks never), so that the force
// kernel carries none of the holder lookup's registers.
// Whether an after-step item loads its count together with the thread's
// first entry (after_step_item): the cube's standalone launch only.
template <int ST, bool Own>
constexpr bool kAfterStepPrefetch = ST == 0 && Own;

// ent0: this thread's entry of its first pass, loaded with the count when
// kAfterStepPrefetch (see after_step_item).
template <typename T, int ST, bool One, bool Own>
__device__ __forceinline__ void after_step_movers(const CoupleArgs<T>& a, int64_t seg, int nmv,
                                                  int L, const int4& ent0) {
  using St = Stencil<ST>;
  const T* __restrict__ pop = a.pop[a.clock->cur];
  // One (a single replica): its constants read once, before any store
  // (uniform, scalar loads)
  RepMD m1;
  if constexpr (One) m1 = a.md[0];
  const int nm = nmv * St::kLanes;
  const int4* __restrict__ ml = reinterpret_cast<const int4*>(a.mlist) + seg * (kBlock / L);
  for (int u = threadIdx.x; u < nm; u += kBlock) {
    const int k = u % St::kLanes;
    if (k >= St::kSites) continue;
    // (particle, replica-local indices of its new and old stencil bases,
    // replica)
    const int4 ent = kAfterStepPrefetch<ST, Own> && u < kBlock ? ent0 : ml[u / St::kLanes];
    const int64_t p = ent.x;
    const RepMD& m = One ? m1 : a.md[a.single ? 0 : ent.w];
    Cube q;
    q.base[0] = ent.y % m.g.nx;
    q.base[1] = (ent.y / m.g.nx) % m.g.ny;
    q.base[2] = ent.y / (m.g.nx * m.g.ny);
    q.s[0] = q.s[1] = q.s[2] = 0.0;
    int cx, cy, cz, site;
    double w;
    St::site(q, m.g, k, cx, cy, cz, site, w);
    // a site of the old stencil was claimed by this particle already, so
    // no other particle holds it alone; for the others, the records of the
    // stencils that may hold it are loaded along with the gather
    constexpr int W = ST == 0 ? 2 : 3;
    int ox = cx - ent.z % m.g.nx, oy = cy - (ent.z / m.g.nx) % m.g.ny,
        oz = cz - ent.z / (m.g.nx * m.g.ny);
    ox += ox < 0 ? m.g.nx : 0;
    oy += oy < 0 ? m.g.ny : 0;
    oz += oz < 0 ? m.g.nz : 0;
    const bool was_mine = ox < W && oy < W && oz < W;
    constexpr bool own_on = Own;
    const int rec_site = m.site_off + ent.y;
    BaseRecords<ST> recs;
    // (the 27 records of the three-point stencil wait for the claim and are
    // read a plane at a time: loaded with the gather they cost more
    // registers than the round trip they save)
    if (ST == 0 && own_on && !was_mine) load_base_records<ST>(a, m, cx, cy, cz, recs);
    *cache_entry<ST>(a, p, k) =
        gather_site_moments<T>(pop, m.site_off, m.g, cx, cy, cz, (T)m.rho0);
    // whether the particle holds the new site alone is read from J at its
    // next MD step (w = 2: undecided): another particle that changed
    // stencils in the same step may claim the same site in this very
    // launch, after this claim
    *own_entry<ST>(a, p, k) = Vec4<T>{T(0), T(0), T(0), T(2)};
    if (claim_site(a, m.site_off + site) && own_on && !was_mine) {
      const int rep = a.single ? 0 : ent.w;
      if (ST == 0)
        owner_of_shared<T, ST>(a, m, rep, m.site_off + site, p, recs);
      else
        owner_of_shared_planes<T, ST>(a, m, rep, m.site_off + site, p, cx, cy, cz);
    }
    // the particle's record at its new base, after every lane of its wave
    // has read the records (one of them may be this very one): the lanes
    // of one wavefront share one in-order memory stream, so a compiler
    // barrier at wavefront scope suffices
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (k == 0 && own_on) a.owner[rec_site] = (int32_t)p;
  }
}

// pre: site0, dv0 hold entry threadIdx.x / 3 of the segment, loaded with the
// count (the cube only, see after_step_item).
template <typename T>
__device__ __forceinline__ void after_step_lists(const CoupleArgs<T>& a, int64_t seg, int n,
                                                 int per, SiteTable<T> tab, bool pre,
                                                 int site0, const Vec4<T>& dv0) {
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
    const bool first = pre && u < kBlock;
    const T d = first ? (comp == 0 ? dv0.x : (comp == 1 ? dv0.y : dv0.z))
                      : reinterpret_cast<const T*>(a.ldelta + base + e)[comp];
    atomicAdd(reinterpret_cast<T*>(a.J + (first ? site0 : a.lsite[base + e])) + comp, d);
  }
}

// Items [0, nseg) are the segments' moved particles, [nseg, 2 nseg) their
// shared-site transfers (one block each in k_after_step and in the force
// kernel's extra blocks).
template <typename T, int ST, bool One, bool Own>
__device__ __forceinline__ void after_step_item(const CoupleArgs<T>& a, int64_t it, int64_t nseg,
                                                int per, int L,
                                                SiteTable<T> tab = SiteTable<T>{nullptr, nullptr}) {
  // For the cube, each item loads its count together with this thread's
  // first entry (one round trip instead of two; 6.2 against 6.4 us per MD
  // step on the 256^3 workload).  The entry lies inside the segment's region
  // whatever the count (a mover region holds kBlock / L entries with L at
  // most the cube's 8 lanes, a transfer region kBlock * per), and one past
  // the count is stale and left unused.  The three-point stencil's items do
  // without: the registers held across its table's set-up cost more; so do
  // the force kernel's extra blocks (Own false), whose registers the force
  // lanes share (14.2 against 16.8 us per MD step on the 128^3 polymer).
  constexpr bool kPre = kAfterStepPrefetch<ST, Own>;
  if (it < nseg) {
    int4 ent0 = make_int4(0, 0, 0, 0);
    if constexpr (kPre)
      ent0 = reinterpret_cast<const int4*>(a.mlist)[it * (kBlock / L) +
                                                    threadIdx.x / Stencil<ST>::kLanes];
    const int nmv = a.mseg[it];
    if (nmv > 0) after_step_movers<T, ST, One, Own>(a, it, nmv, L, ent0);
  } else {
    const int64_t sg = it - nseg;
    const bool pre = kPre && !tab.key;
    int site0 = 0;
    Vec4<T> dv0{T(0), T(0), T(0), T(0)};
    if (pre) {
      const int64_t e0 = sg * (int64_t)(kBlock * per) + threadIdx.x / 3;
      site0 = a.lsite[e0];
      dv0 = a.ldelta[e0];
    }
    const int n = a.lseg[sg];
    if (n > 0) after_step_lists<T>(a, sg, n, per, tab, pre, site0, dv0);
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
  a.own = (Vec4<T>*)at(c, L.own);
  a.owner = (int32_t*)at(c, L.owner);
  a.moved_at = (long long*)at(c, L.moved_at);
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
  a.bin_slot = (int32_t*)at(c, L.bin_slot);
  a.bin_ovf = (int32_t*)at(c, L.bin_ovf);
  a.ncells = c->plan.Ctot;
  a.cell_cap = c->plan.cell_cap;
  a.N = c->plan.Ntot;
  a.substep = substep;
  // Own transfers pay where particles mostly keep their sites to themselves.
  // Along bonded chains most particles that change cubes land on sites a
  // neighbour holds, and finding the holders costs more than reading J:
  // there every MD step reads the sharing and the transfer from J and
  // leaves its transfers in J, as the first step of an interval does.
  a.own_on = c->plan.any_forces2 ? 0 : 1;
  a.retag = a.own_on ? 0 : 1;
  a.last = (substep == c->plan.n_sub - 1 || !a.own_on) ? 1 : 0;
  a.final_step = substep == c->plan.n_sub - 1 ? 1 : 0;
  a.variant = c->p[0].variant;
  a.single = c->plan.R == 1 ? 1 : 0;
  return a;
}

}  // namespace lbmd_impl
