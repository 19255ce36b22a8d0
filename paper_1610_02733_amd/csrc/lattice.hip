// Lattice kernels: the fused pull collide-and-stream step (Eq. 3 with the
// MRT collision, fluid noise and Guo forcing of Sec. 2-3), the FP64 moment
// reductions (Eq. 1-2) and population / transfer copies.  All kernels cover
// every replica of a context in one launch.
#include <algorithm>
#include <mutex>

#include "forcing.hpp"
#include "lbmd_internal.hpp"

namespace lbmd_impl {
using namespace lbmd_dev;

// Replica of a 256-site work item: binary search over the item offsets
// (uniform across the block).
__device__ __forceinline__ int replica_of_item(const int32_t* __restrict__ item_off, int R,
                                               int item) {
  int lo = 0, hi = R;  // item_off[lo] <= item < item_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (item_off[mid] <= item)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Fused collide-and-stream, one thread per site, pull scheme.
//
// The source buffer holds post-collision deviations at the site that produced
// them; the thread at site r gathers population i from r - c_i (the
// post-stream state), adds the pending momentum transfer J(r) as the force
// density of this LB step, collides and writes its 19 results at r in the
// other buffer (coalesced).  J is only read where the site's bit in `mark` is
// set (the coupling sets it when it transfers momentum there), and is cleared
// with it (the shared-site flag in w too), so the untouched bulk of
// the lattice costs no transfer traffic.
// In variant 3 (VarC) the interval's transfer already belongs to the state:
// the collision adds it as the momentum and stress increments of the paper's
// variant C and relaxes with the body force alone.  A work item is 256
// consecutive sites of one replica; replica offsets are multiples of 64, so
// one wavefront owns exactly one 64-bit mark word.  Persistent grid: blocks
// stride over the items.
//
// Row path (replicas with nx = 64, 128 or 256: a wavefront is 64 sites of
// one x row and an item holds whole rows).  Every thread loads the 19
// entries at its own x in the rows that the y and z shifts select, so each
// wavefront load is an aligned, contiguous 64-value run; the +-x shift of the
// ten populations with c_x != 0 is then done in registers: a DPP rotation by
// one lane inside the wavefront, and for the two end lanes of a wavefront the
// value of the neighbouring wavefront of the same row (periodic) through LDS.
// Gathering the shifted entries straight from memory instead makes each
// wavefront touch a partial cache line on either side, which a neighbouring
// wavefront fetches again (measured 1.06x the algorithmic traffic).
// ---------------------------------------------------------------------------
template <typename T>
struct StreamArgs {
  T* pop[2];
  Vec4<T>* __restrict__ J;
  unsigned long long* __restrict__ mark;
  const RepLB<T>* __restrict__ rep;
  const int32_t* __restrict__ item_off;
  const Clock* __restrict__ clock;
  Vec4<T>* __restrict__ jrec;                 // recording: J consumed at marked sites
  unsigned long long* __restrict__ mrec;      // recording: mark words
  int R, nitems;
  int varc;  // variant 3: J belongs to the fluid state (fields read j + J)
};

// Values of the x neighbours inside a wavefront: lane l receives v of lane
// l - 1 (from_left; lane 0 receives lane 63) or of lane l + 1 (from_right;
// lane 63 receives lane 0).  DPP wave_ror:1 / wave_rol:1.
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x13C, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x134, 0xF, 0xF, false));
}
__device__ __forceinline__ double from_left(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x13C, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x13C, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x134, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x134, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// With Rec, the transfer field and the mark words the step consumes are also
// copied out for the reverse sweep (the adjoint needs the force density of
// the step and the set of sites the MD steps touched).
// Mode: 0 every replica takes the general path, 1 every replica the row
// path, 2 per replica (a batch mixing both).
template <typename T, bool Rec, bool VarC, int Mode>
__global__ __launch_bounds__(kBlock) void k_collide_stream(StreamArgs<T> a) {
  // populations pulled from x - 1 (c_x = +1) and from x + 1 (c_x = -1)
  constexpr int kFromLeft[5] = {1, 7, 9, 11, 13};
  constexpr int kFromRight[5] = {2, 8, 10, 12, 14};
  // row path: end-lane values of each wavefront, double-buffered by the
  // parity of the block's row-path items (one barrier per such item, so a
  // wavefront writing one buffer has passed the barrier that follows every
  // read of it)
  __shared__ T edge[2][2][kBlock / 64][5];
  const int cur = a.clock->cur;
  const long long t = a.clock->t_lb;
  const T* __restrict__ src = a.pop[cur];
  T* __restrict__ dst = a.pop[1 - cur];
  const uint32_t step_lo = (uint32_t)((unsigned long long)t & 0xFFFFFFFFull);
  const uint32_t step_hi = (uint32_t)((unsigned long long)t >> 32);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int par = 0;
  // General path: workgroups go to the 8 XCDs in turn and each XCD has its
  // own L2, so XCD x takes the x-th contiguous range of the items; the lines
  // that the shifted runs of neighbouring items share are then fetched once
  // (measured on 512 replicas of 24-48 sites per edge: reads 1.20x -> 1.03x
  // the algorithmic bytes).  The row path reads aligned runs and keeps the
  // plain order.
  int item0 = blockIdx.x;
  if (Mode == 0) {
    const int G = gridDim.x, q8 = G / 8, r8 = G % 8, xcd = blockIdx.x % 8;
    item0 = xcd * q8 + (xcd < r8 ? xcd : r8) + blockIdx.x / 8;
  }
  for (int item = item0; item < a.nitems; item += gridDim.x) {
    // the replica is uniform across the block: keep its constants in scalar
    // registers
    const int rr = __builtin_amdgcn_readfirstlane(
        a.R == 1 ? 0 : replica_of_item(a.item_off, a.R, item));
    const RepLB<T> q = scalar_copy(a.rep + rr);
    const int local = (item - q.item_off) * kBlock + threadIdx.x;
    const bool act = local < q.g.S;
    const T* __restrict__ sbase = src + 19 * (size_t)q.site_off;
    int x, y, z;
    site_coords(q.g, act ? local : 0, x, y, z);
    T d[19];
    const bool rows = Mode == 2 ? q.rows != 0 : Mode == 1;
    // general path: 32-bit offsets where the replica's entries allow (uniform)
    const bool off32 = !rows && 19ull * (unsigned long long)q.g.S < (1ull << 32);
    if (rows) {
      // aligned loads at this lane's own x.  Offsets are 32-bit here (the
      // row path is taken only for replicas of fewer than 2^32 / 19 sites):
      // population i of the row (y', z') is at plane(z') + i A + row(y'),
      // with i A folded into the scalar base
      const uint32_t A = (uint32_t)q.g.A;
      const int ym = y == 0 ? q.g.ny - 1 : y - 1, yp = y == q.g.ny - 1 ? 0 : y + 1;
      const int zm = z == 0 ? q.g.nz - 1 : z - 1, zp = z == q.g.nz - 1 ? 0 : z + 1;
      const uint32_t z0 = (uint32_t)z * 19u * A, zl = (uint32_t)zm * 19u * A,
                     zh = (uint32_t)zp * 19u * A;
      const uint32_t r0 = (uint32_t)(y * q.g.nx + x), rl = (uint32_t)(ym * q.g.nx + x),
                     rh = (uint32_t)(yp * q.g.nx + x);
      // (plane, row) of each population's source: z - c_z, y - c_y
      const uint32_t o00 = z0 + r0, o0l = z0 + rl, o0h = z0 + rh;
      const uint32_t ol0 = zl + r0, olh = zl + rh, oll = zl + rl;
      const uint32_t oh0 = zh + r0, ohl = zh + rl, ohh = zh + rh;
      const uint32_t off[19] = {o00, o00, o00, o0l, o0h, ol0, oh0, o0l, o0h, o0h,
                                o0l, ol0, oh0, oh0, ol0, oll, ohh, ohl, olh};
      // every population is read once per step: non-temporal loads keep the
      // stream from evicting the transfer field and the mark words
#pragma unroll
      for (int i = 0; i < 19; ++i)
        d[i] = act ? __builtin_nontemporal_load(sbase + (size_t)i * A + off[i]) : T(0);
      // the x shift: rotate by one lane; the end lanes take the neighbouring
      // wavefront's end value (periodic inside the row of nx/64 wavefronts)
      if (lane == 63) {
#pragma unroll
        for (int j = 0; j < 5; ++j) edge[par][0][wv][j] = d[kFromLeft[j]];
      }
      if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 5; ++j) edge[par][1][wv][j] = d[kFromRight[j]];
      }
      __syncthreads();
      const int wpr = q.g.nx >> 6;  // wavefronts per row: 1, 2 or 4
      const int wl = wv & (wpr - 1), rb = wv - wl;
      const int wleft = rb + ((wl + wpr - 1) & (wpr - 1));
      const int wright = rb + ((wl + 1) & (wpr - 1));
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const T l = from_left(d[kFromLeft[j]]);
        const T r = from_right(d[kFromRight[j]]);
        d[kFromLeft[j]] = lane == 0 ? edge[par][0][wleft][j] : l;
        d[kFromRight[j]] = lane == 63 ? edge[par][1][wright][j] : r;
      }
      par ^= 1;
    } else if (act && off32) {
      // 32-bit offsets inside population i's slab, i A folded into the
      // scalar base (the replica's 19 S entries fit 32 bits)
      const uint32_t A = (uint32_t)q.g.A;
      const int xm = x == 0 ? q.g.nx - 1 : x - 1, xp = x == q.g.nx - 1 ? 0 : x + 1;
      const int ym = y == 0 ? q.g.ny - 1 : y - 1, yp = y == q.g.ny - 1 ? 0 : y + 1;
      const int zm = z == 0 ? q.g.nz - 1 : z - 1, zp = z == q.g.nz - 1 ? 0 : z + 1;
      const uint32_t z0 = (uint32_t)z * 19u * A, zl = (uint32_t)zm * 19u * A,
                     zh = (uint32_t)zp * 19u * A;
      const uint32_t r0 = (uint32_t)(y * q.g.nx), rl = (uint32_t)(ym * q.g.nx),
                     rh = (uint32_t)(yp * q.g.nx);
      const uint32_t X0 = (uint32_t)x, Xl = (uint32_t)xm, Xh = (uint32_t)xp;
      // source (plane, row, column) of each population: z - c_z, y - c_y, x - c_x
      const uint32_t off[19] = {z0 + r0 + X0, z0 + r0 + Xl, z0 + r0 + Xh, z0 + rl + X0,
                                z0 + rh + X0, zl + r0 + X0, zh + r0 + X0, z0 + rl + Xl,
                                z0 + rh + Xh, z0 + rh + Xl, z0 + rl + Xh, zl + r0 + Xl,
                                zh + r0 + Xh, zh + r0 + Xl, zl + r0 + Xh, zl + rl + X0,
                                zh + rh + X0, zh + rl + X0, zl + rh + X0};
      // (plain loads: a shifted run straddles cache lines that the
      // neighbouring wavefront reads too, so the lines should stay in L2)
#pragma unroll
      for (int i = 0; i < 19; ++i) d[i] = sbase[(size_t)i * A + off[i]];
    } else if (act) {
      size_t off[19];
      pull_offsets(q.g, x, y, z, off);
#pragma unroll
      for (int i = 0; i < 19; ++i) d[i] = __builtin_nontemporal_load(sbase + off[i]);
    }
    if (act) {
      const int gsite = q.site_off + local;
      const unsigned long long word = a.mark[gsite >> 6];
      T Fx = q.k.g[0], Fy = q.k.g[1], Fz = q.k.g[2];
      T Jx = T(0), Jy = T(0), Jz = T(0);
      if ((word >> (gsite & 63)) & 1ull) {
        const Vec4<T> jv = a.J[gsite];
        if (VarC) {
          Jx = jv.x;
          Jy = jv.y;
          Jz = jv.z;
        } else {
          Fx += jv.x;
          Fy += jv.y;
          Fz += jv.z;
        }
        a.J[gsite] = Vec4<T>{T(0), T(0), T(0), T(0)};
        if (Rec) a.jrec[gsite] = jv;
      }
      if (Rec && (gsite & 63) == 0) a.mrec[gsite >> 6] = word;
      uint32_t hw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (q.k.noise) {
        const Words4 o0 = philox10(Words4{(uint32_t)local, step_lo, q.tag0, step_hi}, q.key0, q.key1);
        const Words4 o1 = philox10(Words4{(uint32_t)local, step_lo, q.tag1, step_hi}, q.key0, q.key1);
        hw[0] = o0.w0; hw[1] = o0.w1; hw[2] = o0.w2; hw[3] = o0.w3;
        hw[4] = o1.w0; hw[5] = o1.w1; hw[6] = o1.w2; hw[7] = o1.w3;
      }
      collide_deviation<T, VarC>(d, Fx, Fy, Fz, hw, q.k, Jx, Jy, Jz);
      // every population is written once per step: stream the stores past the
      // caches (non-temporal hint)
      T* __restrict__ o = dst + 19 * (size_t)q.site_off;
      if (rows || off32) {
        const uint32_t own = ((uint32_t)z * 19u) * (uint32_t)q.g.A + (uint32_t)(y * q.g.nx + x);
#pragma unroll
        for (int i = 0; i < 19; ++i)
          __builtin_nontemporal_store(d[i], o + (size_t)i * q.g.A + own);
      } else {
        const size_t own = pop_offset(q.g, 0, x, y, z);
#pragma unroll
        for (int i = 0; i < 19; ++i) __builtin_nontemporal_store(d[i], o + own + (size_t)i * q.g.A);
      }
      if ((gsite & 63) == 0 && word) a.mark[gsite >> 6] = 0ull;
    }
  }
}

template <typename T>
static StreamArgs<T> stream_args(Context* c) {
  StreamArgs<T> a;
  a.pop[0] = (T*)c->popv[0];
  a.pop[1] = (T*)c->popv[1];
  a.J = (Vec4<T>*)at(c, c->plan.lay.transfer);
  a.jrec = (Vec4<T>*)c->rec_J;
  a.mrec = c->rec_mark;
  a.mark = (unsigned long long*)at(c, c->plan.lay.mark);
  a.rep = (const RepLB<T>*)at(c, c->plan.lay.rep_lb);
  a.item_off = (const int32_t*)at(c, c->plan.lay.item_rep);
  a.clock = (const Clock*)at(c, c->plan.lay.clock);
  a.R = c->plan.R;
  a.nitems = c->plan.nitems;
  a.varc = c->p[0].variant == 3 ? 1 : 0;
  return a;
}

template <typename T, int Mode>
static void collide_stream_mode(Context* c, const StreamArgs<T>& a, int blocks) {
  if (c->p[0].variant == 3)  // no adjoint for variant 3: never recording
    hipLaunchKernelGGL((k_collide_stream<T, false, true, Mode>), dim3(blocks), dim3(kBlock), 0,
                       c->stream, a);
  else if (a.jrec)
    hipLaunchKernelGGL((k_collide_stream<T, true, false, Mode>), dim3(blocks), dim3(kBlock), 0,
                       c->stream, a);
  else
    hipLaunchKernelGGL((k_collide_stream<T, false, false, Mode>), dim3(blocks), dim3(kBlock), 0,
                       c->stream, a);
}

template <typename T>
static hipError_t collide_stream_t(Context* c) {
  StreamArgs<T> a = stream_args<T>(c);
  const int blocks = c->tune.lb_blocks > 0 ? std::min(c->tune.lb_blocks, a.nitems) : a.nitems;
  // the row path's kernel is instantiated on its own when no replica needs
  // the general one (fewer registers, more waves in flight)
  if (c->plan.row_replicas == c->plan.R)
    collide_stream_mode<T, 1>(c, a, blocks);
  else if (c->plan.row_replicas == 0)
    collide_stream_mode<T, 0>(c, a, blocks);
  else
    collide_stream_mode<T, 2>(c, a, blocks);
  return hipGetLastError();
}

hipError_t launch_collide_stream(Context* c) {
  return c->plan.prec == 32 ? collide_stream_t<float>(c) : collide_stream_t<double>(c);
}

// End of an LB step: advance the device clock (graph-capturable).
__global__ void k_clock_advance(Clock* __restrict__ clk, int md_steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    clk->t_lb += 1;
    clk->t_md += md_steps;
    clk->cur = 1 - clk->cur;
  }
}

hipError_t launch_clock_advance(Context* c) {
  hipLaunchKernelGGL(k_clock_advance, dim3(1), dim3(64), 0, c->stream,
                     (Clock*)at(c, c->plan.lay.clock), (int)c->subs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block reduction of kRedWidth doubles per thread into out[0..kRedWidth).
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
  __syncthreads();
}

// Partial sums, one row per item (PerBlock = false) or, for a single
// replica, one row per block over all its items (PerBlock = true: a bounded
// number of rows).  Columns: 0 sum drho, 1-3 sum j, 4-6 sum J, 7 sum
// |j/rho|^2.  Fields (density, velocity) of replica `field_rep`.
template <typename T, bool PerBlock>
__global__ __launch_bounds__(kBlock) void k_moments(StreamArgs<T> a, int field_rep,
                                                    T* __restrict__ rho_out,
                                                    T* __restrict__ u_out,
                                                    double* __restrict__ partials) {
  const T* __restrict__ src = a.pop[a.clock->cur];
  double acc[kRedWidth];
#pragma unroll
  for (int k = 0; k < kRedWidth; ++k) acc[k] = 0.0;
  for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
    const int rr = a.R == 1 ? 0 : replica_of_item(a.item_off, a.R, item);
    const RepLB<T>& q = a.rep[rr];
    const int local = (item - q.item_off) * kBlock + threadIdx.x;
    if (!PerBlock) {
#pragma unroll
      for (int k = 0; k < kRedWidth; ++k) acc[k] = 0.0;
    }
    if (local < q.g.S) {
      int x, y, z;
      size_t off[19];
      site_coords(q.g, local, x, y, z);
      pull_offsets(q.g, x, y, z, off);
      const T* __restrict__ sbase = src + 19 * (size_t)q.site_off;
      T d[19];
#pragma unroll
      for (int i = 0; i < 19; ++i) d[i] = sbase[off[i]];
      T drho, jx, jy, jz;
      moments_deviation<T>(d, drho, jx, jy, jz);
      const T rho = q.k.rho0 + drho;
      const Vec4<T> jv = a.J[q.site_off + local];
      acc[1] += (double)jx;
      acc[2] += (double)jy;
      acc[3] += (double)jz;
      if (a.varc) {
        jx += jv.x;
        jy += jv.y;
        jz += jv.z;
      }
      if (rr == field_rep) {
        if (rho_out) rho_out[local] = rho;
        if (u_out) {
          const size_t S = (size_t)q.g.S;
          u_out[local] = jx / rho;
          u_out[S + local] = jy / rho;
          u_out[2 * S + local] = jz / rho;
        }
      }
      acc[0] += (double)drho;
      acc[4] += (double)jv.x;
      acc[5] += (double)jv.y;
      acc[6] += (double)jv.z;
      const double ux = (double)jx / (double)rho, uy = (double)jy / (double)rho,
                   uz = (double)jz / (double)rho;
      acc[7] += ux * ux + uy * uy + uz * uz;
    }
    if (!PerBlock) block_reduce_store(acc, partials + (size_t)item * kRedWidth);
  }
  if (PerBlock) block_reduce_store(acc, partials + (size_t)blockIdx.x * kRedWidth);
}

// One block per replica: sum its partial rows (its items' rows, or with
// nrows > 0, for a single replica, rows [0, nrows)), then its particles'
// momentum and kinetic energy (columns 8-10 sum v, 11 sum |v|^2).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_finalize(StreamArgs<T> a,
                                                     const RepMD* __restrict__ md,
                                                     const double* __restrict__ partials,
                                                     const double* __restrict__ v, int64_t Ntot,
                                                     double* __restrict__ totals, int nrows) {
  const int rr = blockIdx.x;
  const int i0 = nrows > 0 ? 0 : a.item_off[rr], i1 = nrows > 0 ? nrows : a.item_off[rr + 1];
  double acc[kRedWidth];
#pragma unroll
  for (int k = 0; k < kRedWidth; ++k) acc[k] = 0.0;
  for (int it = i0 + threadIdx.x; it < i1; it += kBlock)
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] += partials[(size_t)it * kRedWidth + k];
  if (v) {
    const int p0 = md[rr].part_off, n = md[rr].N;
    for (int p = p0 + threadIdx.x; p < p0 + n; p += kBlock) {
      const double vx = v[p], vy = v[Ntot + p], vz = v[2 * Ntot + p];
      acc[8] += vx;
      acc[9] += vy;
      acc[10] += vz;
      acc[11] += vx * vx + vy * vy + vz * vz;
    }
  }
  block_reduce_store(acc, totals + (size_t)rr * kRedWidth);
}

template <typename T>
static hipError_t moments_t(Context* c, int rep, void* d_rho, void* d_u, double* d_totals) {
  StreamArgs<T> a = stream_args<T>(c);
  double* partials = (double*)at(c, c->plan.lay.partials);
  const int blocks = c->tune.lb_blocks > 0 ? std::min(c->tune.lb_blocks, a.nitems) : a.nitems;
  hipLaunchKernelGGL((k_moments<T, false>), dim3(blocks), dim3(kBlock), 0, c->stream, a, rep,
                     (T*)d_rho, (T*)d_u, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !d_totals) return e;
  hipLaunchKernelGGL(k_finalize<T>, dim3(c->plan.R), dim3(kBlock), 0, c->stream, a,
                     (const RepMD*)at(c, c->plan.lay.rep_md), partials,
                     (const double*)(c->bound ? c->v : nullptr), c->plan.Ntot, d_totals, 0);
  return hipGetLastError();
}

hipError_t launch_moments(Context* c, int rep, void* d_rho, void* d_u, double* d_totals) {
  return c->plan.prec == 32 ? moments_t<float>(c, rep, d_rho, d_u, d_totals)
                            : moments_t<double>(c, rep, d_rho, d_u, d_totals);
}

// ---------------------------------------------------------------------------
// Moments without workspace scratch (lb_moments_noalloc): the reduction rows
// live in a fixed device array of this library instead of the context's
// workspace.  At most kScratchRows blocks, each summing the items it strides
// over into one row, then the totals row.  Every call overwrites all the
// rows it reads, so nothing needs clearing; calls that overlap on one GPU
// (two streams) race on the array.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};
}  // namespace

// Device address of this GPU's copy of the array (current device), looked
// up once per device; in host code the array's name is not a device address.
hipError_t moments_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

template <typename T>
static hipError_t moments_rows_t(Context* c, void* d_rho, void* d_u, double* rows) {
  StreamArgs<T> a = stream_args<T>(c);
  const int blocks = std::min(kScratchRows, a.nitems);
  hipLaunchKernelGGL((k_moments<T, true>), dim3(blocks), dim3(kBlock), 0, c->stream, a, 0,
                     (T*)d_rho, (T*)d_u, rows);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize<T>, dim3(1), dim3(kBlock), 0, c->stream, a,
                     (const RepMD*)at(c, c->plan.lay.rep_md), rows,
                     (const double*)(c->bound ? c->v : nullptr), c->plan.Ntot,
                     rows + (size_t)kScratchRows * kRedWidth, blocks);
  return hipGetLastError();
}

hipError_t launch_moments_rows(Context* c, void* d_rho, void* d_u, double* rows) {
  return c->plan.prec == 32 ? moments_rows_t<float>(c, d_rho, d_u, rows)
                            : moments_rows_t<double>(c, d_rho, d_u, rows);
}

// ---------------------------------------------------------------------------
// Copies between pull storage and the plain post-stream layout of one
// replica ([19][S] and [3][S] arrays in the run precision).
// ---------------------------------------------------------------------------
// Variant 3 (pend != nullptr): a copy out adds the increments of the
// transfer the site has received in the current interval (J at marked
// sites), so that it shows the populations as the paper's variant C holds
// them after each MD step.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy_pop(T* __restrict__ pop, int site_off,
                                                     Geom g, T* __restrict__ plain, int to_plain,
                                                     const Vec4<T>* __restrict__ pend,
                                                     const unsigned long long* __restrict__ mark,
                                                     const RepLB<T>* __restrict__ rep, int rr) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= g.S) return;
  int x, y, z;
  size_t off[19];
  site_coords(g, r, x, y, z);
  pull_offsets(g, x, y, z, off);
  const size_t S = (size_t)g.S;
  T* __restrict__ base = pop + 19 * (size_t)site_off;
  if (!to_plain) {
#pragma unroll
    for (int i = 0; i < 19; ++i) base[off[i]] = plain[(size_t)i * S + r];
    return;
  }
  T d[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) d[i] = base[off[i]];
  const int gs = site_off + r;
  if (pend && ((mark[gs >> 6] >> (gs & 63)) & 1ull)) {
    const Vec4<T> jv = pend[gs];
    const CollideConsts<T>& k = rep[rr].k;
    T drho, jx, jy, jz, sm[6], dd[19];
    moments_deviation<T>(d, drho, jx, jy, jz);
    varc_stress<T>(jx, jy, jz, T(1) / (k.rho0 + drho), jv.x, jv.y, jv.z, k.hb, k.hs, sm);
    mode_increments_to_pops<T>(jv.x, jv.y, jv.z, sm, dd);
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] += dd[i];
  }
#pragma unroll
  for (int i = 0; i < 19; ++i) plain[(size_t)i * S + r] = d[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_get_transfer(const Vec4<T>* __restrict__ J, int site_off,
                                                         int S, T* __restrict__ out) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= S) return;
  const Vec4<T> jv = J[site_off + r];
  out[r] = jv.x;
  out[(size_t)S + r] = jv.y;
  out[2 * (size_t)S + r] = jv.z;
}

template <typename T>
static hipError_t copy_t(Context* c, int rep, void* plain, int what) {
  const lbmd_params& p = c->p[rep];
  Geom g;
  g.nx = p.nx;
  g.ny = p.ny;
  g.nz = p.nz;
  g.S = p.nx * p.ny * p.nz;
  g.A = p.nx * p.ny;
  g.inv_nx = 1.0 / p.nx;
  g.inv_ny = 1.0 / p.ny;
  const int blocks = (g.S + kBlock - 1) / kBlock;
  const int site_off = (int)c->plan.site_off[rep];
  if (what == 2) {
    hipLaunchKernelGGL(k_get_transfer<T>, dim3(blocks), dim3(kBlock), 0, c->stream,
                       (const Vec4<T>*)at(c, c->plan.lay.transfer), site_off, g.S, (T*)plain);
    return hipGetLastError();
  }
  T* pop = (T*)c->popv[c->cur];
  const bool pend = c->p[0].variant == 3;
  hipLaunchKernelGGL(k_copy_pop<T>, dim3(blocks), dim3(kBlock), 0, c->stream, pop,
                     site_off, g, (T*)plain, what == 0 ? 1 : 0,
                     pend ? (const Vec4<T>*)at(c, c->plan.lay.transfer) : nullptr,
                     (const unsigned long long*)at(c, c->plan.lay.mark),
                     (const RepLB<T>*)at(c, c->plan.lay.rep_lb), rep);
  return hipGetLastError();
}

hipError_t launch_get_populations(Context* c, int rep, void* dst) {
  return c->plan.prec == 32 ? copy_t<float>(c, rep, dst, 0) : copy_t<double>(c, rep, dst, 0);
}
hipError_t launch_set_populations(Context* c, int rep, const void* src) {
  return c->plan.prec == 32 ? copy_t<float>(c, rep, (void*)src, 1)
                            : copy_t<double>(c, rep, (void*)src, 1);
}
hipError_t launch_get_transfer(Context* c, int rep, void* dst) {
  return c->plan.prec == 32 ? copy_t<float>(c, rep, dst, 2) : copy_t<double>(c, rep, dst, 2);
}

// ---------------------------------------------------------------------------
// Plain device copy with 16-byte non-temporal loads and stores: the
// read+write streaming ceiling the roofline of the collide-stream kernel is
// set against (and the known-size dispatch the HBM byte counters are
// calibrated with).
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_stream_copy(const v4f* __restrict__ src,
                                                        v4f* __restrict__ dst, size_t n4) {
  for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n4;
       t += (size_t)gridDim.x * kBlock)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + t), dst + t);
}

// One 16-byte element per thread over the whole range (a persistent grid of
// a few blocks per CU measured 10-20% slower).
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t stream) {
  const size_t n4 = bytes / 16;
  const size_t want = (n4 + kBlock - 1) / kBlock;
  const unsigned grid = (unsigned)std::max<size_t>(1, std::min<size_t>(want, (size_t)1 << 30));
  hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(kBlock), 0, stream, (const v4f*)src,
                     (v4f*)dst, n4);
  return hipGetLastError();
}

}  // namespace lbmd_impl
