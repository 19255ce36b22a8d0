// Host-side context of the library and the kernel launchers behind the C ABI.
//
// A context holds R >= 1 independent periodic systems ("replicas") that
// advance in lockstep: the plain API is the case R = 1.  Replica lattices are
// concatenated in one site index space (each starting at a multiple of 64,
// so a 64-bit mark word never spans two replicas) and particles in one
// particle index space.  Kernels cover all replicas in one launch through
// per-replica tables in device memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/lbmd.h"
#include "lbmd_device.hpp"

namespace lbmd_impl {
using lbmd_dev::CollideConsts;
using lbmd_dev::Geom;

constexpr int kBlock = 256;  // threads per block; site chunks of the LB kernels
constexpr int kRedWidth = 16;
// lb_moments_noalloc: reduction rows in a fixed device array of this
// library, 1024 block rows + the totals row of kRedWidth doubles (131,200
// bytes per GPU)
constexpr int kScratchRows = 1024;
constexpr int kScratchDoubles = (kScratchRows + 1) * kRedWidth;

// Per-replica constants of the LB kernels (run precision T).
template <typename T>
struct RepLB {
  Geom g;
  int site_off;  // first global site of the replica
  int item_off;  // first 256-site work item of the replica
  int rows;      // nx is 64, 128 or 256 and 19 S < 2^32: the collide-stream
                 // kernel's row path
  uint32_t key0, key1, tag0, tag1;
  CollideConsts<T> k;
};

// Per-replica constants of the particle kernels (always FP64).
struct RepMD {
  Geom g;
  int site_off;
  int part_off, N;
  int cell_off;  // first force cell of the replica
  int variant, noise, split_kick, force_model, chain_len;
  int stencil;  // 0 trilinear (8 sites), 1 three-point kernel (27 sites)
  uint32_t key0, key1, tag;
  double rho0, gamma, amp, tau, h;  // amp = sqrt(2 gamma kT / tau): the particle noise
                                    // amplitude before the balance factor (noise_amplitude)
  double inv_m;                     // 1 / particle mass (0 without particles)
  double L[3];
  double f_ext[3];
  double k_bond, r0_bond, wca_eps, wca_sigma;
  int nb[3];  // force-cell grid
  double inv_edge[3];
};

// Device step clock: read by the kernels so that a captured cycle replays
// unchanged; advanced by a one-thread kernel at the end of each LB step.
struct Clock {
  long long t_lb;  // LB steps done
  long long t_md;  // MD steps done at the start of the current LB interval
  int cur;         // population buffer holding the current state
  int pad;
};

// Offsets (bytes) of the regions carved out of the caller's workspace.
struct Layout {
  size_t pop[2];     // [19 * Stot] population deviations, pull storage, per replica
                     // z-plane interleaved (pop_offset in lbmd_device.hpp)
  size_t transfer;   // [Stot] Vec4<T>: pending momentum transfer J (x, y, z) and, in w,
                     // a flag set when the site is claimed more than once in the
                     // current LB interval (shared site; claim_site)
  size_t mark;       // [Stot/64] uint64: bit set <=> J may be non-zero at the site
  size_t rep_lb;     // [R] RepLB<T>
  size_t rep_md;     // [R] RepMD
  size_t item_rep;   // [R + 1] int32: work-item offsets (prefix) for the LB kernels
  size_t part_rep;   // [Ntot] int32: replica of each particle
  size_t pid;        // [Ntot] int32: replica-local identity of the particle in each slot
                     // (its index at binding; the particle noise counter follows it)
  size_t clock;      // Clock
  size_t fcons;      // [3][Ntot] double: conservative force at the current positions
  size_t sort_x;     // [3][Ntot] double: particle sort scratch (positions)
  size_t sort_v;     // [3][Ntot] double: particle sort scratch (velocities)
  size_t sort_img;   // [3][Ntot] int32: particle sort scratch (image counters)
  size_t fc_held;    // [3][Ntot] double: coupling force of the MD step (split kick)
  size_t cc;         // [Ntot][32] T: corner cache, per corner k: jx, jy, jz, 1/rho
  size_t own;        // [Ntot][sites per stencil] Vec4<T>: own transfers (couple_state.hpp)
  size_t owner;      // [Stot] int32: at a stencil's lowest site, a particle whose stencil starts there (-1: none)
  size_t moved_at;   // [Ntot] int64: MD step of each particle's last stencil change
  size_t slist_site;  // [sites per stencil * Ntot] int32: shared-site transfers of an MD step
  size_t slist_delta; // [sites per stencil * Ntot] Vec4<T>: their momenta
  size_t mlist;      // [segments * kBlock / lanes] int4: particles whose stencil moved, new and old base, replica
  size_t seg_count;  // [2][segments] int32: entries per segment of the two lists
  size_t bin_count;  // [2 Ctot + 2] int32: particles per force cell, two halves by MD-step
                     // parity, then the two overflow-list lengths (cell_insert)
  size_t bin_of;     // [Ntot] int32: count entry of each particle's force cell,
                     // half * Ctot + global cell (-1: none)
  size_t bin_slot;   // [Ctot][cell_cap] int32: particles of each cell
  size_t bin_ovf;    // [Ntot] int32: particles past their cell's capacity
  size_t sort_keys;  // [2][Ntot] uint64: spatial sort keys (in, out)
  size_t sort_vals;  // [2][Ntot] int32: particle indices (in, out = the permutation)
  size_t sort_temp;  // radix-sort temporary storage
  size_t flags;      // int32[16]: [0] non-finite particle seen
  size_t partials;   // double[nitems][kRedWidth]
  size_t totals;     // double[R][kRedWidth]
  size_t total;      // bytes needed
};

// Launch shapes (autotuner): blocks in flight of the persistent kernels
// (0 = one block per work item) and lanes per particle of the coupling
// kernel (0 = the default DirectShape; candidates couple_lane_candidates).
struct Tune {
  int lb_blocks;
  int part_blocks;
  int couple_lanes;
};

struct Plan {
  int R;
  int prec;
  int n_sub;
  int64_t Stot;  // padded total sites
  int64_t P;     // sites per population buffer (= Stot; a buffer holds 19 * P values)
  int64_t Ntot;  // particles
  int64_t Ctot;  // force cells
  int cell_cap;  // particle slots per force cell
  int nitems;    // 256-site work items of the LB kernels
  int64_t nseg;  // segments (block-sized stretches) of the widest coupling launch
  int row_replicas;  // replicas on the collide-stream row path (see row_path)
  bool any_forces2;
  std::vector<int64_t> site_off, part_off, cell_off, item_off;
  Layout lay;
};

// Reverse-mode state (one system, force models 0 and 1).  A segment of up
// to K cycles is re-run forward with recording: cycle j reads populations
// from slot j (slot 0 is the caller's saved state, slots 1..K-1 live in the
// adjoint workspace) and records the transfer field and mark words its LB
// step consumed and, per MD step, the particle state and the corner
// velocities it interpolated.  The reverse sweep then walks the recorded
// cycles backwards.
struct AdjLayout {
  size_t slots;    // [K-1][19 * P] T: populations read by cycles 1..K-1
  size_t jrec;     // [K][Stot] Vec4<T>: transfer field at the LB step (valid at marked sites)
  size_t mrec;     // [K][Stot/64] uint64: mark words at the LB step
  size_t prec;     // [K][n_sub][kAdjRec][Ntot] double: particle records
  size_t pbar[2];  // [19 * P] T: adjoint of the stored (post-collision) populations
  size_t jbar;     // [Stot] Vec4<T>: adjoint of the transfer field
  size_t abar;     // [Stot] Vec4<T>: adjoint of (j, rho) read by the MD steps
  size_t xbar, vbar, ubar;  // [3][Ntot] double
  size_t pacc;     // [4][Ntot] double: per particle d/dgamma, d/df_ext
  size_t nuacc;    // [kAdjBlocks][4] double: per block d/dgamma_{bulk, shear, ghost}
  size_t total;
};

constexpr int kAdjRec = 38;       // X[3], V[3], U[8][3], 1/rho[8]
constexpr int kAdjBlocks = 2048;  // persistent grid of the adjoint LB kernel

struct AdjState {
  bool attached = false;
  char* ws = nullptr;
  int K = 0;
  AdjLayout lay;
  int ncyc = 0;     // cycles recorded
  int slot = -1;    // cycle the reverse sweep is in
  int sub = -1;     // next MD step to reverse (-1: the LB step is next)
  int pbar_cur = 0; // pbar buffer holding the adjoint of the current slot's output
  std::vector<const void*> src;  // populations read by each recorded cycle
  std::vector<int64_t> t_lb, t_md;
};

struct Context {
  std::vector<lbmd_params> p;  // per replica
  Plan plan;
  hipStream_t stream;
  char* ws;
  // population buffers the kernels read and write (pull storage); the
  // workspace pair, except while a segment is re-run for the adjoint
  void* popv[2];
  // recording targets of the forward kernels (null when not recording)
  double* rec_part;
  void* rec_J;
  unsigned long long* rec_mark;
  AdjState adj;
  // bound particles (concatenated over replicas)
  void* x;
  void* v;
  int32_t* img;
  bool bound;
  bool cache_dirty;  // the corner cache was invalidated since the last refill
  bool retag;        // a refill ran: the next coupling step sets up the own-transfer entries
  int64_t t_lb, t_md;
  int32_t subs;
  int cur;  // population buffer holding the current state (mirrors Clock::cur)
  int sticky;
  Tune tune;
  bool graph_ok;
  double* scratch_rows;  // this GPU's copy of the lb_moments_noalloc array
};

inline void* at(const Context* c, size_t off) { return c->ws + off; }

// Copy of a per-replica table entry that the whole block reads, through the
// constant address space so that it is fetched with scalar loads into
// scalar registers (a plain load of it through a pointer the kernel could
// also write to is fetched per lane and occupies vector registers).  The
// tables are written only by the host between launches.
template <typename U>
__device__ __forceinline__ U scalar_copy(const U* p) {
  static_assert(sizeof(U) % 4 == 0, "table entries are whole 32-bit words");
  typedef __attribute__((address_space(4))) const int* ConstWords;
  const ConstWords src = (ConstWords)p;
  U out;
  int* dst = reinterpret_cast<int*>(&out);
#pragma unroll
  for (int w = 0; w < (int)(sizeof(U) / 4); ++w) dst[w] = src[w];
  return out;
}

// Launchers (return hipError_t of the launch).
hipError_t launch_collide_stream(Context* c);
hipError_t launch_collide_stream_adjoint(Context* c);
hipError_t launch_couple_adjoint(Context* c);
hipError_t launch_adjoint_fold(Context* c);
hipError_t launch_store_counters(Context* c, void* dst, int64_t t_lb, int64_t t_md);
hipError_t launch_clock_advance(Context* c);
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);
size_t sort_temp_bytes(int64_t N);
hipError_t launch_sort_particles(Context* c, int32_t* d_perm, bool* too_small);
hipError_t launch_moments(Context* c, int rep, void* d_rho, void* d_u, double* d_totals);
hipError_t moments_scratch(double** out);
hipError_t launch_moments_rows(Context* c, void* d_rho, void* d_u, double* rows);
hipError_t launch_get_populations(Context* c, int rep, void* dst);
hipError_t launch_set_populations(Context* c, int rep, const void* src);
hipError_t launch_get_transfer(Context* c, int rep, void* dst);
hipError_t launch_couple(Context* c, int substep);
hipError_t launch_couple_refill_only(Context* c);
hipError_t launch_init_forces(Context* c);
hipError_t launch_init_pid(Context* c);
hipError_t invalidate_corner_cache(Context* c);
// the particles' own transfers into J, between two MD steps of an interval
hipError_t launch_leave_transfers(Context* c);
// lanes per particle the coupling kernel is built for: {2, 4, 8} for the
// trilinear stencil, {8, 16} for the three-point one; returns the count
int couple_lane_candidates(int stencil, int out[4]);
hipError_t launch_forces(Context* c);
hipError_t launch_forces_and_kick(Context* c, int substep);
int64_t force_cells(const lbmd_params* p);
int force_cell_capacity(const lbmd_params* p);
// nx is 64, 128 or 256 and the replica's 19 S population entries have 32-bit
// offsets: the collide-stream kernel's row path (aligned rows, DPP x shift)
inline bool row_path(const lbmd_params& p) {
  return (p.nx == 64 || p.nx == 128 || p.nx == 256) &&
         19.0 * (double)p.nx * p.ny * p.nz < 4294967296.0;
}
int cells_per_axis(const lbmd_params* p, int d);

}  // namespace lbmd_impl
