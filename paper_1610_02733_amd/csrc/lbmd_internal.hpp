// Host-side context of the library and the kernel launchers behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lbmd.h"
#include "lbmd_device.hpp"

namespace lbmd_impl {

// Offsets (bytes) of the regions carved out of the caller's workspace.
struct Layout {
  size_t pop[2];     // [19][S] population deviations, pull storage
  size_t transfer;   // [S] Vec4<T>: pending momentum transfer J (x, y, z, unused)
  size_t mark;       // [ceil(S/64)] uint64: bit set <=> J may be non-zero at the site
  size_t fcons;      // [3][N] double: conservative force at the current positions
  size_t rec_cell;   // [3][N] int32: lower corner of the particle's cube (-1: skipped)
  size_t rec_frac;   // [3][N] double: fractional position inside the cube
  size_t rec_dp;     // [3][N] double: momentum change dP of the current MD step
  size_t cc;         // [32][N] T: corner cache, per corner k: 1/rho, jx, jy, jz
  size_t cc_cell;    // [N] int32: cube (linear index of its lower corner) cached
  size_t cc_stamp;   // [N] int32: LB step + 1 at which the cache was filled
  size_t fc_held;    // [3][N] double: coupling force of the MD step (split kick)
  size_t bin_count;  // [ncell] int32: particles per force cell
  size_t bin_start;  // [ncell + 1] int32: exclusive scan of bin_count
  size_t bin_tiles;  // [ceil(ncell / 1024)] int32: scan tile totals
  size_t bin_of;     // [N] int32: force cell of each particle (-1: none)
  size_t bin_rank;   // [N] int32: slot inside the cell
  size_t bin_sorted; // [N] int32: particles ordered by cell
  size_t flags;      // int32[16]: [0] non-finite particle seen
  size_t partials;   // double[kRedBlocks][kRedWidth]
  size_t totals;     // double[kRedWidth]
  size_t total;      // bytes needed
};

constexpr int kRedBlocks = 512;
constexpr int kRedWidth = 16;
constexpr int kBlock = 256;

struct Context {
  lbmd_params p;
  Layout lay;
  hipStream_t stream;
  char* ws;
  lbmd_dev::Geom geom;
  int64_t S;
  int cur;  // index of the population buffer holding the current state
  // bound particles
  void* x;
  void* v;
  int32_t* img;
  bool bound;
  int64_t t_lb, t_md;
  int32_t subs;
  int sticky;
  // derived collision constants (double; cast per precision at launch)
  double gs, gb, gg, mu, ns[15];
};

inline void* at(const Context* c, size_t off) { return c->ws + off; }

// Launchers (return hipError_t of the launch).
hipError_t launch_collide_stream(Context* c);
hipError_t launch_moments(Context* c, void* d_rho, void* d_u, double* d_totals);
hipError_t launch_get_populations(Context* c, void* dst);
hipError_t launch_set_populations(Context* c, const void* src);
hipError_t launch_get_transfer(Context* c, void* dst);
hipError_t launch_couple(Context* c);
hipError_t launch_init_forces(Context* c);
hipError_t invalidate_corner_cache(Context* c);
hipError_t launch_forces(Context* c);
hipError_t launch_forces_and_kick(Context* c);
int64_t force_cells(const lbmd_params* p);

}  // namespace lbmd_impl
