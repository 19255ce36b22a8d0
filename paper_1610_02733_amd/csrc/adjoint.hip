// Reverse-mode kernels of one coupled cycle (n MD steps, then one LB step;
// Eq. 3-8): the adjoint of the collide-and-stream step and of one MD step of
// the particle coupling.  The forward state they linearise about comes from
// a recorded re-run of the cycle (populations read by the cycle, the transfer
// field and mark words of its LB step, per-MD-step particle records); the
// noise is regenerated from the same counters as in the forward kernels.
//
// Adjoint variables, all with respect to the forward quantity of the same
// name at the matching point of the sweep:
//   pbar  stored (post-collision) populations, pull storage, two buffers
//   jbar  transfer field J (force density of the LB step)
//   abar  (j, rho) of the post-stream state at a site, as read by the MD steps
//   xbar, vbar  particle position and velocity
// Single system (one replica); conservative force constant in time.
#include <algorithm>

#include "particle_geom.hpp"

namespace lbmd_impl {
using namespace lbmd_dev;

template <typename T>
struct AdjLBArgs {
  const T* __restrict__ src;                  // populations the cycle read (slot)
  const T* __restrict__ pin;                  // adjoint of the cycle's output
  T* __restrict__ pout;                       // adjoint of the cycle's input
  const Vec4<T>* __restrict__ jrec;           // J at the LB step (marked sites)
  const unsigned long long* __restrict__ mrec;
  Vec4<T>* __restrict__ jbar;
  const RepLB<T>* __restrict__ rep;
  double* __restrict__ nuacc;                 // [gridDim][4]
  long long t_lb;
};

// ---------------------------------------------------------------------------
// Adjoint of the fused collide-and-stream step, one thread per site r.
//
// Forward: out_i(r) = C_i(f(r), F(r)) with f_i(r) = src_i(r - c_i) (pull) and
// F = g + J(r).  Reverse: the collision adjoint at r turns out-bar(r) into
// f-bar(r) and F-bar(r); the transpose of the pull sends f-bar_i(r) back to
// the stored entry it came from, src-bar_i(r - c_i), written exactly once
// per entry (a push, no atomics).  F-bar is kept where a transfer was
// recorded (the sites the MD steps touched).  The derivatives of the result
// with respect to the relaxation factors are summed per block.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_collide_stream_adjoint(AdjLBArgs<T> a) {
  const RepLB<T>& q = a.rep[0];
  const uint32_t step_lo = (uint32_t)((unsigned long long)a.t_lb & 0xFFFFFFFFull);
  const uint32_t step_hi = (uint32_t)((unsigned long long)a.t_lb >> 32);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < q.g.S; r += gridDim.x * kBlock) {
    int x, y, z;
    site_coords(q.g, r, x, y, z);
    size_t off[19];
    pull_offsets(q.g, x, y, z, off);
    const size_t own = pop_offset(q.g, 0, x, y, z);
    T d[19], dbo[19], dbi[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      d[i] = __builtin_nontemporal_load(a.src + off[i]);
      dbo[i] = __builtin_nontemporal_load(a.pin + own + (size_t)i * q.g.A);
    }
    const bool marked = (a.mrec[r >> 6] >> (r & 63)) & 1ull;
    T Fx = q.k.g[0], Fy = q.k.g[1], Fz = q.k.g[2];
    if (marked) {
      const Vec4<T> jv = a.jrec[r];
      Fx += jv.x;
      Fy += jv.y;
      Fz += jv.z;
    }
    uint32_t hw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (q.k.noise) {
      const Words4 o0 = philox10(Words4{(uint32_t)r, step_lo, q.tag0, step_hi}, q.key0, q.key1);
      const Words4 o1 = philox10(Words4{(uint32_t)r, step_lo, q.tag1, step_hi}, q.key0, q.key1);
      hw[0] = o0.w0; hw[1] = o0.w1; hw[2] = o0.w2; hw[3] = o0.w3;
      hw[4] = o1.w0; hw[5] = o1.w1; hw[6] = o1.w2; hw[7] = o1.w3;
    }
    T Fbx, Fby, Fbz, gb[3];
    collide_deviation_adjoint<T>(d, Fx, Fy, Fz, hw, q.k, dbo, dbi, Fbx, Fby, Fbz, gb);
#pragma unroll
    for (int i = 0; i < 19; ++i)
      __builtin_nontemporal_store(dbi[i], a.pout + off[i]);
    if (marked) a.jbar[r] = Vec4<T>{Fbx, Fby, Fbz, T(0)};
    acc[0] += (double)gb[0];
    acc[1] += (double)gb[1];
    acc[2] += (double)gb[2];
  }
  // block sums, accumulated into this block's own slot (deterministic)
  __shared__ double sh[kBlock / 64][3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double s = acc[k];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) sh[wv][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += sh[w][threadIdx.x];
    a.nuacc[(size_t)blockIdx.x * 4 + threadIdx.x] += s;
  }
}

// Fold of the MD steps' reads into the population adjoint: the MD steps of a
// cycle read rho(r) = sum_i f_i(r) and j(r) = sum_i c_i f_i(r) of the
// post-stream state, so f-bar_i(r) gains rho-bar(r) + c_i . j-bar(r), which
// the pull transpose sends to src-bar_i(r - c_i).  Only marked sites can
// carry a read; abar is cleared for the next cycle.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adjoint_fold(const RepLB<T>* __restrict__ rep,
                                                         const unsigned long long* __restrict__ mrec,
                                                         Vec4<T>* __restrict__ abar,
                                                         T* __restrict__ pout) {
  const Geom& g = rep[0].g;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < g.S; r += gridDim.x * kBlock) {
    if (!((mrec[r >> 6] >> (r & 63)) & 1ull)) continue;
    const Vec4<T> ab = abar[r];
    abar[r] = Vec4<T>{T(0), T(0), T(0), T(0)};
    int x, y, z;
    size_t off[19];
    site_coords(g, r, x, y, z);
    pull_offsets(g, x, y, z, off);
#pragma unroll
    for (int i = 0; i < 19; ++i)
      pout[off[i]] +=
          ab.w + (T)kVel[i][0] * ab.x + (T)kVel[i][1] * ab.y + (T)kVel[i][2] * ab.z;
  }
}

struct AdjMDArgs {
  const double* __restrict__ rec;  // [kAdjRec][N] record of this MD step
  const double* __restrict__ fcons;
  double* __restrict__ xbar;
  double* __restrict__ vbar;
  double* __restrict__ ubar;
  double* __restrict__ pacc;       // [4][N]
  const RepMD* __restrict__ md;
  const int32_t* __restrict__ pid;  // particle identity of each slot (noise counter)
  int64_t N;
  long long t_md;                  // MD step being reversed
};

// ---------------------------------------------------------------------------
// Adjoint of one MD step (Eq. 4-8 with velocity Verlet), eight lanes per
// particle, one per corner k of its cube.  Forward, with s = X - floor(X)
// and w_k(s) the corner weights:
//   u   = sum_k w_k U_k / rho_k          (U_k = j_k [+ J_k in variant 2])
//   Fc  = -gamma (V - u) + A xi,         A = c sqrt(gamma B), c = sqrt(2 kT / tau),
//                                         B = 1 - gamma tau (1/m + S/rho0) / 2,
//                                         S = sum_k w_k^2 (noise_amplitude)
//   J_k += -w_k tau Fc                   (transfer, Eq. 7-8)
//   V1  = V + h (f + Fc);  X' = X + tau V1;  V' = V1 + h (f + Fc)
// Reverse: from X'-bar, V'-bar and J-bar at the corners, the adjoints of X,
// V, Fc, u, gamma and f.  Sums over corners are butterfly sums over the
// lanes; the weights are piecewise linear in X, so their slopes enter
// through both the interpolation and the transfer.  The reads of the
// interpolation then have adjoints
//   j-bar_k += w_k / rho_k u-bar,   rho-bar_k -= w_k / rho_k^2 (U_k . u-bar),
// which Fused adds right here (variant 1: J-bar is not read again in this
// step); in variant 2 the read includes J, so J-bar gains the same j-bar,
// and the adds wait for k_scatter_adjoint until every particle of the step
// has read J-bar.
// ---------------------------------------------------------------------------
template <typename T, bool Fused>
__global__ __launch_bounds__(kBlock) void k_couple_adjoint(AdjMDArgs a,
                                                           const Vec4<T>* __restrict__ jbar,
                                                           Vec4<T>* __restrict__ abar) {
  const RepMD& m = a.md[0];
  const int64_t N = a.N;
  const unsigned long long t_md = (unsigned long long)a.t_md;
  const uint32_t step_lo = (uint32_t)(t_md & 0xFFFFFFFFull), step_hi = (uint32_t)(t_md >> 32);
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < N * kCornerLanes;
       t += (int64_t)gridDim.x * kBlock) {
    const int64_t p = t / kCornerLanes;
    const int k = (int)(t & (kCornerLanes - 1));
    const double* r = a.rec;
    double X[3], V[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      X[d] = r[d * N + p];
      V[d] = r[(3 + d) * N + p];
    }
    if (!isfinite(X[0])) continue;  // skipped by the forward step (all 8 lanes)
    Cube q;
    cube_of(X, m.g, q);
    int cx, cy, cz, site;
    double w;
    corner_of(q, m.g, k, cx, cy, cz, site, w);
    // d w_k / d s_e
    const double a0 = (k & 1) ? q.s[0] : 1.0 - q.s[0], e0 = (k & 1) ? 1.0 : -1.0;
    const double a1 = (k & 2) ? q.s[1] : 1.0 - q.s[1], e1 = (k & 2) ? 1.0 : -1.0;
    const double a2 = (k & 4) ? q.s[2] : 1.0 - q.s[2], e2 = (k & 4) ? 1.0 : -1.0;
    const double dw[3] = {e0 * a1 * a2, a0 * e1 * a2, a0 * a1 * e2};
    const double ir = r[(30 + k) * N + p];
    const double U[3] = {r[(6 + 3 * k) * N + p], r[(7 + 3 * k) * N + p], r[(8 + 3 * k) * N + p]};
    const Vec4<T> jb = jbar[site];
    const double jbv[3] = {(double)jb.x, (double)jb.y, (double)jb.z};
    double u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = oct_sum(w * ir * U[d]);
    // noise amplitude A(gamma, S) and its derivatives (zero where A = 0:
    // gamma = 0, or the balance factor clamped)
    const double S = oct_sum(w * w);
    double dS[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) dS[d] = oct_sum(2.0 * w * dw[d]);
    const double A = m.noise ? noise_amplitude(m, S) : 0.0;
    const double c2 = m.gamma > 0.0 ? m.amp * m.amp / m.gamma : 0.0;  // 2 kT / tau
    const double a_damp = 2.0 * (1.0 - noise_balance(m, S));
    const double dA_dg = A > 0.0 ? c2 * (1.0 - a_damp) / (2.0 * A) : 0.0;
    const double dA_dS = A > 0.0 ? -c2 * m.gamma * m.gamma * m.tau / (4.0 * m.rho0 * A) : 0.0;
    double xi[3] = {0.0, 0.0, 0.0};
    if (m.noise) {
      const Words4 o = philox10(Words4{(uint32_t)a.pid[p], step_lo, m.tag, step_hi}, m.key0,
                                m.key1);
      const uint32_t ws[3] = {o.w0, o.w1, o.w2};
#pragma unroll
      for (int d = 0; d < 3; ++d)
        xi[d] = 3.4641016151377546 * (((double)(ws[d] >> 8) + 0.5) * 5.9604644775390625e-08 - 0.5);
    }
    double Fc[3], xb[3], vb[3], Fcb[3], fb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      Fc[d] = -m.gamma * (V[d] - u[d]) + A * xi[d];
      xb[d] = a.xbar[d * N + p];
      vb[d] = a.vbar[d * N + p];
      const double v1b = vb[d] + m.tau * xb[d];
      Fcb[d] = m.h * (vb[d] + v1b);
      fb[d] = Fcb[d];  // f enters exactly where Fc does
      vb[d] = v1b;
    }
    // transfer J_k += -w_k tau Fc
    const double gk = jbv[0] * Fc[0] + jbv[1] * Fc[1] + jbv[2] * Fc[2];
    double xs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      Fcb[d] += oct_sum(-m.tau * w * jbv[d]);
      xs[d] = -m.tau * gk * dw[d];
    }
    // friction and noise
    double ub[3], gbar = 0.0, nb = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      vb[d] -= m.gamma * Fcb[d];
      ub[d] = m.gamma * Fcb[d];
      gbar += Fcb[d] * (-(V[d] - u[d]) + dA_dg * xi[d]);
      nb += Fcb[d] * xi[d];
    }
    // interpolation weights (through u, the transfer and the noise amplitude)
    const double uk = ir * (U[0] * ub[0] + U[1] * ub[1] + U[2] * ub[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) xs[d] = oct_sum(xs[d] + uk * dw[d]) + nb * dA_dS * dS[d];
    if (k == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        a.xbar[d * N + p] = xb[d] + xs[d];
        a.vbar[d * N + p] = vb[d];
        a.ubar[d * N + p] = ub[d];
        a.pacc[(1 + d) * N + p] += fb[d];
      }
      a.pacc[p] += gbar;
    }
    if (Fused) {
      T* dst = (T*)(abar + site);
      atomicAdd(dst + 0, (T)(w * ir * ub[0]));
      atomicAdd(dst + 1, (T)(w * ir * ub[1]));
      atomicAdd(dst + 2, (T)(w * ir * ub[2]));
      atomicAdd(dst + 3, (T)(-w * ir * uk));
    }
  }
}

// Variant 2: the adds of k_couple_adjoint's reads, after every particle of
// the step has read J-bar; 32 lanes per particle (corner k = lane / 4; lanes
// 0-2 of a corner carry j-bar components, lane 3 rho-bar).  The read
// included the transfer field, so J-bar gains the same j-bar.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_adjoint(AdjMDArgs a, Vec4<T>* __restrict__ abar,
                                                            Vec4<T>* __restrict__ jbar) {
  const RepMD& m = a.md[0];
  const int64_t N = a.N;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < N * 32;
       t += (int64_t)gridDim.x * kBlock) {
    const int64_t p = t >> 5;
    const int sl = (int)(t & 31), k = sl >> 2, c = sl & 3;
    const double* r = a.rec;
    double X[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) X[d] = r[d * N + p];
    if (!isfinite(X[0])) continue;
    Cube q;
    cube_of(X, m.g, q);
    int cx, cy, cz, site;
    double w;
    corner_of(q, m.g, k, cx, cy, cz, site, w);
    const double ir = r[(30 + k) * N + p];
    T* dst = (T*)(abar + site);
    if (c == 3) {
      double dotv = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) dotv += r[(6 + 3 * k + d) * N + p] * a.ubar[d * N + p];
      atomicAdd(dst + 3, (T)(-w * ir * ir * dotv));
    } else {
      const T val = (T)(w * ir * a.ubar[c * N + p]);
      atomicAdd(dst + c, val);
      atomicAdd(((T*)(jbar + site)) + c, val);
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T>
static hipError_t lb_adjoint_t(Context* c) {
  const AdjState& s = c->adj;
  const AdjLayout& L = s.lay;
  const size_t S = (size_t)c->plan.Stot;
  const int j = s.slot;
  AdjLBArgs<T> a;
  a.src = (const T*)s.src[j];
  a.pin = (const T*)(s.ws + L.pbar[s.pbar_cur]);
  a.pout = (T*)(s.ws + L.pbar[1 - s.pbar_cur]);
  a.jrec = (const Vec4<T>*)(s.ws + L.jrec) + (size_t)j * S;
  a.mrec = (const unsigned long long*)(s.ws + L.mrec) + (size_t)j * (S / 64);
  a.jbar = (Vec4<T>*)(s.ws + L.jbar);
  a.rep = (const RepLB<T>*)at(c, c->plan.lay.rep_lb);
  a.nuacc = (double*)(s.ws + L.nuacc);
  a.t_lb = (long long)s.t_lb[j];
  const int blocks = (int)std::min<int64_t>(kAdjBlocks, (c->plan.Stot + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_collide_stream_adjoint<T>, dim3(blocks), dim3(kBlock), 0, c->stream, a);
  return hipGetLastError();
}

hipError_t launch_collide_stream_adjoint(Context* c) {
  return c->plan.prec == 32 ? lb_adjoint_t<float>(c) : lb_adjoint_t<double>(c);
}

static AdjMDArgs md_adjoint_args(Context* c) {
  const AdjState& s = c->adj;
  const AdjLayout& L = s.lay;
  const size_t N = (size_t)c->plan.Ntot;
  AdjMDArgs a;
  a.rec = (const double*)(s.ws + L.prec) +
          ((size_t)s.slot * c->plan.n_sub + (size_t)s.sub) * kAdjRec * N;
  a.fcons = (const double*)at(c, c->plan.lay.fcons);
  a.xbar = (double*)(s.ws + L.xbar);
  a.vbar = (double*)(s.ws + L.vbar);
  a.ubar = (double*)(s.ws + L.ubar);
  a.pacc = (double*)(s.ws + L.pacc);
  a.md = (const RepMD*)at(c, c->plan.lay.rep_md);
  a.pid = (const int32_t*)at(c, c->plan.lay.pid);
  a.N = c->plan.Ntot;
  a.t_md = (long long)(s.t_md[s.slot] + s.sub);
  return a;
}

template <typename T>
static hipError_t couple_adjoint_t(Context* c) {
  const AdjMDArgs a = md_adjoint_args(c);
  Vec4<T>* jbar = (Vec4<T>*)(c->adj.ws + c->adj.lay.jbar);
  Vec4<T>* abar = (Vec4<T>*)(c->adj.ws + c->adj.lay.abar);
  const int64_t N = a.N;
  const dim3 grid((unsigned)((N * kCornerLanes + kBlock - 1) / kBlock));
  if (c->p[0].variant == 1) {
    hipLaunchKernelGGL((k_couple_adjoint<T, true>), grid, dim3(kBlock), 0, c->stream, a,
                       (const Vec4<T>*)jbar, abar);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_couple_adjoint<T, false>), grid, dim3(kBlock), 0, c->stream, a,
                     (const Vec4<T>*)jbar, abar);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter_adjoint<T>, dim3((unsigned)((N * 32 + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, c->stream, a, abar, jbar);
  return hipGetLastError();
}

hipError_t launch_couple_adjoint(Context* c) {
  if (c->plan.Ntot == 0) return hipSuccess;
  return c->plan.prec == 32 ? couple_adjoint_t<float>(c) : couple_adjoint_t<double>(c);
}

template <typename T>
static hipError_t fold_t(Context* c) {
  const AdjState& s = c->adj;
  const size_t S = (size_t)c->plan.Stot;
  const int blocks = (int)std::min<int64_t>(kAdjBlocks, (c->plan.Stot + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_adjoint_fold<T>, dim3(blocks), dim3(kBlock), 0, c->stream,
                     (const RepLB<T>*)at(c, c->plan.lay.rep_lb),
                     (const unsigned long long*)(s.ws + s.lay.mrec) + (size_t)s.slot * (S / 64),
                     (Vec4<T>*)(s.ws + s.lay.abar), (T*)(s.ws + s.lay.pbar[1 - s.pbar_cur]));
  return hipGetLastError();
}

// After the MD steps of a cycle were reversed: their reads into the adjoint
// of the cycle's input populations.
hipError_t launch_adjoint_fold(Context* c) {
  if (c->plan.Ntot == 0) return hipSuccess;
  return c->plan.prec == 32 ? fold_t<float>(c) : fold_t<double>(c);
}

// Counters of a saved state, written on the stream like the rest of it.
__global__ void k_store_counters(long long* __restrict__ dst, long long t_lb, long long t_md) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dst[0] = t_lb;
    dst[1] = t_md;
  }
}

hipError_t launch_store_counters(Context* c, void* dst, int64_t t_lb, int64_t t_md) {
  hipLaunchKernelGGL(k_store_counters, dim3(1), dim3(64), 0, c->stream, (long long*)dst,
                     (long long)t_lb, (long long)t_md);
  return hipGetLastError();
}

}  // namespace lbmd_impl
