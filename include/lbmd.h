/*
 * lbmd.h -- C ABI of the MI355X fluctuating lattice-Boltzmann / MD
 * dissipative-coupling library (Tretyakov & Duenweg, arXiv:1610.02733).
 *
 * Units are lattice units: lattice spacing a = 1, LB time step tau_LB = 1,
 * MD time step tau_MD = 1/n_sub (Sec. 3: the time-scale contrast
 * m = tau_LB/tau_MD must be an integer).
 *
 * Memory and ownership.  Every device buffer is allocated by the caller
 * (for instance as a torch tensor) and only borrowed by the library: the
 * workspace of lbmd_workspace_bytes() bytes that lb_create() carves into the
 * two population buffers, the momentum-transfer field and particle scratch,
 * and the particle arrays handed to lbmd_bind_particles().  The library never
 * allocates or frees device memory.  Buffers must stay alive until
 * lb_destroy().  Lattice arrays (populations, densities, velocities,
 * transfer) use the context precision (float for precision 32, double for
 * precision 64); particle positions and velocities are double in both.
 *
 * Streams.  A context is bound to one HIP stream.  Every call is an
 * asynchronous enqueue on it, except lb_moments() with a host totals pointer
 * and the host-side parameter checks.  Calls on one context must not overlap
 * from several host threads.
 *
 * Errors.  Every call returns LBMD_OK or a negative code.  LBMD_EHIP is
 * sticky: after a HIP failure the context refuses further work.
 * lbmd_strerror() gives a message.
 */
#ifndef LBMD_H
#define LBMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbmd lbmd; /* opaque context */

enum {
  LBMD_OK = 0,
  LBMD_EINVAL = -1,     /* bad parameter or argument                          */
  LBMD_ESTATE = -2,     /* call out of order (e.g. lb_step after != n MD steps)*/
  LBMD_EHIP = -3,       /* HIP runtime failure (sticky)                       */
  LBMD_ENOSPACE = -4,   /* workspace smaller than lbmd_workspace_bytes()      */
  LBMD_ENONFINITE = -5  /* a particle coordinate or velocity became NaN/Inf  */
};

/* Layout of the totals returned by lb_moments(). */
enum {
  LBMD_TOT_MASS = 0,     /* sum_r rho(r)                                      */
  LBMD_TOT_PFLUID = 1,   /* [3] sum_r j(r) + sum_r J(r)                       */
  LBMD_TOT_PSEEN = 4,    /* [3] momentum the coupling sees: variant 1 sum j,
                            variants 2 and 3 sum j + sum J                    */
  LBMD_TOT_PPART = 7,    /* [3] sum_p m v_p                                   */
  LBMD_TOT_KEPART = 10,  /* sum_p m |v_p|^2 / 2                               */
  LBMD_TOT_U2FLUID = 11, /* mean over sites of |j/rho|^2 (variant 3: |(j+J)/rho|^2) */
  LBMD_TOT_TLB = 12,     /* LB steps done                                     */
  LBMD_TOT_TMD = 13,     /* MD steps done                                     */
  LBMD_TOT_TPART = 14,   /* particle temperature sum_p m |v_p|^2 / (3 N) with
                            k_B = 1 (the mean kinetic energy of Sec. 3, no
                            centre-of-mass subtraction; 0 when N = 0, NaN
                            once a particle is non-finite)                    */
  LBMD_NTOTALS = 15
};

/*
 * Parameters: the paper's statement of the problem (Sec. 2-3): lattice size,
 * n = tau_LB/tau_MD, viscosity, friction (the paper's zeta, Eq. 4), kT and
 * the coupling variant (1 = variant A, 2 = variant B, 3 = variant C).
 */
typedef struct {
  int32_t nx, ny, nz;     /* sites per axis, periodic, each >= 2               */
  int32_t n_sub;          /* n = tau_LB / tau_MD, integer >= 1 (Sec. 3)        */
  int32_t variant;        /* 1: fluid velocity frozen over the LB interval;
                             2: the sites around each particle see its momentum
                             transfer at the next MD step (Sec. 3);
                             3: each MD step's transfer is applied to the
                             populations of the receiving sites through the
                             forcing part of the collision (Guo, no relaxation,
                             no noise, no streaming), and the LB step then
                             applies only the body force (Sec. 3, variant C)   */
  int32_t precision;      /* 32: float populations stored as deviations from
                             w_i rho0; 64: double (also deviations)            */
  int32_t n_particles;    /* N >= 0                                            */
  int32_t force_model;    /* 0 none; 1 constant force f_ext on every particle;
                             2 harmonic bonds within chains + WCA (all pairs);
                             3 the paper's Kremer-Grest polymer (Sec. 3): FENE
                             bonds + Lennard-Jones cut at 2^(7/6) sigma        */
  int32_t chain_len;      /* beads per chain for force_models 2, 3 (N %
                             chain_len == 0; bead b is bonded to b+1 inside a
                             chain)                                            */
  uint32_t replica;       /* replica id entering the noise counter             */
  uint64_t seed;          /* Philox key                                        */
  double rho0;            /* mean fluid mass density, > 0                      */
  double nu;              /* kinematic shear viscosity, > 0                     */
  double nu_bulk;         /* bulk viscosity; < 0 means "same rate as shear"    */
  double gamma_ghost;     /* relaxation factor of the kinetic modes, |g| < 1   */
  double kT;              /* >= 0; 0 switches all noise off                    */
  double friction;        /* gamma (the paper's zeta), >= 0                    */
  double particle_mass;   /* > 0 when N > 0                                    */
  double body_force[3];   /* uniform force density on the fluid                */
  double f_ext[3];        /* force_model 1                                     */
  double k_bond, r0_bond; /* force_model 2: U = k/2 (r - r0)^2; force_model 3:
                             FENE U = -k R0^2/2 ln(1 - (r/R0)^2), R0 = r0_bond
                             > 0 (a bond at r >= R0 makes its beads
                             non-finite, LBMD_ENONFINITE)                      */
  double wca_eps, wca_sigma; /* Lennard-Jones eps, sigma between all pairs:
                             cut at 2^(1/6) sigma (WCA, model 2) or at
                             2^(7/6) sigma (model 3)                           */
  int32_t stencil;        /* velocity interpolation and force spreading (Eq. 5,
                             Eq. 7, always the same): 0 trilinear over the 8
                             sites of the particle's cube; 1 the three-point
                             kernel of Roma, Peskin and Berger per axis over
                             the 27 nearest sites (the higher-order scheme of
                             Sec. 4).  Equal for all replicas of a batch; the
                             adjoint requires 0                                */
} lbmd_params;

/* Device bytes lb_create() needs for these parameters (0 if invalid). */
size_t lbmd_workspace_bytes(const lbmd_params *p);

/*
 * Create a context.  d_ws: caller-owned device buffer of ws_bytes bytes,
 * 256-byte aligned.  hip_stream: a hipStream_t (NULL = default stream).
 * Initial fluid: at rest, f_i = w_i rho0 (Sec. 2 populations); no momentum
 * transfer pending; step counters zero.  Returns LBMD_EINVAL for invalid
 * parameters, LBMD_ENOSPACE for a short workspace.
 */
int lb_create(const lbmd_params *p, void *d_ws, size_t ws_bytes, void *hip_stream,
              lbmd **out);

/* Destroy the context (host memory only; caller buffers are untouched). */
int lb_destroy(lbmd *c);

/*
 * Bind the caller's particle arrays (device, SoA [3][N]: x, then y, then z
 * rows).  d_x: double positions in [0, L) per axis; d_v: double velocities;
 * d_img: int32 periodic image counters (unwrapped position = x + L * img).  The library
 * updates them in place at every md_couple_substep().  Computes the
 * conservative forces at the bound positions.  Binding in the middle of an
 * LB interval keeps the pending momentum transfer: before it switches to the
 * new arrays the library reads the previously bound ones (positions) to
 * store the transfer that particles keep to themselves into the transfer
 * field, so those arrays must still hold the particles' state during the
 * call.
 */
int lbmd_bind_particles(lbmd *c, void *d_x, void *d_v, int32_t *d_img);

/*
 * Reorder the bound particles along a space-filling curve (Morton order of
 * the 4 x 4 x 4-site tiles their positions fall in, within each replica;
 * stable and deterministic).  The method is unchanged: particles are
 * independent apart from the fluid, so only their storage order moves,
 * which lets the particle kernels of Sec. 3 (interpolation, spreading)
 * share cache lines between neighbours.  x, v and img are permuted in place
 * in the caller's buffers; d_perm (nullable, device int32[Ntot]) receives
 * the permutation: new index t holds the particle that had index d_perm[t].
 * Each particle keeps its identity (its index at binding), which the
 * particle noise counter follows, so a reordered run is the same run up to
 * the rounding order of the transfer sums.  Only at an
 * LB-step boundary (LBMD_ESTATE otherwise, or while an adjoint segment is
 * recorded), for force models 0 and 1 (bonded chains follow the index
 * order: LBMD_EINVAL).  LBMD_ENOSPACE if the sort's scratch is too small.
 */
int lbmd_sort_particles(lbmd *c, int32_t *d_perm);

/*
 * One MD step of the coupled system (Sec. 3, Eq. 4-8): for every particle,
 * from start-of-step values, interpolate the fluid velocity at its position
 * over the 8 sites of its cube (Eq. 5), form F = -gamma (v - u) + F_rand
 * (Eq. 4), dP = tau_MD F (Eq. 6), transfer -delta_k dP to the 8 sites
 * (Eq. 7-8) and advance the particle by velocity Verlet.  In variant 2 the
 * transfer is seen by the velocity interpolation of the next MD step; in
 * variant 1 only by the next lb_step(); in variant 3 it changes the
 * state of the receiving sites before the next MD step (momentum + dJ,
 * stress modes + (1+gamma)/2 times the image of u dJ + dJ u with
 * u = (j + dJ/2)/rho).  Summed over an interval these increments depend
 * only on the interval-start momentum j0, the density and the total
 * transfer J (stress: the image of (j0 J + J j0 + J J)/rho), so the library
 * accumulates J as in variant 2 and adds the increments where the state is
 * read (lb_step(), population copies, moments).  At most n_sub calls per LB
 * interval (LBMD_ESTATE otherwise).
 */
int md_couple_substep(lbmd *c);

/*
 * One LB step (Eq. 3): MRT collision with the force density J/tau_LB of the
 * accumulated momentum transfer (Guo forcing) plus body_force, thermal noise
 * on the 15 non-conserved modes, then streaming.  Variant 3: the interval's
 * site increments join the populations first and the force density is
 * body_force alone.  Requires exactly n_sub
 * md_couple_substep() calls since the previous lb_step() when N > 0
 * (LBMD_ESTATE otherwise).
 */
int lb_step(lbmd *c);

/*
 * Moments of the current (post-stream) state (Eq. 1-2).  d_rho: nullable
 * device [nsites] density; d_u: nullable device [3][nsites] velocity j/rho
 * (variant 3: (j + J)/rho, the momentum of the state after the MD steps);
 * both in the context precision.  h_totals: nullable host double[LBMD_NTOTALS]
 * (FP64 reductions, see the LBMD_TOT_* layout); when given, the call
 * synchronizes the stream and returns LBMD_ENONFINITE if any particle became
 * non-finite since creation.
 */
int lb_moments(lbmd *c, void *d_rho, void *d_u, double *h_totals);

/*
 * lb_moments without workspace scratch, for callers that cannot allocate
 * device memory or enlarge a workspace (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  Same arguments, results
 * and errors as lb_moments() for a single system (a batch context: LBMD_EINVAL);
 * the totals may differ from lb_moments() in the last bits (FP64 sums in
 * another order).  Its reduction rows live in a fixed array of this library,
 * one per GPU (131,200 bytes, held until the process ends, located at
 * lb_create() on the then current device): the call allocates nothing.  The
 * grid is capped at the array's 1024 rows, so every lattice fits
 * (LBMD_ENOSPACE is kept for a larger need, which cannot arise).  All calls
 * on one GPU share the array: calls that overlap on one GPU (several
 * streams or host threads) race and must be serialised by the caller.
 */
int lb_moments_noalloc(lbmd *c, void *d_rho, void *d_u, double *h_totals);

/*
 * Populations of the current post-stream state as deviations
 * df_i(r) = f_i(r) - w_i rho0, device [19][nsites] in the context precision,
 * site index r = x + nx*(y + ny*z), velocity order: 0, +x, -x, +y, -y, +z,
 * -z, (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1),
 * (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).  Get copies out, set
 * replaces the state (variants 1, 2: pending momentum transfer is kept).
 * Variant 3: get includes the increments the MD steps of the current LB
 * interval applied (the populations of the paper's variant C), and set
 * replaces them too (the replica's J is cleared).
 */
int lbmd_get_populations(lbmd *c, void *d_dst);
int lbmd_set_populations(lbmd *c, const void *d_src);

/* Pending momentum transfer J (sum of Eq. 8 over this LB interval), device
 * [3][nsites] in the context precision. */
int lbmd_get_transfer(lbmd *c, void *d_dst);

/* Step counters: LB steps, MD steps, MD steps since the last LB step.
 * Set: the noise streams and the step clock of captured cycles follow the
 * new counts; the particles' transfers kept to themselves go to J first, the
 * corner cache is rebuilt at the next MD step, and with position-dependent
 * forces (models 2, 3) the bound particles are binned into their force
 * cells again and F_cons is recomputed at the current positions (the cells
 * are kept by MD-step parity).  EINVAL for t_lb < 0, subs outside
 * [0, n_sub] or t_md < subs. */
int lbmd_get_counters(lbmd *c, int64_t *t_lb, int64_t *t_md, int32_t *subs);
int lbmd_set_counters(lbmd *c, int64_t t_lb, int64_t t_md, int32_t subs);

/*
 * Bandwidth calibration (not part of the method): copy `bytes` bytes from
 * d_src to d_dst (device, 16-byte aligned, bytes a multiple of 16) with
 * 16-byte non-temporal loads and stores on a persistent grid, asynchronously
 * on hip_stream.  This is the read+write streaming ceiling that the
 * collide-stream kernel's roofline is compared with, and the known-size
 * dispatch that HBM byte counters are calibrated against.  LBMD_EINVAL for
 * misaligned or null arguments.
 */
int lbmd_stream_copy(void *d_dst, const void *d_src, size_t bytes, void *hip_stream);

/* Message for a status code. */
const char *lbmd_strerror(int code);

/*
 * Captured cycles.  Runs ncycles coupled cycles (n_sub md_couple_substep()
 * steps and one lb_step() each, the schedule of Sec. 3 / Fig. 2) by replaying
 * one HIP graph of the cycle on the context's stream; identical in effect to
 * the step-by-step calls.  The graph is captured on first use and again after
 * lbmd_bind_particles() or lbmd_autotune().  Must start at an LB-step
 * boundary (LBMD_ESTATE otherwise).  Asynchronous.
 */
int lbmd_run_cycles(lbmd *c, int32_t ncycles);

/*
 * Batched replicas: n_rep independent periodic systems, each described by its
 * own lbmd_params (box size, particle count, friction, kT, seed, replica id
 * ...), advanced in lockstep by the same calls as a single system, every
 * kernel covering all replicas in one launch.  They must share n_sub,
 * precision and variant (LBMD_EINVAL otherwise).  A replica draws the noise
 * of a single system created with the same seed and replica id, so its
 * trajectory is that system's trajectory.  Lattices are stored one after
 * the other; particle arrays bound with lbmd_bind_particles() are the
 * replicas' [3][N_r] arrays concatenated along the particle axis (row x of
 * all replicas, then y, then z; replica order, N = sum of N_r).
 */
size_t lbmd_batch_workspace_bytes(const lbmd_params *per_rep, int32_t n_rep);
int lb_create_batch(const lbmd_params *per_rep, int32_t n_rep, void *d_ws, size_t ws_bytes,
                    void *hip_stream, lbmd **out);
int lbmd_replica_count(lbmd *c);
/* totals of every replica, host double[n_rep][LBMD_NTOTALS]; synchronizes */
int lbmd_batch_moments(lbmd *c, double *h_totals);
/* per-replica versions of the population / transfer copies (replica rep) */
int lbmd_batch_get_populations(lbmd *c, int32_t rep, void *d_dst);
int lbmd_batch_set_populations(lbmd *c, int32_t rep, const void *d_src);
int lbmd_batch_get_transfer(lbmd *c, int32_t rep, void *d_dst);

/*
 * Launch-shape autotuner (form ii): times, on this context, candidate
 * launch shapes of each hot kernel on the kernel itself and keeps the
 * fastest: the persistent grid of the collide-stream kernel ({one block per
 * 256 sites, 4, 8, 16, 32 blocks per CU}), the grid of the particle
 * kernels (timed on the corner refill) and the lanes per particle of the
 * coupling kernel ({2, 4, 8} trilinear, {8, 16} three-point stencil; timed
 * on whole MD steps, coupling plus after-step work; force models 0 and 1,
 * whose particle state is saved and restored around the timing).  The block
 * size is fixed at 256 threads (the kernels' segments and LDS layouts
 * assume it).  The picks are cached in a JSON file at cache_path (nullable:
 * no cache), keyed by device architecture, precision, variant, replica count
 * and size class.  Must run at an LB-step boundary (LBMD_ESTATE otherwise);
 * the simulation state is left unchanged (the next MD step refills the
 * corner cache).  Synchronizes.  Outputs (nullable): the chosen block
 * counts (0 = one block per work item) and lanes (0 = the built-in default).
 */
int lbmd_autotune(lbmd *c, const char *cache_path, int32_t *lb_blocks, int32_t *part_blocks,
                  int32_t *couple_lanes);

/*
 * Set the launch shapes the autotuner would pick (the same meanings: block
 * counts >= 0, 0 = one block per work item; couple_lanes 0 = default, else
 * one of the candidates above, LBMD_EINVAL otherwise).  At an LB-step
 * boundary only (LBMD_ESTATE).  Results do not depend on the shapes beyond
 * the order of the transfer sums.
 */
int lbmd_set_launch_shape(lbmd *c, int32_t lb_blocks, int32_t part_blocks, int32_t couple_lanes);

/*
 * Saved states (checkpoint / resume).  A state holds the step counters, the
 * populations, and the particle positions, velocities and image counters:
 * with the counter-based noise this fixes the future trajectory exactly.
 * d_dst / d_src: caller-owned device buffers of lbmd_state_bytes() bytes,
 * opaque layout.  Save only at an LB-step boundary (LBMD_ESTATE otherwise;
 * the transfer field is empty there); asynchronous.  Load restores the
 * state into the context and the bound particle arrays; synchronizes once
 * to read the counters.
 */
size_t lbmd_state_bytes(lbmd *c);
int lbmd_save_state(lbmd *c, void *d_dst);
int lbmd_load_state(lbmd *c, const void *d_src);

/*
 * Reverse mode (adjoint) of the coupled cycles, for a single system with
 * force_model 0 or 1 (LBMD_EINVAL otherwise).  The method of Sec. 2-3
 * (Eq. 3-8) is differentiated exactly along one noise realisation: the
 * gradients are those of the deterministic map from (gamma, nu, f_ext,
 * initial particle state) to the particle state after T cycles, with the
 * noise variates held fixed (regenerated from their counters, never
 * stored).
 *
 * Protocol: save states every K cycles on the way forward; then
 *   lbmd_adjoint_attach(c, ws, bytes, K)      adjoint workspace for segments of <= K cycles
 *   lbmd_adjoint_seed(c, xbar, vbar)          dL/dx(T), dL/dv(T) (device [3][N] double, nullable = 0)
 *   for each segment, last first:
 *     lbmd_adjoint_record(c, state, k)        re-run the k cycles from the saved state, recording
 *     k times: lb_step_adjoint(c), then n_sub times md_couple_substep_adjoint(c)
 *   lbmd_adjoint_result(c, xbar0, vbar0, grads)
 * Calls out of this order return LBMD_ESTATE.  The saved state passed to
 * lbmd_adjoint_record() is read again by the reverse steps of its segment
 * and must stay unchanged until they are done.  Recording advances the
 * context like the same number of forward cycles (its state afterwards is
 * the state after the segment).
 *
 * lbmd_adjoint_workspace_bytes: bytes of the adjoint workspace for segments
 * of seg_cycles cycles (0 if unsupported); about (seg_cycles + 1) population
 * sets plus per-MD-step particle records.  d_ws must be 256-byte aligned.
 *
 * lbmd_adjoint_result: dL/dx and dL/dv at the start of the swept cycles
 * (device [3][N] double, nullable) and, in h_grads (host double[5],
 * nullable, synchronizes): dL/dgamma (friction, Eq. 4), dL/dnu (shear
 * viscosity; with nu_bulk < 0 the bulk rate follows it), dL/df_ext[3]
 * (constant force on every particle).
 */
size_t lbmd_adjoint_workspace_bytes(lbmd *c, int32_t seg_cycles);
int lbmd_adjoint_attach(lbmd *c, void *d_ws, size_t bytes, int32_t seg_cycles);
int lbmd_adjoint_seed(lbmd *c, const double *d_xbar, const double *d_vbar);
int lbmd_adjoint_record(lbmd *c, const void *d_state, int32_t ncycles);
/* reverse of one lb_step() of the recorded segment (last first) */
int lb_step_adjoint(lbmd *c);
/* reverse of one md_couple_substep() (last first within the cycle) */
int md_couple_substep_adjoint(lbmd *c);
int lbmd_adjoint_result(lbmd *c, double *d_xbar, double *d_vbar, double *h_grads);

#ifdef __cplusplus
}
#endif

#endif /* LBMD_H */
