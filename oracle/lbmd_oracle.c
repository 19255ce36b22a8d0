/*
 * lbmd_oracle.c -- plain, slow FP64 CPU reference of the fluctuating D3Q19
 * lattice-Boltzmann fluid with dissipative (Ahlrichs-Duenweg) point-particle
 * coupling, in the coupling variants of Tretyakov & Duenweg,
 * arXiv:1610.02733 (variant A = 1, variant B = 2, variant C = 3).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * table or header with the HIP implementation; the two meet only through the
 * seeded inputs the tests hand to both.
 *
 * Everything here is written for a reader to check against the paper by eye:
 * full populations f_i (not deviations), explicit 19x19 mode matrix, plain
 * loops, no blocking, no fusion.  Units are lattice units: a = 1, tau_LB = 1,
 * tau_MD = 1/n with the integer time-scale contrast n (Sec. 3, Fig. 2).
 *
 * Readings of points the paper leaves to its references (MRT basis, rates,
 * equilibrium, Guo forcing, noise amplitudes and distribution, Philox
 * counter layout, wrap rule) are stated at the function that uses them.
 *
 * Parity pins: every function below is pinned by a CPU test (conservation
 * laws, closed forms, textbook special cases, known-answer vectors,
 * statistics); none is "parity unpinned".
 *
 * Threads (OpenMP, for timing the CPU baseline only): the loops over sites
 * (collision, streaming) and over particles (interpolation, friction, kicks)
 * run in parallel; every result element is computed by the same arithmetic
 * in the same order whatever the thread count, and the spreading onto the
 * lattice stays serial in particle order, so results are bitwise independent
 * of the number of threads (pinned by a test).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* ------------------------------------------------------------------------- */
/* D3Q19 velocity set (Sec. 2, Fig. 1a: 19 velocities including c_0 = 0),    */
/* listed with opposite velocities adjacent.                                  */
/* ------------------------------------------------------------------------- */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double Wt[Q];      /* lattice weights                                   */
static double Emat[Q][Q]; /* Emat[k][i] = e_k(c_i), the MRT mode polynomials   */
static double Bn[Q];      /* mode norms b_k = sum_i w_i e_k(c_i)^2             */
static int tables_ready = 0;

/* Mode polynomials of the weighted-orthogonal D3Q19 basis used by the
 * MRT collision the paper refers to (Sec. 2): mass, momentum, six stress
 * modes, nine kinetic ("ghost") modes. */
static double mode_poly(int k, double cx, double cy, double cz) {
  double c2 = cx * cx + cy * cy + cz * cz;
  switch (k) {
    case 0: return 1.0;
    case 1: return cx;
    case 2: return cy;
    case 3: return cz;
    case 4: return c2 - 1.0;
    case 5: return 3.0 * cx * cx - c2;
    case 6: return cy * cy - cz * cz;
    case 7: return cx * cy;
    case 8: return cy * cz;
    case 9: return cx * cz;
    case 10: return (3.0 * c2 - 5.0) * cx;
    case 11: return (3.0 * c2 - 5.0) * cy;
    case 12: return (3.0 * c2 - 5.0) * cz;
    case 13: return (cy * cy - cz * cz) * cx;
    case 14: return (cz * cz - cx * cx) * cy;
    case 15: return (cx * cx - cy * cy) * cz;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * cx * cx - c2);
    case 18: return (2.0 * c2 - 3.0) * (cy * cy - cz * cz);
  }
  return 0.0;
}

static void tables_init(void) {
  if (tables_ready) return;
  for (int i = 0; i < Q; ++i) {
    int c2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
    Wt[i] = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  for (int k = 0; k < Q; ++k) {
    Bn[k] = 0.0;
    for (int i = 0; i < Q; ++i) {
      Emat[k][i] = mode_poly(k, CV[i][0], CV[i][1], CV[i][2]);
      Bn[k] += Wt[i] * Emat[k][i] * Emat[k][i];
    }
  }
  tables_ready = 1;
}

void orc_tables(int32_t *c_out, double *w_out, double *e_out, double *b_out) {
  tables_init();
  for (int i = 0; i < Q; ++i) {
    for (int d = 0; d < 3; ++d) c_out[3 * i + d] = CV[i][d];
    w_out[i] = Wt[i];
  }
  for (int k = 0; k < Q; ++k) {
    b_out[k] = Bn[k];
    for (int i = 0; i < Q; ++i) e_out[Q * k + i] = Emat[k][i];
  }
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), from its published      */
/* definition: 10 rounds of two 32x32->64 multiplications; the key is bumped  */
/* by the Weyl constants between rounds.                                     */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter layout of the noise stream (the paper only requires noise that
 * balances each dissipation, Sec. 1 and Sec. 3; the generator is ours):
 *   counter = (index, step mod 2^32, purpose<<28 | replica<<8 | call, step>>32)
 *   key     = (seed mod 2^32, seed >> 32)
 * purpose 1 = fluid (index = site, step = LB step), 2 = particle
 * (index = particle, step = MD step). */
#define PURPOSE_FLUID 1u
#define PURPOSE_PARTICLE 2u

static void noise_words(uint64_t seed, uint32_t purpose, uint32_t replica,
                        uint32_t call, uint64_t index, uint64_t step,
                        uint32_t out[4]) {
  uint32_t ctr[4], key[2];
  ctr[0] = (uint32_t)index;
  ctr[1] = (uint32_t)(step & 0xFFFFFFFFu);
  ctr[2] = (purpose << 28) | ((replica & 0xFFFFFu) << 8) | (call & 0xFFu);
  ctr[3] = (uint32_t)(step >> 32);
  key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
  key[1] = (uint32_t)(seed >> 32);
  orc_philox4x32_10(ctr, key, out);
}

/* Zero-mean, unit-variance uniform variate from an integer of `bits` bits:
 * u = (h + 1/2) / 2^bits in (0,1), r = sqrt(12) (u - 1/2).  Only second
 * moments enter the fluctuation-dissipation balance, so a uniform variate
 * serves as well as a Gaussian one. */
static double unit_variate(uint32_t h, int bits) {
  double u = ((double)h + 0.5) / ldexp(1.0, bits);
  return sqrt(12.0) * (u - 0.5);
}

/* The 15 fluid variates of one site and LB step, for modes k = 4..18:
 * two Philox calls give eight 32-bit words; variate v uses 16-bit half
 * (v mod 2) of word v/2, low half first. */
void orc_fluid_variates(uint64_t seed, uint32_t replica, uint64_t site,
                        uint64_t step, double r_out[15]) {
  uint32_t words[8];
  noise_words(seed, PURPOSE_FLUID, replica, 0, site, step, words);
  noise_words(seed, PURPOSE_FLUID, replica, 1, site, step, words + 4);
  for (int v = 0; v < 15; ++v) {
    uint32_t w = words[v / 2];
    uint32_t h = (v % 2 == 0) ? (w & 0xFFFFu) : (w >> 16);
    r_out[v] = unit_variate(h, 16);
  }
}

/* The 3 particle variates of one particle and MD step: one Philox call,
 * words 0..2, top 24 bits of each. */
void orc_particle_variates(uint64_t seed, uint32_t replica, uint64_t particle,
                           uint64_t step, double r_out[3]) {
  uint32_t words[4];
  noise_words(seed, PURPOSE_PARTICLE, replica, 0, particle, step, words);
  for (int d = 0; d < 3; ++d) r_out[d] = unit_variate(words[d] >> 8, 24);
}

/* ------------------------------------------------------------------------- */
/* Parameters (the paper's statement of the problem: lattice, n, viscosity,   */
/* friction zeta (called gamma here), kT, coupling variant).                  */
/* ------------------------------------------------------------------------- */
typedef struct {
  int32_t nx, ny, nz;
  int32_t n_sub;       /* n = tau_LB / tau_MD, integer >= 1 (Sec. 3)      */
  int32_t variant;     /* 1 = variant A, 2 = variant B, 3 = variant C       */
  int32_t n_particles;
  int32_t force_model; /* 0 none, 1 constant f_ext, 2 harmonic bonds + WCA,
                          3 Kremer-Grest: FENE bonds + LJ cut at 2^(7/6) sigma */
  int32_t chain_len;   /* beads per chain for force model 2                 */
  uint32_t replica;    /* enters the noise counter                          */
  int32_t stencil;     /* interpolation / spreading stencil (Eq. 5, 7):
                          0 trilinear over the 8 cube sites, 1 the 3-point
                          kernel per axis over 27 sites                     */
  uint64_t seed;
  double rho0, nu, nu_bulk, gamma_ghost, kT, friction, particle_mass;
  double body_force[3], f_ext[3];
  double k_bond, r0_bond, wca_eps, wca_sigma;
} orc_params;

typedef struct {
  orc_params p;
  int64_t nsites;
  double *f;    /* [Q][nsites] post-stream populations (the physical state)  */
  double *J;    /* [3][nsites] momentum transferred by the particles since
                   the last LB step (Eq. 8 summed over the MD steps);
                   variants A and B only                                     */
  double *dJ;   /* [3][nsites] transfer of the current MD step (variant C)   */
  double *post; /* [Q][nsites] scratch: post-collision populations          */
  double *x, *v, *fcons; /* [3][N]                                          */
  int32_t *img;          /* [3][N] periodic image counters                   */
  int64_t t_lb, t_md;
  int32_t subs_since_lb;
  int32_t nonfinite;
  double gamma_s, gamma_b, gamma_g, mu;
} orc_ctx;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ESTATE = -2, ORC_ENONFINITE = -5 };

static int64_t site_index(const orc_ctx *c, int64_t x, int64_t y, int64_t z) {
  return x + (int64_t)c->p.nx * (y + (int64_t)c->p.ny * z);
}

static int64_t wrap_coord(int64_t a, int64_t n) {
  a %= n;
  return a < 0 ? a + n : a;
}

/* Relaxation parameters (Sec. 2: the stress-relaxation rates set the
 * viscosities).  In lattice units with c_s^2 = 1/3:
 *   shear  nu   = (1 + g_s) / (6 (1 - g_s))      -> g_s = (6 nu - 1)/(6 nu + 1)
 *   bulk   nu_b = (1 + g_b) / (9 (1 - g_b))      -> g_b = (9 nu_b - 1)/(9 nu_b + 1)
 * (so that equal rates give BGK, whose bulk viscosity is 2/3 of the shear
 * viscosity).
 * nu_bulk < 0 selects g_b = g_s; kinetic modes relax with gamma_ghost.
 * Fluctuation amplitude mu = kT / (c_s^2 a^3) = 3 kT. */
static void derive_rates(orc_ctx *c) {
  const orc_params *p = &c->p;
  c->gamma_s = (6.0 * p->nu - 1.0) / (6.0 * p->nu + 1.0);
  c->gamma_b = (p->nu_bulk < 0.0)
                   ? c->gamma_s
                   : (9.0 * p->nu_bulk - 1.0) / (9.0 * p->nu_bulk + 1.0);
  c->gamma_g = p->gamma_ghost;
  c->mu = 3.0 * p->kT;
}

static double mode_rate(const orc_ctx *c, int k) {
  if (k == 4) return c->gamma_b;
  if (k >= 5 && k <= 9) return c->gamma_s;
  return c->gamma_g; /* k = 10..18 */
}

int orc_create(const orc_params *p, orc_ctx **out) {
  tables_init();
  *out = NULL;
  if (p->nx < 2 || p->ny < 2 || p->nz < 2) return ORC_EINVAL;
  if (p->n_sub < 1 || p->variant < 1 || p->variant > 3) return ORC_EINVAL;
  if (!(p->nu > 0.0) || !(p->kT >= 0.0) || !(p->friction >= 0.0)) return ORC_EINVAL;
  if (!(p->rho0 > 0.0) || p->n_particles < 0) return ORC_EINVAL;
  if (p->n_particles > 0 && !(p->particle_mass > 0.0)) return ORC_EINVAL;
  if (p->force_model < 0 || p->force_model > 3) return ORC_EINVAL;
  if (p->stencil < 0 || p->stencil > 1) return ORC_EINVAL;
  if (p->force_model >= 2 && (p->chain_len < 1 || p->n_particles % p->chain_len))
    return ORC_EINVAL;
  if (p->force_model == 3 && !(p->r0_bond > 0.0)) return ORC_EINVAL;
  orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
  c->p = *p;
  c->nsites = (int64_t)p->nx * p->ny * p->nz;
  c->f = (double *)malloc(sizeof(double) * Q * c->nsites);
  c->J = (double *)calloc(3 * c->nsites, sizeof(double));
  c->dJ = (double *)calloc(3 * c->nsites, sizeof(double));
  c->post = (double *)malloc(sizeof(double) * Q * c->nsites);
  int64_t n = p->n_particles > 0 ? p->n_particles : 1;
  c->x = (double *)calloc(3 * n, sizeof(double));
  c->v = (double *)calloc(3 * n, sizeof(double));
  c->fcons = (double *)calloc(3 * n, sizeof(double));
  c->img = (int32_t *)calloc(3 * n, sizeof(int32_t));
  derive_rates(c);
  /* fluid at rest with mean density rho0: f_i = w_i rho0 */
  for (int i = 0; i < Q; ++i)
    for (int64_t r = 0; r < c->nsites; ++r) c->f[i * c->nsites + r] = Wt[i] * p->rho0;
  *out = c;
  return ORC_OK;
}

void orc_destroy(orc_ctx *c) {
  if (!c) return;
  free(c->f); free(c->J); free(c->dJ); free(c->post);
  free(c->x); free(c->v); free(c->fcons); free(c->img);
  free(c);
}

/* ------------------------------------------------------------------------- */
/* Conservative forces F_cons (Eq. 4; they do not act on the fluid).          */
/* ------------------------------------------------------------------------- */
static double min_image(double d, double L) { return d - L * nearbyint(d / L); }

static void conservative_forces(orc_ctx *c) {
  const orc_params *p = &c->p;
  int64_t N = p->n_particles;
  double *F = c->fcons;
  for (int64_t q = 0; q < 3 * N; ++q) F[q] = 0.0;
  if (p->force_model == 1) {
    for (int64_t a = 0; a < N; ++a)
      for (int d = 0; d < 3; ++d) F[d * N + a] = p->f_ext[d];
  } else if (p->force_model >= 2) {
    double L[3] = {p->nx, p->ny, p->nz};
    /* bonds between consecutive beads of a chain.  Model 2: harmonic
       U = k/2 (r - r0)^2.  Model 3 (Kremer-Grest, Sec. 3): FENE
       U = -k R0^2/2 ln(1 - (r/R0)^2) with R0 = r0_bond, undefined (NaN
       force) for r >= R0 */
    for (int64_t a = 0; a + 1 < N; ++a) {
      if ((a + 1) % p->chain_len == 0) continue;
      int64_t b = a + 1;
      double d[3], r2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        d[k] = min_image(c->x[k * N + a] - c->x[k * N + b], L[k]);
        r2 += d[k] * d[k];
      }
      double fmag; /* force on a along d, per unit of d */
      if (p->force_model == 2) {
        double r = sqrt(r2);
        fmag = -p->k_bond * (r - p->r0_bond) / r;
      } else {
        double x2 = r2 / (p->r0_bond * p->r0_bond);
        fmag = x2 < 1.0 ? -p->k_bond / (1.0 - x2) : NAN;
      }
      for (int k = 0; k < 3; ++k) {
        F[k * N + a] += fmag * d[k];
        F[k * N + b] -= fmag * d[k];
      }
    }
    /* Lennard-Jones 4 eps[(s/r)^12 - (s/r)^6] between all pairs (bonded
       ones included), cut at r_c: model 2 WCA, r_c = 2^(1/6) s (shifted by
       + eps); model 3 the paper's cut-off r_c = 2^(7/6) s.  The energy
       shift at r_c does not enter the force. */
    double rc2 = (p->force_model == 2 ? pow(2.0, 1.0 / 3.0) : pow(2.0, 7.0 / 3.0)) *
                 p->wca_sigma * p->wca_sigma;
    for (int64_t a = 0; a < N; ++a)
      for (int64_t b = a + 1; b < N; ++b) {
        double d[3], r2 = 0.0;
        for (int k = 0; k < 3; ++k) {
          d[k] = min_image(c->x[k * N + a] - c->x[k * N + b], L[k]);
          r2 += d[k] * d[k];
        }
        /* beyond the cut-off, or a bead that is no longer finite: no pair
           force (a diverged bead leaves the pair sums of the others) */
        if (!(r2 < rc2)) continue;
        double sr2 = p->wca_sigma * p->wca_sigma / r2;
        double sr6 = sr2 * sr2 * sr2;
        double fmag = 24.0 * p->wca_eps * (2.0 * sr6 * sr6 - sr6) / r2;
        for (int k = 0; k < 3; ++k) {
          F[k * N + a] += fmag * d[k];
          F[k * N + b] -= fmag * d[k];
        }
      }
  }
}

int orc_set_particles(orc_ctx *c, const double *x, const double *v,
                      const int32_t *img) {
  int64_t N = c->p.n_particles;
  memcpy(c->x, x, sizeof(double) * 3 * N);
  memcpy(c->v, v, sizeof(double) * 3 * N);
  if (img)
    memcpy(c->img, img, sizeof(int32_t) * 3 * N);
  else
    memset(c->img, 0, sizeof(int32_t) * 3 * N);
  conservative_forces(c);
  return ORC_OK;
}

int orc_get_particles(const orc_ctx *c, double *x, double *v, int32_t *img) {
  int64_t N = c->p.n_particles;
  if (x) memcpy(x, c->x, sizeof(double) * 3 * N);
  if (v) memcpy(v, c->v, sizeof(double) * 3 * N);
  if (img) memcpy(img, c->img, sizeof(int32_t) * 3 * N);
  return ORC_OK;
}

/* populations of the post-stream state, [Q][nsites], full values f_i */
int orc_set_populations(orc_ctx *c, const double *f) {
  memcpy(c->f, f, sizeof(double) * Q * c->nsites);
  return ORC_OK;
}
int orc_get_populations(const orc_ctx *c, double *f) {
  memcpy(f, c->f, sizeof(double) * Q * c->nsites);
  return ORC_OK;
}
int orc_get_J(const orc_ctx *c, double *J) {
  memcpy(J, c->J, sizeof(double) * 3 * c->nsites);
  return ORC_OK;
}
int orc_set_J(orc_ctx *c, const double *J) {
  memcpy(c->J, J, sizeof(double) * 3 * c->nsites);
  return ORC_OK;
}
void orc_counters(const orc_ctx *c, int64_t *t_lb, int64_t *t_md, int32_t *subs,
                  int32_t *nonfinite) {
  *t_lb = c->t_lb; *t_md = c->t_md; *subs = c->subs_since_lb;
  *nonfinite = c->nonfinite;
}
void orc_set_counters(orc_ctx *c, int64_t t_lb, int64_t t_md, int32_t subs) {
  c->t_lb = t_lb; c->t_md = t_md; c->subs_since_lb = subs;
}

/* ------------------------------------------------------------------------- */
/* Collision at one site (Eq. 3, Sec. 2 and Sec. 3).                          */
/* f: the 19 post-stream populations at the site; J: momentum transferred by  */
/* the particles over the last n MD steps (so the force density acting over  */
/* the LB step is F = J / tau_LB, Eq. 7-8); g: uniform body-force density.    */
/* Writes the 19 post-collision populations.                                 */
/*                                                                           */
/*  rho = sum f_i,  j = sum c_i f_i                          (Eq. 1-2)       */
/*  u   = (j + F/2) / rho                 (Guo's half-force velocity)        */
/*  m_k = sum_i e_k(c_i) f_i                                 (MRT modes)     */
/*  f^eq_i = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2)     (2nd order)     */
/*  G_i = w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F              (Guo source)    */
/*  m*_0 = rho, m*_{1,2,3} = j + F                                          */
/*  m*_k = m^eq_k + g_k (m_k - m^eq_k) + (1 + g_k)/2 G_k + phi_k r_k,        */
/*         k = 4..18, phi_k = sqrt(mu rho b_k (1 - g_k^2))                   */
/*  f*_i = w_i sum_k e_k(c_i) m*_k / b_k                                    */
/* With all g_k equal this is BGK relaxation with Guo forcing.  rho in phi_k */
/* is the site's own density.                                               */
/* ------------------------------------------------------------------------- */
static void collide_site(const orc_ctx *c, int64_t site, int64_t step,
                         const double f[Q], const double J[3], double out[Q]) {
  const orc_params *p = &c->p;
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    for (int d = 0; d < 3; ++d) j[d] += CV[i][d] * f[i];
  }
  double F[3], u[3];
  for (int d = 0; d < 3; ++d) {
    F[d] = J[d] + p->body_force[d];
    u[d] = (j[d] + 0.5 * F[d]) / rho;
  }
  double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double feq[Q], G[Q];
  for (int i = 0; i < Q; ++i) {
    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    feq[i] = Wt[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * u2);
    double g = 0.0;
    for (int d = 0; d < 3; ++d) g += (3.0 * (CV[i][d] - u[d]) + 9.0 * cu * CV[i][d]) * F[d];
    G[i] = Wt[i] * g;
  }
  double m[Q], meq[Q], gk[Q], mstar[Q];
  for (int k = 0; k < Q; ++k) {
    m[k] = meq[k] = gk[k] = 0.0;
    for (int i = 0; i < Q; ++i) {
      m[k] += Emat[k][i] * f[i];
      meq[k] += Emat[k][i] * feq[i];
      gk[k] += Emat[k][i] * G[i];
    }
  }
  double r[15];
  if (p->kT > 0.0) orc_fluid_variates(p->seed, p->replica, (uint64_t)site, (uint64_t)step, r);
  mstar[0] = rho;
  for (int d = 0; d < 3; ++d) mstar[1 + d] = j[d] + F[d];
  for (int k = 4; k < Q; ++k) {
    double g = mode_rate(c, k);
    mstar[k] = meq[k] + g * (m[k] - meq[k]) + 0.5 * (1.0 + g) * gk[k];
    if (p->kT > 0.0) mstar[k] += sqrt(c->mu * rho * Bn[k] * (1.0 - g * g)) * r[k - 4];
  }
  for (int i = 0; i < Q; ++i) {
    double s = 0.0;
    for (int k = 0; k < Q; ++k) s += Emat[k][i] * mstar[k] / Bn[k];
    out[i] = Wt[i] * s;
  }
}

/* One LB step (Eq. 3): collide at every site with F = J / tau_LB, then
 * stream f*_i(r) to r + c_i (periodic).  J is consumed and reset; the
 * ordering "n MD steps, then collide with the accumulated transfer and
 * stream" is that of Sec. 3 (variant A and B alike). */
int orc_lb_step(orc_ctx *c) {
  if (c->p.n_particles > 0 && c->subs_since_lb != c->p.n_sub) return ORC_ESTATE;
  int64_t S = c->nsites;
  double *post = c->post;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < S; ++r) {
    double fin[Q], fout[Q], Jr[3];
    for (int i = 0; i < Q; ++i) fin[i] = c->f[i * S + r];
    for (int d = 0; d < 3; ++d) Jr[d] = c->J[d * S + r];
    collide_site(c, r, c->t_lb, fin, Jr, fout);
    for (int i = 0; i < Q; ++i) post[i * S + r] = fout[i];
  }
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < c->p.nz; ++z)
    for (int64_t y = 0; y < c->p.ny; ++y)
      for (int64_t x = 0; x < c->p.nx; ++x) {
        int64_t r = site_index(c, x, y, z);
        for (int i = 0; i < Q; ++i) {
          int64_t xd = wrap_coord(x + CV[i][0], c->p.nx);
          int64_t yd = wrap_coord(y + CV[i][1], c->p.ny);
          int64_t zd = wrap_coord(z + CV[i][2], c->p.nz);
          c->f[i * S + site_index(c, xd, yd, zd)] = post[i * S + r];
        }
      }
  memset(c->J, 0, sizeof(double) * 3 * S);
  c->t_lb += 1;
  c->subs_since_lb = 0;
  return ORC_OK;
}

/* The post-stream populations that the next LB step would produce at a
 * list of sites, without changing the state: f_i(r) = f*_i(r - c_i). */
int orc_lb_step_sampled(const orc_ctx *c, int64_t nsample, const int64_t *sites,
                        double *out /* [nsample][Q] */) {
  int64_t S = c->nsites;
  for (int64_t s = 0; s < nsample; ++s) {
    int64_t r = sites[s];
    int64_t x = r % c->p.nx, y = (r / c->p.nx) % c->p.ny, z = r / ((int64_t)c->p.nx * c->p.ny);
    for (int i = 0; i < Q; ++i) {
      int64_t src = site_index(c, wrap_coord(x - CV[i][0], c->p.nx),
                               wrap_coord(y - CV[i][1], c->p.ny),
                               wrap_coord(z - CV[i][2], c->p.nz));
      double fin[Q], fout[Q], Jr[3];
      for (int q = 0; q < Q; ++q) fin[q] = c->f[q * S + src];
      for (int d = 0; d < 3; ++d) Jr[d] = c->J[d * S + src];
      collide_site(c, src, c->t_lb, fin, Jr, fout);
      out[s * Q + i] = fout[i];
    }
  }
  return ORC_OK;
}

/* single-site collision exposed for special-case tests */
int orc_collide_site(const orc_ctx *c, int64_t site, int64_t step, const double *f,
                     const double *J, double *out) {
  collide_site(c, site, step, f, J, out);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Coupling geometry (Eq. 5 and Eq. 7): the eight sites of the cube that      */
/* contains the particle and their weights, from the distances along x, y, z. */
/* Sites sit at integer coordinates; the cube's lower corner is floor(R);    */
/* with s = R - floor(R), corner o in {0,1}^3 has weight                     */
/* prod_d (o_d ? s_d : 1 - s_d)  (trilinear).                               */
/* ------------------------------------------------------------------------- */
void orc_cube_weights(const orc_ctx *c, const double R[3], int64_t sites[8],
                      double w[8]) {
  int64_t base[3];
  double s[3];
  int64_t L[3] = {c->p.nx, c->p.ny, c->p.nz};
  for (int d = 0; d < 3; ++d) {
    double fl = floor(R[d]);
    base[d] = (int64_t)fl;
    s[d] = R[d] - fl;
  }
  for (int k = 0; k < 8; ++k) {
    int o[3] = {k & 1, (k >> 1) & 1, (k >> 2) & 1};
    w[k] = 1.0;
    int64_t q[3];
    for (int d = 0; d < 3; ++d) {
      w[k] *= o[d] ? s[d] : 1.0 - s[d];
      q[d] = wrap_coord(base[d] + o[d], L[d]);
    }
    sites[k] = site_index(c, q[0], q[1], q[2]);
  }
}

/* Three-point kernel per axis (Roma, Peskin and Berger, J. Comput. Phys.
 * 153 (1999) 509), the higher-order alternative the paper mentions for
 * Eq. 5 and Eq. 7 (Sec. 4): for a distance r from a site along one axis
 *   phi(r) = (1 + sqrt(1 - 3 r^2)) / 3                for |r| <= 1/2,
 *   phi(r) = (5 - 3|r| - sqrt(1 - 3 (1 - |r|)^2)) / 6 for 1/2 <= |r| <= 3/2,
 *   phi(r) = 0 otherwise.
 * The particle at R uses the three sites nearest along each axis,
 * j = c - 1, c, c + 1 with c = floor(R + 1/2); the site weight is the
 * product of the three axis weights (27 sites). */
static double phi3(double r) {
  double a = fabs(r);
  if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
  if (a <= 1.5) {
    double b = 1.0 - a;
    double q = 1.0 - 3.0 * b * b;
    return (5.0 - 3.0 * a - sqrt(q > 0.0 ? q : 0.0)) / 6.0;
  }
  return 0.0;
}

void orc_stencil3_weights(const orc_ctx *c, const double R[3], int64_t sites[27],
                          double w[27]) {
  int64_t L[3] = {c->p.nx, c->p.ny, c->p.nz};
  int64_t ctr[3];
  double wa[3][3];
  for (int d = 0; d < 3; ++d) {
    ctr[d] = (int64_t)floor(R[d] + 0.5);
    for (int j = 0; j < 3; ++j) wa[d][j] = phi3(R[d] - (double)(ctr[d] + j - 1));
  }
  for (int k = 0; k < 27; ++k) {
    int o[3] = {k % 3, (k / 3) % 3, k / 9};
    w[k] = wa[0][o[0]] * wa[1][o[1]] * wa[2][o[2]];
    sites[k] = site_index(c, wrap_coord(ctr[0] + o[0] - 1, L[0]),
                          wrap_coord(ctr[1] + o[1] - 1, L[1]),
                          wrap_coord(ctr[2] + o[2] - 1, L[2]));
  }
}

/* The sites and weights of the context's stencil; returns their count. */
static int stencil_weights(const orc_ctx *c, const double R[3], int64_t sites[27],
                           double w[27]) {
  if (c->p.stencil == 1) {
    orc_stencil3_weights(c, R, sites, w);
    return 27;
  }
  orc_cube_weights(c, R, sites, w);
  return 8;
}

/* fluid velocity seen by the coupling at a site: u = j/rho of the
 * post-stream state (variant A), plus the momentum already transferred in
 * this LB interval, (j + J)/rho (variant B: "update the lattice velocities
 * on the surrounding sites"; the populations themselves are not touched).
 * In variant C the transfers are applied to the populations at every MD
 * step, so u = j/rho of the current populations (J stays zero). */
static void site_velocity(const orc_ctx *c, int64_t r, double u[3]) {
  int64_t S = c->nsites;
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    double fi = c->f[i * S + r];
    rho += fi;
    for (int d = 0; d < 3; ++d) j[d] += CV[i][d] * fi;
  }
  for (int d = 0; d < 3; ++d) {
    double jd = j[d] + (c->p.variant == 2 ? c->J[d * S + r] : 0.0);
    u[d] = jd / rho;
  }
}

/* Periodic wrap of a coordinate into [0, L) with image counting, for any
 * displacement: x -= k L with k = floor(x / L).  A value that rounds to
 * exactly L after the shift is moved to 0 in the next image. */
static void wrap_position(double *x, int32_t *img, double L) {
  if (*x >= 0.0 && *x < L) return;
  double k = floor(*x / L);
  if (fabs(k) > 1e9) k = copysign(1e9, k); /* keep the image count in range */
  *x -= k * L;
  *img += (int32_t)k;
  if (*x >= L) {
    *x -= L;
    *img += 1;
  } else if (*x < 0.0) {
    *x += L;
    *img -= 1;
  }
}

/* ------------------------------------------------------------------------- */
/* Variant C (Sec. 3, the refined variant): at every MD step the momentum     */
/* transfer dJ of the step is applied to the populations of each receiving    */
/* site through the forcing part of the collision operator alone -- no        */
/* relaxation, no noise, no streaming.  Reading: the same mode-space forcing  */
/* as in the LB step (Guo), with the site's current velocity                  */
/*   u = (j + dJ/2) / rho,                                                    */
/*   G_i = w_i [3 (c_i - u) + 9 (c_i.u) c_i] . dJ,    g_k = sum_i e_k(c_i) G_i  */
/*   dm_0 = 0,  dm_{1,2,3} = dJ (= g_{1,2,3}),                                */
/*   dm_k = (1 + gamma_k)/2 g_k  (stress modes, k = 4..9),  dm_k = 0 (k >= 10) */
/*   f_i += w_i sum_k e_k(c_i) dm_k / b_k.                                    */
/* Mass and the kinetic modes are unchanged, the momentum changes by exactly  */
/* dJ (momentum is conserved at every MD step, as in variant B), and the     */
/* next MD step reads its velocities from the changed populations.           */
/* ------------------------------------------------------------------------- */
static void forcing_update(const orc_ctx *c, int64_t r, const double dJ[3]) {
  int64_t S = c->nsites;
  double f[Q], rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    f[i] = c->f[i * S + r];
    rho += f[i];
    for (int d = 0; d < 3; ++d) j[d] += CV[i][d] * f[i];
  }
  double u[3];
  for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * dJ[d]) / rho;
  double G[Q];
  for (int i = 0; i < Q; ++i) {
    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    double g = 0.0;
    for (int d = 0; d < 3; ++d) g += (3.0 * (CV[i][d] - u[d]) + 9.0 * cu * CV[i][d]) * dJ[d];
    G[i] = Wt[i] * g;
  }
  double dm[Q];
  for (int k = 0; k < Q; ++k) {
    double gk = 0.0;
    for (int i = 0; i < Q; ++i) gk += Emat[k][i] * G[i];
    if (k == 0 || k >= 10)
      dm[k] = 0.0;
    else if (k <= 3)
      dm[k] = dJ[k - 1];
    else
      dm[k] = 0.5 * (1.0 + mode_rate(c, k)) * gk;
  }
  for (int i = 0; i < Q; ++i) {
    double s = 0.0;
    for (int k = 0; k < Q; ++k) s += Emat[k][i] * dm[k] / Bn[k];
    c->f[i * S + r] = f[i] + Wt[i] * s;
  }
}

/* One MD step of the coupled system (Sec. 3, Eq. 4-8 and the variant-B
 * schedule):
 *  1. for every particle, from start-of-step R, v and a fresh F_rand:
 *       u(R) = sum_k delta_k u(r_k)                                 (Eq. 5)
 *       F_c  = -gamma (v - u(R)) + F_rand                          (Eq. 4)
 *       dP   = tau_MD F_c                                           (Eq. 6)
 *     F_rand has <F_a F_b> = (2 gamma kT / tau_MD) (1 - a/2) delta_ab
 *     per MD step with a = gamma tau_MD (1/m + S/rho0), S = sum_k delta_k^2:
 *     the fluctuation-dissipation balance of the explicit step itself.  The
 *     step damps the relative velocity w of the particle and the fluid at
 *     its stencil (which in variant B takes -dP at once, an effective mass
 *     rho0/S) as w' = (1 - a) w + (1/m + S/rho0) dP_rand; that AR(1) process
 *     has the equilibrium variance kT (1/m + S/rho0) of the pair's relative
 *     velocity exactly when <dP_rand^2> = 2 gamma kT tau_MD (1 - a/2).  The
 *     paper requires noise balancing the friction (Sec. 1, Sec. 3) without
 *     giving the discrete amplitude; this one reproduces its temperature
 *     statements (Sec. 3: variant B within 2% at m = 10, dt = 0.01 tau for
 *     zeta up to 20; variant A heating with zeta, dt and m, equally at equal
 *     LB step), the continuous-time amplitude (a -> 0) does not.  Clamped at
 *     0 for a >= 2, beyond the stability bound of the explicit step.
 *  2. every particle transfers -delta_k dP to J(r_k)          (Eq. 7-8)
 *     -- all particles read the velocities of step 1 first, so within one
 *     MD step no particle sees another's transfer of the same step.  In
 *     variant C the step's transfers are collected per site and applied to
 *     the populations (forcing_update).
 *  3. velocity Verlet with F_c held over the step:
 *       v += tau/(2m) (F_cons(R) + F_c);  R += tau v;  wrap;
 *       F_cons(R_new);  v += tau/(2m) (F_cons(R_new) + F_c).
 * The particle gains exactly dP from the coupling, the fluid exactly -dP. */
int orc_md_couple_substep(orc_ctx *c) {
  const orc_params *p = &c->p;
  if (c->subs_since_lb >= p->n_sub) return ORC_ESTATE;
  int64_t N = p->n_particles, S = c->nsites;
  double tau = 1.0 / p->n_sub;
  double amp = sqrt(2.0 * p->friction * p->kT / tau);
  double *Fc = (double *)calloc(3 * (N > 0 ? N : 1), sizeof(double));
  int64_t (*sites)[27] = malloc(sizeof(int64_t[27]) * (N > 0 ? N : 1));
  double (*wts)[27] = malloc(sizeof(double[27]) * (N > 0 ? N : 1));
  const int K = p->stencil == 1 ? 27 : 8; /* sites per particle (Eq. 5 stencil) */
  char *ok = (char *)calloc(N > 0 ? N : 1, 1);
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < N; ++a) {
    double R[3], v[3];
    int finite = 1;
    for (int d = 0; d < 3; ++d) {
      R[d] = c->x[d * N + a];
      v[d] = c->v[d * N + a];
      if (!isfinite(R[d]) || !isfinite(v[d])) finite = 0;
    }
    if (!finite) continue;
    ok[a] = 1;
    stencil_weights(c, R, sites[a], wts[a]);
    double uR[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < K; ++k) {
      double uk[3];
      site_velocity(c, sites[a][k], uk);
      for (int d = 0; d < 3; ++d) uR[d] += wts[a][k] * uk[d];
    }
    double xi[3] = {0.0, 0.0, 0.0};
    if (p->kT > 0.0 && p->friction > 0.0)
      orc_particle_variates(p->seed, p->replica, (uint64_t)a, (uint64_t)c->t_md, xi);
    double S2 = 0.0; /* S = sum of the squared stencil weights */
    for (int k = 0; k < K; ++k) S2 += wts[a][k] * wts[a][k];
    double adamp = p->friction * tau * (1.0 / p->particle_mass + S2 / p->rho0);
    double amp_a = amp * sqrt(fmax(0.0, 1.0 - 0.5 * adamp));
    for (int d = 0; d < 3; ++d)
      Fc[d * N + a] = -p->friction * (v[d] - uR[d]) + amp_a * xi[d];
  }
  for (int64_t a = 0; a < N; ++a)
    if (!ok[a]) c->nonfinite = 1;
  /* spreading: serial, in particle order */
  double *target = p->variant == 3 ? c->dJ : c->J;
  for (int64_t a = 0; a < N; ++a) {
    if (!ok[a]) continue;
    for (int k = 0; k < K; ++k)
      for (int d = 0; d < 3; ++d)
        target[d * S + sites[a][k]] -= wts[a][k] * tau * Fc[d * N + a];
  }
  if (p->variant == 3) {
    /* variant C: apply each receiving site's total transfer of this step to
       its populations, once (every site reads the state as of the step
       start: the updates touch disjoint sites) */
    for (int64_t a = 0; a < N; ++a) {
      if (!ok[a]) continue;
      for (int k = 0; k < K; ++k) {
        int64_t r = sites[a][k];
        double dJ[3] = {c->dJ[r], c->dJ[S + r], c->dJ[2 * S + r]};
        if (dJ[0] == 0.0 && dJ[1] == 0.0 && dJ[2] == 0.0) continue; /* done or empty */
        forcing_update(c, r, dJ);
        c->dJ[r] = c->dJ[S + r] = c->dJ[2 * S + r] = 0.0;
      }
    }
  }
  double L[3] = {p->nx, p->ny, p->nz};
  double h = tau / (2.0 * p->particle_mass);
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < N; ++a) {
    if (!ok[a]) continue;
    for (int d = 0; d < 3; ++d) {
      c->v[d * N + a] += h * (c->fcons[d * N + a] + Fc[d * N + a]);
      c->x[d * N + a] += tau * c->v[d * N + a];
      wrap_position(&c->x[d * N + a], &c->img[d * N + a], L[d]);
    }
  }
  conservative_forces(c);
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < N; ++a) {
    if (!ok[a]) continue;
    for (int d = 0; d < 3; ++d) c->v[d * N + a] += h * (c->fcons[d * N + a] + Fc[d * N + a]);
  }
  free(Fc); free(sites); free(wts); free(ok);
  c->t_md += 1;
  c->subs_since_lb += 1;
  return c->nonfinite ? ORC_ENONFINITE : ORC_OK;
}

/* Threads used by the parallel loops (OpenMP; 1 without it). */
void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int32_t orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Moments and global totals (Eq. 1-2; temperature from the mean kinetic      */
/* energy, Sec. 3).                                                          */
/* totals: [0] M = sum rho, [1..3] sum j + sum J, [4..6] momentum seen by the */
/* coupling (variant A: sum j; variant B: sum j + sum J), [7..9] sum m v,     */
/* [10] sum m v^2 / 2, [11] mean over sites of |j/rho|^2, [12] t_LB, [13]    */
/* t_MD, [14] particle temperature T_p = sum m |v|^2 / (3 N) (k_B = 1; the   */
/* mean kinetic energy per degree of freedom, no centre-of-mass subtraction; */
/* 0 without particles).                                                     */
/* ------------------------------------------------------------------------- */
int orc_moments(const orc_ctx *c, double *rho_out, double *u_out, double *totals) {
  int64_t S = c->nsites, N = c->p.n_particles;
  double M = 0.0, P[3] = {0, 0, 0}, Jt[3] = {0, 0, 0}, u2 = 0.0;
  for (int64_t r = 0; r < S; ++r) {
    double rho = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
      double fi = c->f[i * S + r];
      rho += fi;
      for (int d = 0; d < 3; ++d) j[d] += CV[i][d] * fi;
    }
    M += rho;
    for (int d = 0; d < 3; ++d) {
      P[d] += j[d];
      Jt[d] += c->J[d * S + r];
      u2 += (j[d] / rho) * (j[d] / rho);
    }
    if (rho_out) rho_out[r] = rho;
    if (u_out)
      for (int d = 0; d < 3; ++d) u_out[d * S + r] = j[d] / rho;
  }
  if (totals) {
    double Pp[3] = {0, 0, 0}, ke = 0.0, m = c->p.particle_mass;
    for (int64_t a = 0; a < N; ++a)
      for (int d = 0; d < 3; ++d) {
        double v = c->v[d * N + a];
        Pp[d] += m * v;
        ke += 0.5 * m * v * v;
      }
    totals[0] = M;
    for (int d = 0; d < 3; ++d) {
      totals[1 + d] = P[d] + Jt[d];
      totals[4 + d] = P[d] + (c->p.variant == 2 ? Jt[d] : 0.0);
      totals[7 + d] = Pp[d];
    }
    totals[10] = ke;
    totals[11] = u2 / (double)S;
    totals[12] = (double)c->t_lb;
    totals[13] = (double)c->t_md;
    totals[14] = N > 0 ? 2.0 * ke / (3.0 * (double)N) : 0.0;
  }
  return ORC_OK;
}
