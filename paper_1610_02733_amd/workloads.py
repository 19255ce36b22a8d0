"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the method itself: it only draws initial
particle positions and velocities, bead-spring chain conformations and
perturbed lattice states from numpy generators, and names the standard
configurations.  Both the HIP path and the CPU oracle are fed from here.

Workloads (lattice units a = tau_LB = 1; the paper's own system, a
pre-relaxed Kremer-Grest melt of 10 x 256 beads in (20 sigma)^3 (Sec. 3), is
not reproducible, so these stand in for it):

* ``c1``: 16^3, FP64, 32 free particles, n = 5, 100 LB steps (parity case).
* ``c2``: 128^3, FP32, 200 chains x 50 beads, harmonic bonds + WCA, n = 10.
* ``c2p``: the same shapes at stable dimensionless parameters (companion of c2).
* ``c3``: 256^3, FP32, 1e5 free particles at least 2 sites apart, n = 10
  (bandwidth-roofline case).
* ``c4``: 512 replicas, edges in {24,32,40,48}, 20..400 particles each.
* ``c5``: 64^3, 1000 particles under a constant force, n = 5 (adjoint case).
"""
from __future__ import annotations

import numpy as np

NU_1_6 = 1.0 / 6.0

CONFIGS = {
    "c1": dict(shape=(16, 16, 16), rho0=1.0, nu=NU_1_6, nu_bulk=-1.0, gamma_ghost=0.0,
               kT=1e-3, n_particles=32, particle_mass=1.0, friction=1.0, n_sub=5,
               lb_steps=100, seed=1, precision=64),
    "c2": dict(shape=(128, 128, 128), rho0=1.0, nu=NU_1_6, nu_bulk=-1.0, gamma_ghost=0.0,
               kT=1.0, n_particles=10_000, chain_len=50, particle_mass=1.0, friction=20.0,
               n_sub=10, lb_steps=1000, seed=2, precision=32, variant=2, force_model=2,
               k_bond=30.0, r0_bond=1.0, wca_eps=1.0, wca_sigma=1.0),
    # the same shapes as c2 at stable dimensionless parameters: energies in
    # units of kT (eps = kT, k = 30 kT / sigma^2), gamma tau_MD / m = 0.2,
    # chains grown without overlaps closer than 0.9 sigma
    "c2p": dict(shape=(128, 128, 128), rho0=1.0, nu=NU_1_6, nu_bulk=-1.0, gamma_ghost=0.0,
                kT=1e-4, n_particles=10_000, chain_len=50, particle_mass=1.0, friction=2.0,
                n_sub=10, lb_steps=1000, seed=2, precision=32, variant=2, force_model=2,
                k_bond=3e-3, r0_bond=1.0, wca_eps=1e-4, wca_sigma=1.0, min_dist=0.9),
    # the paper's polymer model (Kremer-Grest: FENE k = 30 kT, R0 = 1.5 sigma,
    # Lennard-Jones eps = kT cut at 2^(7/6) sigma) on the c2p shapes, in the
    # lattice units of n = 10, dt = 0.01 tau (kT = 0.01, nu = 0.3,
    # zeta = 20 mu/tau -> gamma = 2)
    "c2kg": dict(shape=(128, 128, 128), rho0=1.0, nu=0.3, nu_bulk=-1.0, gamma_ghost=0.0,
                 kT=0.01, n_particles=10_000, chain_len=50, particle_mass=1.0, friction=2.0,
                 n_sub=10, lb_steps=1000, seed=2, precision=32, variant=2, force_model=3,
                 k_bond=0.3, r0_bond=1.5, wca_eps=0.01, wca_sigma=1.0, min_dist=0.9),
    # gamma tau_MD / m = 1: two particles near one site exceed the explicit
    # step's stability bound in variant B, and a uniform draw holds ~280
    # same-cube pairs, so the particles are placed at least 2 sites apart
    # (with kT / gamma = 1e-5 they diffuse ~0.1 site in 1000 LB steps)
    "c3": dict(shape=(256, 256, 256), rho0=1.0, nu=NU_1_6, nu_bulk=-1.0, gamma_ghost=0.0,
               kT=1e-4, n_particles=100_000, particle_mass=1.0, friction=10.0, n_sub=10,
               lb_steps=200, seed=3, precision=32, min_dist=2.0),
    "c5": dict(shape=(64, 64, 64), rho0=1.0, nu=NU_1_6, nu_bulk=-1.0, gamma_ghost=0.0,
               kT=1e-4, n_particles=1000, particle_mass=1.0, friction=5.0, n_sub=5,
               lb_steps=50, seed=5, precision=32, force_model=1, f_ext=(1e-3, 0.0, 0.0)),
}


def free_particles(shape, n, kT, mass, seed):
    """Uniform positions in the periodic box, Maxwell velocities N(0, kT/m).

    Returns x[3,N], v[3,N] as float64 arrays (callers cast)."""
    rng = np.random.default_rng(seed)
    L = np.asarray(shape, np.float64).reshape(3, 1)
    x = rng.random((3, n)) * L
    x = np.minimum(x, np.nextafter(L, 0))  # keep strictly inside [0, L)
    v = rng.normal(0.0, np.sqrt(kT / mass) if kT > 0 else 0.0, (3, n))
    return x, v


def separated_particles(shape, n, kT, mass, seed, min_dist):
    """Homogeneous random positions with no two particles closer than min_dist
    (periodic minimum image): uniform positions, then, until no pair is too
    close, the higher-indexed particle of every close pair is drawn again
    uniformly; Maxwell velocities N(0, kT/m).

    Returns x[3,N], v[3,N] as float64 arrays."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    Ls = np.asarray(shape, np.float64)
    x = rng.random((n, 3)) * Ls
    x = np.minimum(x, np.nextafter(Ls, 0))
    for _ in range(1000):
        pairs = cKDTree(x, boxsize=Ls).query_pairs(min_dist, output_type="ndarray")
        if len(pairs) == 0:
            break
        redo = np.unique(pairs.max(1))
        x[redo] = np.minimum(rng.random((len(redo), 3)) * Ls, np.nextafter(Ls, 0))
    else:
        raise RuntimeError("could not separate the particles")
    v = rng.normal(0.0, np.sqrt(kT / mass) if kT > 0 else 0.0, (3, n))
    return np.ascontiguousarray(x.T), v


def workload_particles(cfg):
    """The particles of a named configuration: bead-spring chains when it has
    chains, separated free particles when it sets min_dist, else uniform free
    particles."""
    shape = cfg["shape"]
    if cfg.get("chain_len", 0) > 1 and cfg.get("force_model", 0) >= 2:
        return chains(shape, cfg["n_particles"] // cfg["chain_len"], cfg["chain_len"], cfg["kT"],
                      cfg["particle_mass"], cfg["seed"], min_dist=cfg.get("min_dist", 0.0))
    if cfg.get("min_dist", 0.0) > 0.0:
        return separated_particles(shape, cfg["n_particles"], cfg["kT"], cfg["particle_mass"],
                                   cfg["seed"], cfg["min_dist"])
    return free_particles(shape, cfg["n_particles"], cfg["kT"], cfg["particle_mass"], cfg["seed"])


def chains(shape, n_chains, chain_len, kT, mass, seed, bond=1.0, min_dist=0.0):
    """Bead-spring chains as random walks of fixed step `bond` from uniform
    starting points, wrapped into the box; consecutive indices are bonded.
    With min_dist > 0 a step (or chain start) closer than min_dist to any
    earlier bead (minimum image) is redrawn."""
    rng = np.random.default_rng(seed)
    L = np.asarray(shape, np.float64)
    x = np.zeros((3, n_chains * chain_len))
    placed = 0

    def clear(pos):
        if min_dist <= 0.0 or placed == 0:
            return True
        d = x[:, :placed] - pos[:, None]
        d -= L[:, None] * np.round(d / L[:, None])
        return np.min(np.sum(d * d, 0)) >= min_dist ** 2

    for c in range(n_chains):
        prev = None
        for b in range(chain_len):
            for _ in range(1000):
                if prev is None:
                    pos = rng.random(3) * L
                else:
                    d = rng.normal(size=3)
                    pos = prev + bond * d / np.linalg.norm(d)
                if clear(pos):
                    break
            x[:, c * chain_len + b] = pos
            prev = pos
            placed += 1
    x = np.mod(x, L.reshape(3, 1))
    x = np.minimum(x, np.nextafter(L.reshape(3, 1), 0))
    v = rng.normal(0.0, np.sqrt(kT / mass) if kT > 0 else 0.0, x.shape)
    return x, v


def perturbed_deviations(shape, weights, rho0, amplitude, seed, dtype=np.float64):
    """A random lattice state for parity tests, given as deviations
    df_i(r) = f_i(r) - w_i rho0 = w_i rho0 * amplitude * N(0,1), [19, nsites].

    The values are rounded to `dtype` so that a float32 run and the FP64
    oracle start from bit-identical numbers."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    w = np.asarray(weights, np.float64).reshape(19, 1)
    d = (w * rho0 * amplitude) * rng.standard_normal((19, n))
    return d.astype(dtype)


def to_cast(a, dtype):
    """Round an input array to the run precision and back to float64, so both
    sides see identical values."""
    return np.asarray(a, dtype).astype(np.float64)


def batch_replicas(n_rep, seed, edges=(24, 32, 40, 48), np_range=(20, 400),
                   gamma_range=(1.0, 20.0)):
    """Per-replica (edge, n_particles, gamma) draws of the batched ensemble."""
    rng = np.random.default_rng(seed)
    e = rng.choice(np.asarray(edges), n_rep)
    n = rng.integers(np_range[0], np_range[1] + 1, n_rep)
    g = rng.uniform(gamma_range[0], gamma_range[1], n_rep)
    return e.astype(int), n.astype(int), g
