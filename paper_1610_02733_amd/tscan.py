"""Particle temperature against friction, time-scale contrast and MD step
for the coupling variants: the experiment behind the paper's Figs. 3, 4 and 6
(Sec. 3), run on the batched engine.

The paper measures the mean kinetic temperature of a bead-spring polymer
solution coupled to the fluid, in Lennard-Jones units (length sigma, mass
mu, time tau): kT = eps, fluid density 1 mu/sigma^3, shear viscosity
eta = 3 eps tau/sigma^3, lattice spacing a = sigma, 10 chains of 256 beads
in a (20 sigma)^3 box, MD steps dt in {0.001, 0.005, 0.01} tau, contrasts
n = tau_LB/dt in {1, 5, 10}.  The library works in lattice units (a = 1,
tau_LB = 1, bead mass 1), so with s = n dt (tau_LB in units of tau):

    kT = s^2,  nu = 3 s,  zeta_lattice = zeta s,
    bead forces: LJ eps = kT, sigma = 1; bond stiffness k = 30 kT.

The paper's system is a pre-relaxed Kremer-Grest solution (Lennard-Jones
between all beads cut at 2^(7/6) sigma, FENE bonds k = 30 eps/sigma^2,
R0 = 1.5 sigma): model "kg" (force model 3) uses that force field on
seeded random-walk chains, which are not pre-relaxed; model "wca"
(force model 2: harmonic bonds, WCA repulsion) is a good-solvent variant.  One batch per (variant, n, dt) holds one
replica per friction value; every replica starts from the same seeded
configuration and draws its own noise (replica id).  The temperature is
2 KE / (3 N kT), sampled every `sample_tau` after `equil_tau`, with a
block-average error.

Every step runs in the library (``lbmd.Batch``); this module only sets up
the replicas and collects the totals.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import lbmd
from . import workloads as wl

PAPER_SYSTEM = dict(box=20, n_chains=10, chain_len=256)
PAPER_DTS = (0.001, 0.005, 0.01)
PAPER_NS = (1, 5, 10)
ZETAS = (1.0, 2.0, 5.0, 10.0, 20.0)


def lattice_params(n, dt, zeta, model="kg"):
    """Lattice-unit parameters of one scan point (LJ units in, see module
    doc).  model "kg": the paper's Kremer-Grest force field (FENE k = 30 eps,
    R0 = 1.5 sigma; LJ cut at 2^(7/6) sigma); "wca": harmonic bonds
    (k = 30 eps, r0 = sigma) and WCA."""
    s = n * dt
    kT = s * s
    p = dict(kT=kT, nu=3.0 * s, friction=zeta * s, k_bond=30.0 * kT, wca_eps=kT, wca_sigma=1.0)
    if model == "kg":
        p.update(force_model=3, r0_bond=1.5)
    else:
        p.update(force_model=2, r0_bond=1.0)
    return p


def _block_error(samples, blocks=8):
    a = np.asarray(samples, float)
    if len(a) < 2 * blocks:
        return float(np.std(a) / max(np.sqrt(len(a)), 1.0))
    m = a[: len(a) // blocks * blocks].reshape(blocks, -1).mean(1)
    return float(np.std(m, ddof=1) / np.sqrt(blocks))


_CONFIGS = {}


def _start(box, n_chains, chain_len, seed):
    """Seeded chain positions and unit-temperature velocities (cached: every
    batch of a scan starts from the same configuration)."""
    key = (box, n_chains, chain_len, seed)
    if key not in _CONFIGS:
        _CONFIGS[key] = wl.chains((box, box, box), n_chains, chain_len, 1.0, 1.0, seed,
                                  bond=0.97, min_dist=0.9)
    return _CONFIGS[key]


def scan_batch(variant, n, dt, zetas, *, box=20, n_chains=10, chain_len=256, t_tau=50.0,
               equil_tau=10.0, sample_tau=0.5, seed=1, precision=32, model="kg", stencil=0,
               device="cuda"):
    """One batch: the friction values `zetas` at fixed (variant, n, dt).
    Returns one dict per friction value."""
    shape = (box, box, box)
    N = n_chains * chain_len
    s = n * dt
    x, v1 = _start(box, n_chains, chain_len, seed)
    v = v1 * s  # Maxwell velocities at kT = s^2
    reps = []
    for r, z in enumerate(zetas):
        kw = dict(precision=precision, n_sub=n, variant=variant, seed=seed, replica=r,
                  n_particles=N, particle_mass=1.0, chain_len=chain_len, rho0=1.0,
                  stencil=stencil)
        kw.update(lattice_params(n, dt, z, model))
        reps.append((shape, kw))
    B = lbmd.Batch(reps, device=device)
    B.bind_particles([x] * len(zetas), [v] * len(zetas))
    every = max(1, int(round(sample_tau / s)))
    equil = int(round(equil_tau / s))
    total = int(round(t_tau / s))
    B.run_cycles(equil)
    samples = []
    done = equil
    while done + every <= total:
        B.run_cycles(every)
        done += every
        samples.append(B.temperatures())
    B.close()
    T = np.array(samples)  # [samples, replicas]
    out = []
    for r, z in enumerate(zetas):
        col = T[:, r]
        ok = bool(np.isfinite(col).all())
        out.append(dict(variant=variant, n=n, dt=dt, zeta=float(z), stencil=stencil,
                        zeta_dt=float(z * dt), T_over_kT=float(np.mean(col)) if ok else None,
                        err=_block_error(col) if ok else None, samples=len(col),
                        cycles=done, finite=ok))
    return out


def temperature_scan(variants=(1, 2), ns=PAPER_NS, dts=PAPER_DTS, zetas=ZETAS, log=None,
                     **kw):
    """The full scan: one batch per (variant, n, dt); returns the rows."""
    rows = []
    for variant in variants:
        for n in ns:
            for dt in dts:
                t0 = time.perf_counter()
                res = scan_batch(variant, n, dt, zetas, **kw)
                if log is not None:
                    log(f"variant {variant} n {n} dt {dt}: " +
                        ", ".join(f"zeta {r['zeta']:g} T/kT {r['T_over_kT']:.4f}"
                                  f"+-{r['err']:.4f}" if r['finite'] else f"zeta {r['zeta']:g} diverged"
                                  for r in res) + f"  ({time.perf_counter() - t0:.1f} s)")
                rows += res
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--variants", default="1,2,3")
    ap.add_argument("--ns", default="1,5,10")
    ap.add_argument("--dts", default="0.001,0.005,0.01")
    ap.add_argument("--zetas", default=",".join(f"{z:g}" for z in ZETAS))
    ap.add_argument("--t-tau", type=float, default=50.0, help="run length per point, tau")
    ap.add_argument("--equil-tau", type=float, default=10.0)
    ap.add_argument("--sample-tau", type=float, default=0.5)
    ap.add_argument("--precision", type=int, default=32)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--model", default="kg", choices=["kg", "wca"],
                    help="kg: the paper's Kremer-Grest force field; wca: harmonic + WCA")
    ap.add_argument("--stencil", type=int, default=0, choices=[0, 1],
                    help="0: trilinear interpolation; 1: three-point kernel (27 sites)")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    rows = temperature_scan(
        variants=[int(t) for t in args.variants.split(",")],
        ns=[int(t) for t in args.ns.split(",")],
        dts=[float(t) for t in args.dts.split(",")],
        zetas=[float(t) for t in args.zetas.split(",")],
        t_tau=args.t_tau, equil_tau=args.equil_tau, sample_tau=args.sample_tau,
        precision=args.precision, seed=args.seed, model=args.model, stencil=args.stencil,
        log=log, **PAPER_SYSTEM)
    for r in rows:
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
