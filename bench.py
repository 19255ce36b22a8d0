"""Throughput of the coupled LB/MD cycle on one MI355X.

One step = one coupled cycle of the method: n MD steps of the particle
coupling (md_couple_substep) followed by one LB collide-and-stream step
(lb_step), over the bandwidth-roofline workload: a 256^3 periodic lattice
(16.8 M sites), FP32 populations stored as deviations, 1e5 free particles,
n = 10, gamma = 10, kT = 1e-4, variant 2.  Variant 1 is timed the same way
for the cost ratio.  Inputs are seeded and synthetic (uniform positions,
Maxwell velocities) and resident in HBM before timing starts.

Prints one JSON line.  value = lattice-site updates per second of the whole
coupled cycle (MLUPS).  roofline: the fused collide-stream kernel, 152
algorithmic bytes per FP32 site update (19 populations read, 19 written),
timed with HIP events around each launch inside the timed region.
cpu_baseline: the FP64 CPU oracle (OpenMP) on the same workload, 20 cycles.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_SITE = {32: 152, 64: 304}
METRIC = "LB MLUPS & %HBM peak; coupled steps/s: batched & adjoint vs plain, at tol"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(launches_bytes_key="traffic_bytes"):
    """HBM bytes per collide-stream launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernel sources changed
    since the counters were taken."""
    import hashlib
    f = os.path.join(ROOT, "profiles", "traffic_collide_stream_scale256_fp32.json")
    if not os.path.exists(f):
        return None
    rec = json.load(open(f))
    h = hashlib.sha256()
    for src in ("paper_1610_02733_amd/csrc/lattice.hip", "paper_1610_02733_amd/csrc/lbmd_device.hpp",
                "paper_1610_02733_amd/csrc/lbmd_internal.hpp", "paper_1610_02733_amd/csrc/forcing.hpp"):
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != rec.get("source_sha256"):
        return None
    return rec[launches_bytes_key]


WORKLOAD_NAMES = {
    "c3": "scale-256^3: 256^3 lattice, 1e5 free particles (>= 2 sites apart), n=10, "
          "gamma=10, kT=1e-4, "
          "FP32 deviations, variant 2",
    "c2": "polymer-128^3: 128^3 lattice, 200 chains x 50 beads (harmonic k=30 + WCA, cell "
          "list), n=10, gamma=20, kT=1, FP32 deviations, variant 2",
    "c2p": "polymer-128^3-stable: 128^3 lattice, 200 chains x 50 beads (harmonic k=30 kT + "
           "WCA eps=kT, cell list), n=10, gamma=2, kT=1e-4, FP32 deviations, variant 2",
    "c2kg": "polymer-128^3-kremer-grest: 128^3 lattice, 200 chains x 50 beads (FENE k=30 kT, "
            "R0=1.5 + LJ eps=kT cut at 2^(7/6), cell list), n=10, gamma=2, kT=0.01, nu=0.3, "
            "FP32 deviations, variant 2",
}
# workload whose collide-stream launch the committed PMC summary covers
TRAFFIC_WORKLOAD = "c3"
FORCE_KEYS = ("force_model", "chain_len", "k_bond", "r0_bond", "wca_eps", "wca_sigma", "f_ext")


def sim_kwargs(cfg, variant):
    kw = dict(precision=cfg["precision"], n_sub=cfg["n_sub"], variant=variant, kT=cfg["kT"],
              nu=cfg["nu"], rho0=cfg["rho0"], friction=cfg["friction"],
              n_particles=cfg["n_particles"], seed=cfg["seed"],
              particle_mass=cfg["particle_mass"])
    kw.update({k: cfg[k] for k in FORCE_KEYS if k in cfg})
    return kw


def run_variant(lbmd, torch, cfg, variant, x, v, steps, warmup, stencil=0, sort_every=0):
    shape = cfg["shape"]
    sim = lbmd.Lattice(shape, stencil=stencil, **sim_kwargs(cfg, variant))
    sim.bind_particles(x, v)
    sort = sort_every > 0 and cfg.get("force_model", 0) <= 1
    if sort:
        sim.sort_particles()
    stream = sim.stream
    L = lbmd.lib()
    h = sim._h
    n = cfg["n_sub"]

    def cycle(ev_a=None, ev_b=None, ev_0=None):
        if ev_0 is not None:
            ev_0.record(stream)
        for _ in range(n):
            rc = L.md_couple_substep(h)
            if rc:
                raise lbmd.LbmdError(rc, "md_couple_substep")
        if ev_a is not None:
            ev_a.record(stream)
        rc = L.lb_step(h)
        if rc:
            raise lbmd.LbmdError(rc, "lb_step")
        if ev_b is not None:
            ev_b.record(stream)

    for _ in range(warmup):
        cycle()
    torch.cuda.synchronize()
    # HIP events bracket the collide-stream launch of every 10th cycle, and
    # the MD steps (corner refill included) of every 10th cycle offset by 5
    # (an event between two kernels lets the queue drain before the next
    # launch, which costs idle time, so they are kept sparse)
    every = 10
    half = every // 2
    ev_a = [torch.cuda.Event(enable_timing=True) for _ in range(0, steps, every)]
    ev_b = [torch.cuda.Event(enable_timing=True) for _ in range(0, steps, every)]
    ev_p0 = [torch.cuda.Event(enable_timing=True) for _ in range(half, steps, every)]
    ev_p1 = [torch.cuda.Event(enable_timing=True) for _ in range(half, steps, every)]
    t0 = time.perf_counter()
    for k in range(steps):
        # spatial reordering of the particles at LB-step boundaries, timed
        if sort and k > 0 and k % sort_every == 0:
            sim.sort_particles()
        if k % every == 0:
            cycle(ev_a[k // every], ev_b[k // every])
        elif k % every == half:
            cycle(ev_p1[k // every], None, ev_p0[k // every])
        else:
            cycle()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k1_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(ev_a, ev_b)]))
    part_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(ev_p0, ev_p1)])) \
        if ev_p0 else float("nan")
    tot = sim.moments(allow_nonfinite=True)
    finite = bool(np.isfinite(tot).all())
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return wall, k1_ms, finite, part_ms


def copy_ceiling(lbmd, torch, nbytes, reps=20):
    """Measured ceiling of a read+write stream of the collide-stream kernel's
    volume: the library's non-temporal 16-byte device copy of one population
    buffer into the other, in GB/s of bytes read plus bytes written."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        lbmd.stream_copy(dst, src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        lbmd.stream_copy(dst, src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def error_statement(lbmd, torch, cfg, x, v, cycles=10):
    """Form (iii) error statement on the full workload: the FP32 run (deviations
    stored in FP32) against the same run in FP64 (same seed, same noise, same
    start) after `cycles` coupled cycles, variant 2.  Population error per
    population relative to its rest value w_i rho0, max and RMS over all 19 x
    S populations; particle velocity error relative to max(|v|, sqrt(kT/m)).
    The FP64 run itself is checked against the FP64 oracle at this size by
    the sampled-site parity test."""
    shape = cfg["shape"]
    out = {}
    sims = {}
    for prec in (64, 32):
        kw = sim_kwargs(cfg, 2)
        kw["precision"] = prec
        s = lbmd.Lattice(shape, **kw)
        s.bind_particles(x, v)
        s.run_cycles(cycles)
        sims[prec] = s
    w = torch.tensor(lbmd.WEIGHTS, dtype=torch.float64, device="cuda").reshape(19, 1) * cfg["rho0"]
    sq = 0.0
    mx = 0.0
    f64 = sims[64].populations()
    f32 = sims[32].populations()
    for i in range(19):  # one velocity at a time keeps the FP64 temporaries small
        d = (f32[i].double() - f64[i]).abs() / w[i]
        mx = max(mx, d.max().item())
        sq += (d * d).sum().item()
    n = 19 * f64.shape[1]
    v64, v32 = sims[64].v, sims[32].v
    vs = max(v64.abs().max().item(), float(np.sqrt(cfg["kT"] / cfg["particle_mass"])))
    out = dict(cycles=cycles, compared="FP32 vs FP64 run on the GPU, variant 2",
               pop_max_rel=mx, pop_rms_rel=float(np.sqrt(sq / n)),
               v_max_rel=(v32 - v64).abs().max().item() / vs,
               finite=bool(torch.isfinite(f64).all().item() and torch.isfinite(f32).all().item()))
    for s in sims.values():
        s.close()
    del sims, f64, f32
    torch.cuda.empty_cache()
    return out


def _c4_replicas(lbmd, nrep, gamma_range=(1.0, 20.0), variant=2, draw_seed=4):
    """The batched ensemble: nrep periodic replicas, edges in {24,32,40,48},
    20..400 free particles, gamma uniform in gamma_range, kT = 1e-3, n = 5,
    FP32; replica r draws its particles from seed 4000 + r."""
    from paper_1610_02733_amd import workloads as wl
    edges, nps, gammas = wl.batch_replicas(nrep, seed=draw_seed, gamma_range=gamma_range)
    reps, xs, vs = [], [], []
    for r in range(nrep):
        shape = (int(edges[r]),) * 3
        kw = dict(precision=32, n_sub=5, variant=variant, kT=1e-3, nu=1.0 / 6.0, seed=4,
                  replica=r, n_particles=int(nps[r]), friction=float(gammas[r]),
                  particle_mass=1.0)
        x, v = wl.free_particles(shape, int(nps[r]), 1e-3, 1.0, 4000 + r)
        reps.append((shape, kw))
        xs.append(x)
        vs.append(v)
    return reps, xs, vs, edges, nps, gammas


def _time_batch_vs_serial(lbmd, torch, reps, xs, vs, cycles, warm=2):
    """Batched (one launch per phase, captured cycle) against the same
    replicas as separate systems, per-call launches and per-replica captured
    cycles.  Every leg starts from the same bound state, runs `warm` untimed
    cycles and then the same `cycles` timed cycles, so all legs do the same
    work (a replica that diverges does so at the same cycle in each)."""
    import tempfile
    out = {}
    B = lbmd.Batch(reps)
    B.bind_particles(xs, vs)
    out["autotune"] = B.autotune(os.path.join(tempfile.gettempdir(), "lbmd_autotune.json"))
    B.run_cycles(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.run_cycles(cycles)
    torch.cuda.synchronize()
    out["batched_ms_per_cycle"] = (time.perf_counter() - t0) / cycles * 1e3
    out["finite_replicas_batched"] = int(np.isfinite(B.temperatures()).sum())
    B.close()
    del B
    torch.cuda.empty_cache()
    sims = []
    for (shape, kw), x, v in zip(reps, xs, vs):
        s = lbmd.Lattice(shape, **kw)
        s.bind_particles(x, v)
        sims.append(s)
    for s in sims:
        s.cycle(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.cycle(cycles)
    torch.cuda.synchronize()
    out["serial_ms_per_cycle"] = (time.perf_counter() - t0) / cycles * 1e3
    for s in sims:  # the per-replica graphs, captured outside the timed window
        s.run_cycles(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.run_cycles(cycles)
    torch.cuda.synchronize()
    out["serial_graph_ms_per_cycle"] = (time.perf_counter() - t0) / cycles * 1e3
    fin = 0
    for s in sims:
        tot = s.moments(allow_nonfinite=True)
        fin += int(np.isfinite(tot[lbmd.TOT["tpart"]]) or s.N == 0)
        s.close()
    out["finite_replicas_serial"] = fin
    del sims
    torch.cuda.empty_cache()
    out["speedup_vs_serial"] = round(out["serial_ms_per_cycle"] / out["batched_ms_per_cycle"], 2)
    out["speedup_vs_serial_graphs"] = round(
        out["serial_graph_ms_per_cycle"] / out["batched_ms_per_cycle"], 2)
    for k in ("batched_ms_per_cycle", "serial_ms_per_cycle", "serial_graph_ms_per_cycle"):
        out[k] = round(out[k], 3)
    return out


def _temperature_drift(lbmd, torch, reps, xs, vs, gammas, cycles=1000, every=10):
    """Per-replica particle temperature T_p / kT over `cycles` LB steps
    (the ensemble statistics of the paper's Sec. 3 temperature test), in
    bins of the dimensionless friction gamma tau_MD / m: replicas, diverged
    replicas, mean T_p/kT of the finite ones over the second half, and its
    drift (last quarter minus second quarter)."""
    B = lbmd.Batch(reps)
    B.bind_particles(xs, vs)
    series = []
    for _ in range(cycles // every):
        B.run_cycles(every)
        series.append(B.temperatures())
    B.close()
    del B
    torch.cuda.empty_cache()
    T = np.array(series)  # [samples, replicas]
    ns = T.shape[0]
    g_tau = np.asarray(gammas) * 0.2  # tau_MD = 1/5, m = 1
    fin = np.isfinite(T).all(0)
    bins = [(0.2, 0.5), (0.5, 1.0), (1.0, 2.0), (2.0, 4.0)]
    rows = []
    for lo, hi in bins:
        sel = (g_tau >= lo) & (g_tau < hi) if hi < 4.0 else (g_tau >= lo)
        ok = sel & fin
        row = dict(gamma_tau=[lo, hi], replicas=int(sel.sum()), diverged=int((sel & ~fin).sum()))
        if ok.any():
            half = T[ns // 2:, ok]
            q2, q4 = T[ns // 4: ns // 2, ok], T[3 * ns // 4:, ok]
            row.update(mean_T_over_kT=round(float(half.mean()), 4),
                       replica_sd=round(float(half.mean(0).std()), 4),
                       drift=round(float(q4.mean() - q2.mean()), 4))
        rows.append(row)
    return dict(lb_steps=cycles, sample_every=every, finite_replicas=int(fin.sum()),
                replicas=int(T.shape[1]), bins=rows)


def batch_measure(lbmd, torch, nrep=512, cycles=10, drift_cycles=1000):
    """Batched ensemble (form ii): 512 independent replicas of uneven box and
    particle counts in one batch against the same replicas as separate
    systems, and the ensemble's temperature statistics over 1000 LB steps
    in variants A and B.  The C4 draws reach gamma tau_MD / m = 4, beyond the
    explicit step's stability bound (about 2 / (1 + S)), so part of that
    ensemble diverges; the timing is therefore also taken on a stable redraw
    (gamma in [1, 4.5]) where every replica stays finite."""
    reps, xs, vs, edges, nps, gammas = _c4_replicas(lbmd, nrep)
    sites = int(sum(int(e) ** 3 for e in edges))
    out = dict(replicas=nrep, sites=sites, particles=int(nps.sum()), timed_cycles=cycles)
    log("  batch timing, C4 draws (gamma in [1, 20])")
    out["c4"] = _time_batch_vs_serial(lbmd, torch, reps, xs, vs, cycles)
    out["c4"]["batched_mlups"] = round(sites / (out["c4"]["batched_ms_per_cycle"] * 1e-3) / 1e6, 1)
    log("  batch timing, stable redraw (gamma in [1, 4.5])")
    sreps, sxs, svs, sedges, snps, sg = _c4_replicas(lbmd, nrep, gamma_range=(1.0, 4.5))
    out["stable"] = _time_batch_vs_serial(lbmd, torch, sreps, sxs, svs, cycles)
    out["stable"]["sites"] = int(sum(int(e) ** 3 for e in sedges))
    drift = {}
    for variant in (1, 2):
        log(f"  temperature drift, variant {variant}, {drift_cycles} LB steps")
        vreps = [(shape, dict(kw, variant=variant)) for shape, kw in reps]
        drift[f"variant{variant}"] = _temperature_drift(lbmd, torch, vreps, xs, vs, gammas,
                                                         cycles=drift_cycles)
    out["temperature_drift"] = drift
    return out


def adjoint_measure(lbmd, torch, reps=3):
    """Reverse mode on the 64^3 adjoint case (1000 particles under a constant
    force, gamma = 5, kT = 1e-4, n = 5, 50 LB steps, FP32 populations,
    variant 2): wall time of the plain forward pass (captured cycles) against
    the backward pass (re-run of each 10-cycle segment from its saved state
    with recording, then the adjoint sweep), for the drift gradient."""
    from paper_1610_02733_amd import workloads as wl
    cfg = dict(wl.CONFIGS["c5"])
    shape, N, T, K = cfg["shape"], cfg["n_particles"], cfg["lb_steps"], 10
    rng = np.random.default_rng(cfg["seed"])
    x0 = rng.random((3, N)) * np.asarray(shape, float)[:, None]
    v0 = 1e-2 * rng.standard_normal((3, N))
    kw = dict(n_sub=cfg["n_sub"], variant=2, kT=cfg["kT"], seed=cfg["seed"], nu=cfg["nu"],
              friction=cfg["friction"], particle_mass=cfg["particle_mass"], precision=32,
              n_particles=N, force_model=1, f_ext=cfg["f_ext"])
    sim = lbmd.Lattice(shape, **kw)
    sim.bind_particles(x0, v0)
    states = [sim.save_state() for _ in range(T // K)]
    sim.adjoint_attach(K)
    xbar = torch.zeros((3, N), dtype=torch.float64, device="cuda")
    xbar[0] = 1.0 / N
    fwd, fwd_ck, bwd = [], [], []
    grads = None
    for it in range(reps + 1):
        sim.load_state(states[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run_cycles(T)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sim.load_state(states[0])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for k in range(T // K):
            if k > 0:
                sim.save_state(states[k])
            sim.run_cycles(K)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        sim.adjoint_seed(xbar, None)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        for k in reversed(range(T // K)):
            sim.adjoint_record(states[k], K)
            sim.adjoint_sweep(K)
        xb, vb, g = sim.adjoint_result()
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        if it > 0:  # the first pass warms up graphs and allocations
            fwd.append(t1 - t0)
            fwd_ck.append(t3 - t2)
            bwd.append(t5 - t4)
            grads = g
    sim.close()
    f, fc, b = (float(np.median(a)) for a in (fwd, fwd_ck, bwd))
    return dict(config="64^3, 1000 particles, n=5, 50 LB steps, checkpoint 10, FP32, variant 2",
                forward_ms=round(f * 1e3, 3), forward_with_checkpoints_ms=round(fc * 1e3, 3),
                backward_ms=round(b * 1e3, 3), backward_over_forward=round(b / f, 3),
                forward_plus_backward_over_forward=round((fc + b) / f, 3),
                drift_grad={"gamma": grads["gamma"], "nu": grads["nu"],
                            "f_ext": [float(t) for t in grads["f_ext"]]})


def autotune_report(lbmd, torch, cfg, x, v, cycles=20):
    """The autotuner's picks (collide-stream grid, particle-kernel grid,
    coupling lanes per particle) on the benchmark workload and on the 64^3,
    1000-particle adjoint case, each with the cycle time under the picks and
    under the built-in shapes (grids 0: one block per work item; lanes 0:
    two per particle)."""
    import tempfile
    from paper_1610_02733_amd import workloads as wl
    c5 = dict(wl.CONFIGS["c5"])
    x5, v5 = wl.free_particles(c5["shape"], c5["n_particles"], c5["kT"], 1.0, c5["seed"])
    cases = {"bench workload": (cfg, x, v), "64^3 / 1000 particles (adjoint case)": (c5, x5, v5)}
    out = {}
    for name, (cf, xx, vv) in cases.items():
        sim = lbmd.Lattice(cf["shape"], **sim_kwargs(cf, 2))
        sim.bind_particles(xx, vv)
        if cf.get("force_model", 0) <= 1 and cf["n_particles"] > 1000:
            sim.sort_particles()
        sim.run_cycles(2)
        path = os.path.join(tempfile.gettempdir(), "lbmd_autotune_report.json")
        if os.path.exists(path):
            os.remove(path)
        pick = sim.autotune(path)
        times = {}
        for label, shape in (("tuned", pick), ("default", dict(lb_blocks=0, part_blocks=0,
                                                               couple_lanes=0))):
            sim.set_launch_shape(**shape)
            sim.run_cycles(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.run_cycles(cycles)
            torch.cuda.synchronize()
            times[label] = (time.perf_counter() - t0) / cycles * 1e3
        sim.close()
        del sim
        torch.cuda.empty_cache()
        out[name] = dict(pick=pick, ms_per_cycle_tuned=round(times["tuned"], 4),
                         ms_per_cycle_default=round(times["default"], 4))
    return out


def cpu_baseline(cfg, x, v, cycles=20, warmup=1):
    """FP64 CPU oracle on the full workload (same lattice, particles, seed and
    parameters, variant 2): `warmup` untimed cycles (first touch of its ~6 GB),
    then `cycles` coupled cycles (one LB step each) timed, on the OpenMP
    threads of the host process (OMP_NUM_THREADS, else every core in its
    affinity set)."""
    import oracle
    oracle.build(force=False)
    shape = cfg["shape"]
    S = int(np.prod(shape))
    N = cfg["n_particles"]
    if cfg.get("force_model", 0) >= 2:
        # the oracle's conservative forces are a serial all-pairs sum
        cycles = min(cycles, 2)
    o = oracle.Oracle(*shape, n_sub=cfg["n_sub"], variant=2, kT=cfg["kT"], nu=cfg["nu"],
                      rho0=cfg["rho0"], friction=cfg["friction"], n_particles=N,
                      seed=cfg["seed"], particle_mass=cfg["particle_mass"],
                      **{k: cfg[k] for k in FORCE_KEYS if k in cfg})
    o.set_particles(x, v)
    o.cycle(warmup)
    t0 = time.perf_counter()
    o.cycle(cycles)
    dt = time.perf_counter() - t0
    o.close()
    threads = oracle.max_threads()
    return dict(value=round(S * cycles / dt / 1e6, 3), unit="MLUPS", cores=threads, kind="oracle",
                substeps_per_s=round(cycles * cfg["n_sub"] / dt, 3),
                affinity_cpus=len(os.sched_getaffinity(0)),
                sample=f"full workload: {shape[0]}x{shape[1]}x{shape[2]} lattice, {N} particles, "
                       f"{cycles} coupled cycles (LB steps) of n={cfg['n_sub']} after {warmup} "
                       f"untimed, variant 2, FP64, {threads} OpenMP threads, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the 256^3 workload in variant 2 sits on its stability bound (two
    # particles in one cube): with its seeded start the first particles
    # diverge after about 175 cycles, so the default timed window (10 + 100
    # cycles) stays well inside the finite stretch
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cycles", type=int, default=20,
                    help="coupled cycles (LB steps) of the FP64 oracle timed on the host")
    ap.add_argument("--no-error-statement", action="store_true",
                    help="skip the FP32-vs-FP64 comparison on the workload")
    ap.add_argument("--variants", default="1,2,3",
                    help="coupling variants to time (1 = A, 2 = B, 3 = C); the JSON value is variant 2")
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "c2p", "c2kg"],
                    help="c3: 256^3, 1e5 free particles (default); c2: 128^3 polymer "
                         "solution, 200 chains x 50 beads, bonds + WCA, as specified "
                         "(unstable); c2p: the same shapes at stable parameters; c2kg: "
                         "the same shapes with the paper's Kremer-Grest force field")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner report")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 512-replica batched-ensemble measurement")
    ap.add_argument("--drift-cycles", type=int, default=1000,
                    help="LB steps of the batched ensemble's temperature statistics")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the reverse-mode (adjoint) cost measurement")
    ap.add_argument("--sort-every", type=int, default=50,
                    help="reorder the particles spatially every K cycles inside the timed "
                         "loop (and once after binding); 0 keeps the input order")
    ap.add_argument("--no-stencil3", action="store_true",
                    help="skip timing the three-point (27-site) interpolation stencil")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the lattice "
              "is not sharded across devices in this library", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1610_02733_amd import lbmd
    from paper_1610_02733_amd import workloads as wl

    if args.copy_calibration:
        n = 19 * 256 ** 3  # one FP32 population buffer of the 256^3 lattice
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            lbmd.stream_copy(dst, src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read_per_dispatch": 4 * n,
                                               "bytes_written_per_dispatch": 4 * n,
                                               "dispatches": 5}}), flush=True)
        return

    cfg = dict(wl.CONFIGS[args.workload])
    shape = cfg["shape"]
    S = int(np.prod(shape))
    copy_gbs = copy_ceiling(lbmd, torch, 19 * S * (4 if cfg["precision"] == 32 else 8))
    x, v = wl.workload_particles(cfg)

    res = {}
    for variant in [int(t) for t in args.variants.split(",")]:
        log(f"timing variant {variant}: {args.warmup} warmup + {args.steps} cycles")
        res[variant] = run_variant(lbmd, torch, cfg, variant, x, v, args.steps, args.warmup,
                                   sort_every=args.sort_every)
        log(f"  wall {res[variant][0]:.3f} s, collide-stream {res[variant][1]:.4f} ms/launch, "
            f"MD steps {res[variant][3]:.4f} ms/cycle")
    main_v = 2 if 2 in res else min(res)
    wall, k1_ms, finite, part_ms = res[main_v]
    ms_per_step = wall / args.steps * 1e3
    mlups = S * args.steps / wall / 1e6
    bpu = BYTES_PER_SITE[cfg["precision"]]
    achieved = bpu * S / (k1_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES[args.workload],
                   "lattice": list(shape), "particles": cfg["n_particles"],
                   "n_sub": cfg["n_sub"], "variant": main_v,
                   "particle_sort_every": args.sort_every
                   if cfg.get("force_model", 0) <= 1 else 0},
        "coupled_substeps_per_s": round(cfg["n_sub"] * args.steps / wall, 1),
        "coupled_cycle_mlups": round(mlups, 1),
        "lb_only_mlups": round(S / (k1_ms * 1e-3) / 1e6, 1),
        "particle_side": {"ms_per_cycle": round(part_ms, 4),
                          "us_per_md_step": round(part_ms / cfg["n_sub"] * 1e3, 2),
                          "note": "HIP events around the n MD steps of a cycle (corner "
                                  "refill, coupling and after-step kernels)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic() if args.workload == TRAFFIC_WORKLOAD else None,
                     "kernel": "collide_stream (fused pull MRT+noise+Guo)",
                     "bytes_per_site": bpu, "launch_ms": round(k1_ms, 4),
                     "copy_ceiling_GBs": round(copy_gbs, 1),
                     "frac_of_copy_ceiling": round(achieved / copy_gbs, 4)},
        "finite_after_run": {f"variant{vv}": res[vv][2] for vv in res},
    }
    if 1 in res and 2 in res:
        out["variant1_ms_per_step"] = round(res[1][0] / args.steps * 1e3, 4)
        out["variant2_over_variant1"] = round(res[2][0] / res[1][0], 4)
    if 1 in res and 3 in res:
        out["variant3_ms_per_step"] = round(res[3][0] / args.steps * 1e3, 4)
        out["variant3_over_variant1"] = round(res[3][0] / res[1][0], 4)
        out["variant3_note"] = ("variant C timed in the library's closed form: the interval's "
                                "accumulated transfer applied as momentum and stress increments "
                                "inside the LB step, equal to the per-MD-step population update "
                                "in exact arithmetic (parity with the oracle's per-step update); "
                                "not comparable with the paper's per-step CPU cost")
    if not args.no_stencil3 and main_v in res:
        log(f"three-point stencil, variant {main_v}: {args.warmup} warmup + {args.steps} cycles")
        w3, k3, f3, p3 = run_variant(lbmd, torch, cfg, main_v, x, v, args.steps, args.warmup,
                                     stencil=1, sort_every=args.sort_every)
        out["stencil3"] = {"variant": main_v, "ms_per_step": round(w3 / args.steps * 1e3, 4),
                           "over_trilinear": round(w3 / res[main_v][0], 4), "finite": f3,
                           "particle_us_per_md_step": round(p3 / cfg["n_sub"] * 1e3, 2)}
    if not args.no_autotune:
        log("autotune: picks against the built-in launch shapes")
        out["autotune"] = autotune_report(lbmd, torch, cfg, x, v)
    if not args.no_batch:
        log("batched ensemble: 512 replicas, batched vs serial, temperature drift")
        out["batch"] = batch_measure(lbmd, torch, drift_cycles=args.drift_cycles)
    if not args.no_adjoint:
        log("adjoint: 64^3 / 1000 particles, backward vs forward")
        out["adjoint"] = adjoint_measure(lbmd, torch)
    if not args.no_error_statement:
        log("error statement: FP32 vs FP64 run of the workload")
        out["error_statement"] = error_statement(lbmd, torch, cfg, x, v)
    if not args.no_cpu_baseline:
        log(f"cpu baseline: FP64 oracle on the full workload, {args.cpu_cycles} cycles")
        out["cpu_baseline"] = cpu_baseline(cfg, x, v, cycles=args.cpu_cycles)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
