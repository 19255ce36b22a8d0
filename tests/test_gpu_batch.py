"""Batched replicas, captured cycles and the autotuner, through the C ABI.

A replica of a batch must reproduce the single system with the same
parameters (same seed and replica id, hence the same noise) up to the order
of floating-point sums; captured cycles must reproduce step-by-step calls;
autotuning must leave the state unchanged.
"""
import json
import os

import numpy as np
import pytest

from paper_1610_02733_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_02733_amd import lbmd
    lbmd.lib()
    return lbmd


def rel_pop(a, b, w, rho0):
    return float((np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))
                  / (w[:, None] * rho0)).max())


@pytest.mark.parametrize("variant", [1, 2])
def test_run_cycles_equals_stepwise(lb, orc, variant):
    c, w, e, b = orc.tables()
    shape = (16, 12, 10)
    x, v = wl.free_particles(shape, 50, 1e-3, 1.0, 4)
    kw = dict(precision=64, n_sub=5, variant=variant, kT=1e-3, seed=3, n_particles=50,
              friction=1.0)
    a = lb.Lattice(shape, **kw)
    a.bind_particles(x, v)
    a.cycle(12)
    g = lb.Lattice(shape, **kw)
    g.bind_particles(x, v)
    g.run_cycles(5)
    g.cycle(2)   # mixing both paths keeps the clock consistent
    g.run_cycles(5)
    assert g.counters() == a.counters()
    assert rel_pop(a.populations().cpu(), g.populations().cpu(), w, 1.0) < 1e-13
    assert np.abs(a.x.cpu().numpy() - g.x.cpu().numpy()).max() < 1e-12
    assert np.abs(a.v.cpu().numpy() - g.v.cpu().numpy()).max() < 1e-14
    # and against the oracle
    o = orc.Oracle(*shape, **{k: v_ for k, v_ in kw.items() if k != "precision"})
    o.set_particles(x, v)
    o.cycle(12)
    assert rel_pop(g.populations().cpu().numpy() + w[:, None], o.populations(), w, 1.0) < 1e-12


def make_replicas(nrep, prec, variant, seed=11, stencil=0):
    rng = np.random.default_rng(seed)
    reps, xs, vs = [], [], []
    for r in range(nrep):
        e = int(rng.choice([6, 8, 10, 12]))
        shape = (e, e + (r % 3), max(4, e - 2))
        n = int(rng.integers(0, 40)) if r != 1 else 0  # one replica without particles
        kw = dict(precision=prec, n_sub=4, variant=variant, kT=1e-3, seed=7 + r, replica=r,
                  n_particles=n, friction=float(rng.uniform(0.5, 3.0)),
                  nu=float(rng.uniform(0.1, 0.5)), stencil=stencil)
        x, v = wl.free_particles(shape, n, 1e-3, 1.0, 100 + r)
        reps.append((shape, kw))
        xs.append(x)
        vs.append(v)
    return reps, xs, vs


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("variant", [1, 2])
def test_batch_replicas_match_single_runs(lb, orc, prec, variant):
    c, w, e, b = orc.tables()
    reps, xs, vs = make_replicas(7, prec, variant)
    B = lb.Batch(reps)
    B.bind_particles(xs, vs)
    B.run_cycles(6)
    B.cycle(2)
    tol = 1e-12 if prec == 64 else 2e-6
    tot = B.moments()
    for r, (shape, kw) in enumerate(reps):
        s = lb.Lattice(shape, **kw)
        if kw["n_particles"] > 0:
            s.bind_particles(xs[r], vs[r])
        s.cycle(8)
        assert rel_pop(B.populations(r).cpu(), s.populations().cpu(), w, 1.0) < tol, r
        if kw["n_particles"] > 0:
            bx, bv, bi = B.particles(r)
            ptol = 1e-10 if prec == 64 else 1e-6  # FP32 transfer sums reorder
            assert np.abs(bx.cpu().numpy() - s.x.cpu().numpy()).max() < ptol
            assert np.abs(bv.cpu().numpy() - s.v.cpu().numpy()).max() < ptol
        ts = s.moments()
        mtol = 1e-9 if prec == 64 else 1e-6
        assert abs(tot[r, 0] - ts[0]) < mtol * ts[0]
        # particle momentum: a sum that cancels, compared on the scale of its
        # terms; kinetic energy relative to itself
        pscale = kw.get("particle_mass", 1.0) * np.abs(s.v.cpu().numpy()).sum(1) + 1e-300 \
            if kw["n_particles"] > 0 else np.ones(3)
        assert (np.abs(tot[r, 7:10] - ts[7:10]) <= mtol * pscale + 1e-15).all(), r
        assert abs(tot[r, 10] - ts[10]) <= mtol * abs(ts[10]) + 1e-15, r


@pytest.mark.parametrize("variant,stencil", [(2, 0), (3, 0), (2, 1)])
def test_batch_replicas_match_oracle(lb, orc, variant, stencil):
    c, w, e, b = orc.tables()
    reps, xs, vs = make_replicas(4, 64, variant, seed=5, stencil=stencil)
    B = lb.Batch(reps)
    B.bind_particles(xs, vs)
    B.run_cycles(5)
    for r, (shape, kw) in enumerate(reps):
        o = orc.Oracle(*shape, **{k: v for k, v in kw.items() if k != "precision"})
        if kw["n_particles"] > 0:
            o.set_particles(xs[r], vs[r])
        o.cycle(5)
        assert rel_pop(B.populations(r).cpu().numpy() + w[:, None], o.populations(), w, 1.0) < 1e-12
        if kw["n_particles"] > 0:
            assert np.abs(B.particles(r)[1].cpu().numpy() - o.particles()[1]).max() < 1e-12


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_batch_mixed_force_models_match_oracle(lb, orc, variant):
    """Replicas with different force models in one batch (Kremer-Grest
    chains, harmonic + WCA chains, free particles, a uniform external force):
    the coupling kernel bins only the bead-spring replicas, and the after-step
    work of variants 2 and 3 rides in the force kernel's launch.  Every
    replica must equal its own oracle run (FP64)."""
    c, w, e, b = orc.tables()
    common = dict(precision=64, n_sub=10, variant=variant)
    reps, xs, vs = [], [], []
    x, v = wl.chains((20, 20, 20), 12, 10, 0.01, 1.0, seed=33, bond=0.97, min_dist=0.95)
    reps.append(((20, 20, 20), dict(common, kT=0.01, nu=0.3, seed=9, replica=0, n_particles=120,
                                    friction=2.0, force_model=3, chain_len=10, k_bond=0.3,
                                    r0_bond=1.5, wca_eps=0.01, wca_sigma=1.0)))
    xs.append(x)
    vs.append(v)
    x, v = wl.chains((16, 16, 12), 6, 8, 1e-3, 1.0, seed=34, bond=0.97, min_dist=0.95)
    reps.append(((16, 16, 12), dict(common, kT=1e-3, seed=10, replica=1, n_particles=48,
                                    friction=1.0, force_model=2, chain_len=8, k_bond=0.3,
                                    r0_bond=1.0, wca_eps=0.01, wca_sigma=1.0)))
    xs.append(x)
    vs.append(v)
    x, v = wl.free_particles((10, 12, 8), 25, 1e-3, 1.0, 35)
    reps.append(((10, 12, 8), dict(common, kT=1e-3, seed=11, replica=2, n_particles=25,
                                   friction=1.5)))
    xs.append(x)
    vs.append(v)
    x, v = wl.free_particles((8, 8, 8), 10, 1e-3, 1.0, 36)
    reps.append(((8, 8, 8), dict(common, kT=1e-3, seed=12, replica=3, n_particles=10,
                                 friction=0.5, force_model=1, f_ext=(1e-3, -2e-3, 5e-4))))
    xs.append(x)
    vs.append(v)
    B = lb.Batch(reps)
    B.bind_particles(xs, vs)
    B.run_cycles(5)
    for r, (shape, kw) in enumerate(reps):
        o = orc.Oracle(*shape, **{k: v for k, v in kw.items() if k != "precision"})
        o.set_particles(xs[r], vs[r])
        o.cycle(5)
        assert rel_pop(B.populations(r).cpu().numpy() + w[:, None], o.populations(), w, 1.0) < 1e-12, r
        assert np.abs(B.particles(r)[1].cpu().numpy() - o.particles()[1]).max() < 1e-11, r


def test_batch_nonfinite_replica_is_isolated(lb, orc):
    c, w, e, b = orc.tables()
    reps, xs, vs = make_replicas(5, 64, 2, seed=9)
    for r in range(5):
        reps[r][1]["n_particles"] = 10
        xs[r], vs[r] = wl.free_particles(reps[r][0], 10, 1e-3, 1.0, 50 + r)
    xs[2] = xs[2].copy()
    xs[2][0, 3] = np.nan
    B = lb.Batch(reps)
    B.bind_particles(xs, vs)
    B.run_cycles(4)
    tot = B.moments(allow_nonfinite=True)
    assert np.isfinite(tot[:, :12]).all()
    for r in (0, 4):
        s = lb.Lattice(reps[r][0], **reps[r][1])
        s.bind_particles(xs[r], vs[r])
        s.cycle(4)
        assert rel_pop(B.populations(r).cpu(), s.populations().cpu(), w, 1.0) < 1e-12


def test_autotune_leaves_state_and_caches(lb, orc, tmp_path):
    c, w, e, b = orc.tables()
    shape = (24, 20, 16)
    x, v = wl.free_particles(shape, 300, 1e-3, 1.0, 6)
    kw = dict(precision=32, n_sub=5, variant=2, kT=1e-3, seed=2, n_particles=300, friction=1.0)
    a = lb.Lattice(shape, **kw)
    a.bind_particles(x, v)
    a.run_cycles(3)
    t = lb.Lattice(shape, **kw)
    t.bind_particles(x, v)
    t.run_cycles(3)
    path = str(tmp_path / "tune.json")
    first = t.autotune(path)
    assert os.path.exists(path)
    cache = json.load(open(path))
    assert len(cache) == 1 and list(cache.values())[0] == [
        first["lb_blocks"], first["part_blocks"], first["couple_lanes"]]
    assert first["couple_lanes"] in (2, 4, 8)  # timed, so a candidate is picked
    assert t.autotune(path) == first  # served from the cache
    a.run_cycles(4)
    t.run_cycles(4)
    # FP32 run: the two systems differ only by the order of transfer sums
    assert rel_pop(a.populations().cpu(), t.populations().cpu(), w, 1.0) < 2e-6
    assert np.abs(a.x.cpu().numpy() - t.x.cpu().numpy()).max() < 1e-6


def test_run_cycles_requires_boundary(lb):
    shape = (8, 8, 8)
    x, v = wl.free_particles(shape, 4, 0.0, 1.0, 1)
    g = lb.Lattice(shape, precision=64, n_sub=3, n_particles=4, friction=1.0)
    with pytest.raises(lb.LbmdError):
        g.run_cycles(1)  # particles not bound
    g.bind_particles(x, v)
    g.md_couple_substep()
    assert lb.lib().lbmd_run_cycles(g._h, 1) == lb.ESTATE
    g.md_couple_substep()
    g.md_couple_substep()
    g.lb_step()
    g.run_cycles(2)
    assert g.counters() == dict(t_lb=3, t_md=9, subs=0)


def test_batch_sort_keeps_replica_ranges(lb, orc):
    """Sorting a batch reorders particles inside each replica only, and the
    reordered batch still equals the oracle's unsorted run, slot for
    particle."""
    c, w, e, b = orc.tables()
    reps, xs, vs = make_replicas(4, 64, 2, seed=8)
    B = lb.Batch(reps)
    B.bind_particles(xs, vs)
    perm = B.sort_particles().cpu().numpy()
    off = B.offsets
    refs = []
    for r, (shape, kw) in enumerate(reps):
        # expected order inside the replica: stable sort of the Z-order keys
        # of the 4^3-site tiles, written out from the definition
        t = (np.floor(xs[r]).astype(np.int64) % np.asarray(shape)[:, None]) >> 2
        key = np.zeros(t.shape[1], np.int64)
        for bit in range(12):
            for d in range(3):
                key |= ((t[d] >> bit) & 1) << (3 * bit + d)
        refs.append(np.argsort(key, kind="stable"))
        assert (perm[off[r]:off[r + 1]] - off[r] == refs[r]).all()
    B.run_cycles(4)
    for r, (shape, kw) in enumerate(reps):
        # the particles keep their identities (and noise): the oracle runs unsorted
        o = orc.Oracle(*shape, **{k: v for k, v in kw.items() if k != "precision"})
        if kw["n_particles"] > 0:
            o.set_particles(xs[r], vs[r])
        o.cycle(4)
        assert rel_pop(B.populations(r).cpu().numpy() + w[:, None], o.populations(), w, 1.0) < 1e-12
        if kw["n_particles"] > 0:
            assert np.abs(B.particles(r)[1].cpu().numpy() - o.particles()[1][:, refs[r]]).max() < 1e-12


@pytest.mark.parametrize("prec", [64, 32])
def test_batch_mixing_row_and_general_lattices(lb, orc, prec):
    """A batch whose replicas take different collide-stream paths (x rows of
    64 and 128 sites on the row path, 10 and 12 on the general one): every
    replica equals its own oracle run, populations and particles."""
    c, w, e, b = orc.tables()
    shapes = [(64, 3, 2), (10, 8, 6), (128, 2, 3), (12, 5, 4)]
    reps, xs, vs, orcs = [], [], [], []
    for r, shape in enumerate(shapes):
        n = 6 + 5 * r
        kw = dict(n_sub=3, variant=2, kT=1e-3, seed=41, replica=r, n_particles=n,
                  friction=1.0 + 0.5 * r, nu=0.2 + 0.05 * r)
        x, v = wl.free_particles(shape, n, 1e-3, 1.0, 50 + r)
        reps.append((shape, dict(precision=prec, **kw)))
        xs.append(x)
        vs.append(v)
        o = orc.Oracle(*shape, **kw)
        o.set_particles(x, v)
        o.cycle(6)
        orcs.append(o)
    B = lb.Batch(reps)
    B.bind_particles(xs, vs)
    B.cycle(3)
    B.run_cycles(3)
    tol = 1e-12 if prec == 64 else 1e-5
    for r, o in enumerate(orcs):
        err = rel_pop(B.populations(r).cpu().numpy() + w[:, None], o.populations(), w, 1.0)
        assert err < tol, (r, err)
        xg, vg, ig = (t.cpu().numpy() for t in B.particles(r))
        xo, vo, io = o.particles()
        L = np.asarray(shapes[r], float)[:, None]
        assert np.abs((xg + L * ig) - (xo + L * io)).max() < tol * max(shapes[r])
        assert np.abs(vg - vo).max() < tol * max(np.abs(vo).max(), np.sqrt(1e-3))
