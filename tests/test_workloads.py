"""Host-side checks of the seeded input generators (no GPU): the placements
that the named workloads use have the properties their docstrings state."""
import numpy as np
from scipy.spatial import cKDTree

from paper_1610_02733_amd import workloads as wl


def test_separated_particles_keep_their_distance():
    shape = (20, 16, 12)
    x, v = wl.separated_particles(shape, 400, 1e-3, 2.0, seed=5, min_dist=1.5)
    assert x.shape == (3, 400) and v.shape == (3, 400)
    L = np.asarray(shape, float)
    assert (x >= 0).all() and (x < L[:, None]).all()
    # minimum-image distances, brute force
    d = x[:, :, None] - x[:, None, :]
    d -= L[:, None, None] * np.round(d / L[:, None, None])
    r = np.sqrt((d ** 2).sum(0))
    np.fill_diagonal(r, np.inf)
    assert r.min() >= 1.5
    # Maxwell velocities at kT / m
    assert abs(v.var() / (1e-3 / 2.0) - 1.0) < 0.15
    # seeded: the same draw again
    x2, v2 = wl.separated_particles(shape, 400, 1e-3, 2.0, seed=5, min_dist=1.5)
    assert (x2 == x).all() and (v2 == v).all()


def test_scale_workload_has_no_close_pairs():
    """The 256^3 workload: 1e5 particles, none closer than 2 sites (so no two
    share a lattice cube), positions uniform on average."""
    cfg = wl.CONFIGS["c3"]
    x, v = wl.workload_particles(cfg)
    assert x.shape == (3, cfg["n_particles"])
    L = float(cfg["shape"][0])
    assert len(cKDTree(x.T, boxsize=L).query_pairs(cfg["min_dist"])) == 0
    cubes = np.floor(x).astype(np.int64)
    key = cubes[0] + 256 * (cubes[1] + 256 * cubes[2])
    assert len(np.unique(key)) == cfg["n_particles"]
    # homogeneous: particle counts of the 8 octants within 2% of each other
    octant = (x[0] >= L / 2).astype(int) + 2 * (x[1] >= L / 2) + 4 * (x[2] >= L / 2)
    counts = np.bincount(octant, minlength=8)
    assert counts.min() > 0.98 * counts.mean() and counts.max() < 1.02 * counts.mean()


def test_workload_particles_dispatch():
    """Chains for the polymer workloads, uniform free particles where no
    minimum distance is set."""
    c1 = wl.CONFIGS["c1"]
    x, v = wl.workload_particles(c1)
    xf, vf = wl.free_particles(c1["shape"], c1["n_particles"], c1["kT"], c1["particle_mass"],
                               c1["seed"])
    assert (x == xf).all() and (v == vf).all()
    c2p = dict(wl.CONFIGS["c2p"], n_particles=100, chain_len=10)
    x, v = wl.workload_particles(c2p)
    L = np.asarray(c2p["shape"], float)[:, None]
    d = x[:, 1:] - x[:, :-1]
    d -= L * np.round(d / L)
    bonded = np.ones(99, bool)
    bonded[9::10] = False  # chain ends
    assert np.allclose(np.sqrt((d[:, bonded] ** 2).sum(0)), 1.0)
