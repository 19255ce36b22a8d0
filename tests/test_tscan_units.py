"""The temperature scan's map from the paper's Lennard-Jones units to
lattice units (CPU)."""
import math

from paper_1610_02733_amd.tscan import lattice_params


def test_lj_to_lattice_units():
    # n = 10, dt = 0.01 tau: tau_LB = 0.1 tau
    p = lattice_params(10, 0.01, 20.0)
    s = 0.1
    assert math.isclose(p["kT"], s * s)                 # eps = mu sigma^2 / tau^2
    assert math.isclose(p["nu"], 3.0 * s)               # eta / rho = 3 sigma^2 / tau
    assert math.isclose(p["friction"], 20.0 * s)        # zeta in mu / tau
    assert math.isclose(p["k_bond"], 30.0 * s * s)      # 30 eps / sigma^2
    assert math.isclose(p["wca_eps"], p["kT"]) and p["wca_sigma"] == 1.0
    assert p["force_model"] == 3 and p["r0_bond"] == 1.5           # FENE R0 = 1.5 sigma
    assert lattice_params(10, 0.01, 20.0, "wca")["force_model"] == 2
    # the dimensionless friction per MD step is unit-free: zeta dt = zeta_lat tau_MD / m
    assert math.isclose(p["friction"] * (1.0 / 10), 20.0 * 0.01)
