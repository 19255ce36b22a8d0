"""The FP64 reference for gradients: the oracle's algorithm restated in
PyTorch (``oracle/torch_oracle.py``) and differentiated by torch.autograd.

Pinned to the C oracle twice: its forward trajectory must equal the C
oracle's (same steps, same noise), and its gradients must equal central
finite differences taken through the C oracle, an independent code path.
"""
import numpy as np
import pytest
import torch

from oracle.torch_oracle import TorchOracle

SHAPE = (6, 5, 4)
N = 6


def setup(orc, variant, kT, seed=3):
    c, w, e, b = orc.tables()
    rng = np.random.default_rng(seed)
    S = int(np.prod(SHAPE))
    f0 = w[:, None] * (1.0 + 0.02 * rng.standard_normal((19, S)))
    L = np.asarray(SHAPE, float)[:, None]
    x0 = rng.random((3, N)) * L
    v0 = 0.02 * rng.standard_normal((3, N))
    prm = dict(n_sub=3, variant=variant, kT=kT, seed=seed, n_particles=N, particle_mass=1.3,
               force_model=1)
    return f0, x0, v0, prm


def c_oracle_run(orc, f0, x0, v0, prm, gamma, nu, fext, cycles):
    o = orc.Oracle(*SHAPE, friction=gamma, nu=nu, f_ext=tuple(fext), **prm)
    o.set_populations(f0)
    o.set_particles(x0, v0)
    o.cycle(cycles)
    x, v, img = o.particles()
    return x + img * np.asarray(SHAPE, float)[:, None], v, o.populations()


@pytest.mark.parametrize("variant", [1, 2])
def test_torch_oracle_forward_equals_c_oracle(orc, variant):
    f0, x0, v0, prm = setup(orc, variant, 1e-3)
    gamma, nu, fext, cycles = 2.0, 0.2, np.array([1e-3, -2e-3, 5e-4]), 4
    xc, vc, fc = c_oracle_run(orc, f0, x0, v0, prm, gamma, nu, fext, cycles)
    T = TorchOracle(SHAPE, prm["n_sub"], variant, prm["kT"], seed=prm["seed"],
                    particle_mass=prm["particle_mass"])
    td = torch.float64
    xt, vt, ft = T.run(torch.tensor(f0, dtype=td), torch.tensor(x0, dtype=td),
                       torch.tensor(v0, dtype=td), torch.tensor(gamma, dtype=td),
                       torch.tensor(nu, dtype=td), torch.tensor(fext, dtype=td), cycles)
    assert np.abs(xt.numpy() - xc).max() < 1e-13
    assert np.abs(vt.numpy() - vc).max() < 1e-14
    assert np.abs(ft.numpy() - fc).max() < 1e-15


def loss_of(x, v, x0, a):
    """Drift along x plus a weighted sum of final velocities and the MSD."""
    d = x - x0
    return d[0].mean() + (a * v).sum() + (d * d).sum(0).mean()


@pytest.mark.parametrize("variant", [1, 2])
def test_torch_oracle_gradients_equal_c_oracle_fd(orc, variant):
    f0, x0, v0, prm = setup(orc, variant, 1e-3, seed=4)
    gamma, nu, fext, cycles = 2.0, 0.2, np.array([1e-3, -2e-3, 5e-4]), 4
    a = np.random.default_rng(9).standard_normal((3, N))
    td = torch.float64
    g = torch.tensor(gamma, dtype=td, requires_grad=True)
    n = torch.tensor(nu, dtype=td, requires_grad=True)
    fe = torch.tensor(fext, dtype=td, requires_grad=True)
    v0t = torch.tensor(v0, dtype=td, requires_grad=True)
    T = TorchOracle(SHAPE, prm["n_sub"], variant, prm["kT"], seed=prm["seed"],
                    particle_mass=prm["particle_mass"])
    x0t = torch.tensor(x0, dtype=td)
    xt, vt, _ = T.run(torch.tensor(f0, dtype=td), x0t, v0t, g, n, fe, cycles)
    loss_of(xt, vt, x0t, torch.tensor(a)).backward()

    def L(gamma_, nu_, fext_, v0_):
        x, v, _ = c_oracle_run(orc, f0, x0, v0_, prm, gamma_, nu_, fext_, cycles)
        return loss_of(x, v, x0, a)

    h = 1e-4
    fd = [(L(gamma + h, nu, fext, v0) - L(gamma - h, nu, fext, v0)) / (2 * h),
          (L(gamma, nu + h, fext, v0) - L(gamma, nu - h, fext, v0)) / (2 * h)]
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd.append((L(gamma, nu, fext + e, v0) - L(gamma, nu, fext - e, v0)) / (2 * h))
    ad = [g.grad.item(), n.grad.item()] + list(fe.grad.numpy())
    for k, (x, y) in enumerate(zip(ad, fd)):
        assert abs(x - y) <= 1e-6 * max(abs(y), 1e-3), (k, x, y)
    # two velocity components and one random direction
    for (d, p) in [(0, 1), (2, 4)]:
        e = np.zeros((3, N))
        e[d, p] = h
        fdv = (L(gamma, nu, fext, v0 + e) - L(gamma, nu, fext, v0 - e)) / (2 * h)
        assert abs(v0t.grad[d, p].item() - fdv) <= 1e-6 * max(abs(fdv), 1e-3)
    u = np.random.default_rng(2).standard_normal((3, N))
    u /= np.linalg.norm(u)
    fdu = (L(gamma, nu, fext, v0 + h * u) - L(gamma, nu, fext, v0 - h * u)) / (2 * h)
    assert abs((v0t.grad.numpy() * u).sum() - fdu) <= 1e-6 * max(abs(fdu), 1e-3)
