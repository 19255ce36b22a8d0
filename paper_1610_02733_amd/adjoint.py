"""Gradients of coupled LB/MD trajectories through the library's adjoint.

``coupled_run(gamma, nu, f_ext, x0, v0, shape=..., cycles=..., ...)`` runs
``cycles`` coupled cycles (n_sub MD steps + one LB step each; Sec. 3 of the
paper) of a particle suspension and returns the unwrapped particle positions
and the velocities at the end.  It is differentiable (``torch.autograd``)
with respect to the friction gamma (Eq. 4), the shear viscosity nu, the
constant force f_ext on every particle, and the initial positions and
velocities, along the noise realisation fixed by the seed.

The forward pass saves a state every ``checkpoint`` cycles.  The backward
pass walks the segments from last to first: it re-runs each segment from its
saved state with recording, then sweeps the recorded cycles backwards with
the library's adjoint kernels, which regenerate the noise from its counters.
Argument marshalling only: every step runs in ``liblbmd.so``.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lbmd


class _CoupledRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma, nu, f_ext, x0, v0, spec):
        kw = dict(spec["params"])
        kw.update(friction=float(gamma), nu=float(nu),
                  f_ext=tuple(float(t) for t in f_ext.detach().cpu().tolist()), force_model=1)
        shape = spec["shape"]
        N = x0.shape[1]
        sim = lbmd.Lattice(shape, n_particles=N, **kw)
        if spec.get("populations") is not None:
            sim.set_populations(spec["populations"])
        sim.bind_particles(x0.detach(), v0.detach())
        cycles, K = int(spec["cycles"]), int(spec["checkpoint"])
        states = []
        done = 0
        while done < cycles:
            k = min(K, cycles - done)
            states.append((sim.save_state(), k))
            if spec.get("graph", True):
                sim.run_cycles(k)
            else:
                sim.cycle(k)
            done += k
        L = torch.tensor(shape, dtype=torch.float64, device=sim.device).reshape(3, 1)
        x_end = sim.x + sim.img.to(torch.float64) * L
        ctx.sim, ctx.states, ctx.K = sim, states, K
        ctx.f_ext_shape = f_ext.shape
        return x_end.clone(), sim.v.clone()

    @staticmethod
    def backward(ctx, xbar, vbar):
        sim = ctx.sim
        if not hasattr(sim, "adj_ws"):
            sim.adjoint_attach(ctx.K)
        sim.adjoint_seed(xbar.to(torch.float64) if xbar is not None else None,
                         vbar.to(torch.float64) if vbar is not None else None)
        for state, k in reversed(ctx.states):
            sim.adjoint_record(state, k)
            sim.adjoint_sweep(k)
        xb0, vb0, g = sim.adjoint_result()
        dev = xb0.device
        gg = torch.tensor(g["gamma"], dtype=torch.float64, device=dev)
        gn = torch.tensor(g["nu"], dtype=torch.float64, device=dev)
        gf = torch.as_tensor(np.asarray(g["f_ext"]), dtype=torch.float64, device=dev)
        return gg, gn, gf.reshape(ctx.f_ext_shape), xb0, vb0, None


def coupled_run(gamma, nu, f_ext, x0, v0, *, shape, cycles, checkpoint=10, populations=None,
                graph=True, **params):
    """Differentiable coupled run; returns (x_unwrapped(T), v(T)), each [3, N].

    gamma, nu: 0-d tensors; f_ext: 3-vector tensor; x0, v0: [3, N] FP64 device
    tensors (positions inside the box).  ``params``: the remaining system
    parameters of ``lbmd.Lattice`` (n_sub, kT, rho0, seed, precision,
    variant, particle_mass, ...).  ``populations``: optional initial
    deviations [19, nsites].
    """
    spec = dict(shape=tuple(int(s) for s in shape), cycles=cycles, checkpoint=checkpoint,
                populations=populations, params=params, graph=graph)
    return _CoupledRun.apply(gamma, nu, f_ext, x0, v0, spec)
