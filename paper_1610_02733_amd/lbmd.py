"""ctypes binding of the C ABI in ``include/lbmd.h``.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``liblbmd.so``.  PyTorch provides the device memory (workspace, particle
arrays) and the stream.  Importing this module on a machine without the
built library raises immediately: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmd.so")

OK, EINVAL, ESTATE, EHIP, ENOSPACE, ENONFINITE = 0, -1, -2, -3, -4, -5
NTOTALS = 15
TOT = dict(mass=0, pfluid=slice(1, 4), pseen=slice(4, 7), ppart=slice(7, 10), ke=10,
           u2=11, t_lb=12, t_md=13, tpart=14)
# D3Q19 weights in the library's velocity order (include/lbmd.h): rest,
# the 6 axis directions, the 12 face diagonals.
WEIGHTS = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("n_sub", C.c_int32), ("variant", C.c_int32), ("precision", C.c_int32),
        ("n_particles", C.c_int32), ("force_model", C.c_int32), ("chain_len", C.c_int32),
        ("replica", C.c_uint32), ("seed", C.c_uint64),
        ("rho0", C.c_double), ("nu", C.c_double), ("nu_bulk", C.c_double),
        ("gamma_ghost", C.c_double), ("kT", C.c_double), ("friction", C.c_double),
        ("particle_mass", C.c_double),
        ("body_force", C.c_double * 3), ("f_ext", C.c_double * 3),
        ("k_bond", C.c_double), ("r0_bond", C.c_double),
        ("wca_eps", C.c_double), ("wca_sigma", C.c_double),
        ("stencil", C.c_int32),
    ]


class LbmdError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {lib().lbmd_strerror(code).decode()} ({code})")
        self.code = code


_lib = None


def lib():
    """Load liblbmd.so (fails loudly if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_1610_02733_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.lbmd_workspace_bytes.argtypes = [C.POINTER(Params)]
        L.lbmd_workspace_bytes.restype = C.c_size_t
        L.lb_create.argtypes = [C.POINTER(Params), P, C.c_size_t, P, C.POINTER(P)]
        L.lb_destroy.argtypes = [P]
        L.lbmd_bind_particles.argtypes = [P, P, P, P]
        L.md_couple_substep.argtypes = [P]
        L.lb_step.argtypes = [P]
        L.lb_moments.argtypes = [P, P, P, P]
        L.lb_moments_noalloc.argtypes = [P, P, P, P]
        L.lbmd_get_populations.argtypes = [P, P]
        L.lbmd_set_populations.argtypes = [P, P]
        L.lbmd_get_transfer.argtypes = [P, P]
        L.lbmd_get_counters.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                        C.POINTER(C.c_int32)]
        L.lbmd_set_counters.argtypes = [P, C.c_int64, C.c_int64, C.c_int32]
        L.lbmd_strerror.argtypes = [C.c_int]
        L.lbmd_strerror.restype = C.c_char_p
        L.lbmd_run_cycles.argtypes = [P, C.c_int32]
        L.lbmd_batch_workspace_bytes.argtypes = [C.POINTER(Params), C.c_int32]
        L.lbmd_batch_workspace_bytes.restype = C.c_size_t
        L.lb_create_batch.argtypes = [C.POINTER(Params), C.c_int32, P, C.c_size_t, P, C.POINTER(P)]
        L.lbmd_replica_count.argtypes = [P]
        L.lbmd_batch_moments.argtypes = [P, P]
        L.lbmd_batch_get_populations.argtypes = [P, C.c_int32, P]
        L.lbmd_batch_set_populations.argtypes = [P, C.c_int32, P]
        L.lbmd_batch_get_transfer.argtypes = [P, C.c_int32, P]
        L.lbmd_autotune.argtypes = [P, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]
        L.lbmd_set_launch_shape.argtypes = [P, C.c_int32, C.c_int32, C.c_int32]
        L.lbmd_stream_copy.argtypes = [P, P, C.c_size_t, P]
        L.lbmd_stream_copy.restype = C.c_int
        L.lbmd_state_bytes.argtypes = [P]
        L.lbmd_state_bytes.restype = C.c_size_t
        L.lbmd_save_state.argtypes = [P, P]
        L.lbmd_load_state.argtypes = [P, P]
        L.lbmd_adjoint_workspace_bytes.argtypes = [P, C.c_int32]
        L.lbmd_adjoint_workspace_bytes.restype = C.c_size_t
        L.lbmd_adjoint_attach.argtypes = [P, P, C.c_size_t, C.c_int32]
        L.lbmd_adjoint_seed.argtypes = [P, P, P]
        L.lbmd_adjoint_record.argtypes = [P, P, C.c_int32]
        L.lb_step_adjoint.argtypes = [P]
        L.md_couple_substep_adjoint.argtypes = [P]
        L.lbmd_adjoint_result.argtypes = [P, P, P, P]
        L.lbmd_sort_particles.argtypes = [P, P]
        for n in ("lbmd_sort_particles", "lb_create", "lb_destroy", "lbmd_bind_particles", "md_couple_substep",
                  "lb_step", "lb_moments", "lb_moments_noalloc", "lbmd_get_populations",
                  "lbmd_set_populations",
                  "lbmd_get_transfer", "lbmd_get_counters", "lbmd_set_counters",
                  "lbmd_run_cycles", "lb_create_batch", "lbmd_replica_count",
                  "lbmd_batch_moments", "lbmd_batch_get_populations",
                  "lbmd_batch_set_populations", "lbmd_batch_get_transfer", "lbmd_autotune",
                  "lbmd_set_launch_shape",
                  "lbmd_save_state", "lbmd_load_state", "lbmd_adjoint_attach",
                  "lbmd_adjoint_seed", "lbmd_adjoint_record", "lb_step_adjoint",
                  "md_couple_substep_adjoint", "lbmd_adjoint_result"):
            getattr(L, n).restype = C.c_int
        _lib = L
    return _lib


DEFAULTS = dict(n_sub=1, variant=2, precision=32, n_particles=0, force_model=0, chain_len=1,
                replica=0, seed=0, rho0=1.0, nu=1.0 / 6.0, nu_bulk=-1.0, gamma_ghost=0.0,
                kT=0.0, friction=0.0, particle_mass=1.0, body_force=(0.0, 0.0, 0.0),
                f_ext=(0.0, 0.0, 0.0), k_bond=0.0, r0_bond=1.0, wca_eps=0.0, wca_sigma=1.0,
                stencil=0)


def stream_copy(dst, src, stream=None):
    """Device copy of src into dst (same byte size, 16-byte multiple) with the
    library's non-temporal streaming kernel (bandwidth calibration)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    _check(lib().lbmd_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()),
                                  nbytes, C.c_void_p(s.cuda_stream)), "lbmd_stream_copy")


def make_params(shape, **kw) -> Params:
    p = dict(DEFAULTS)
    unknown = set(kw) - set(p)
    if unknown:
        raise TypeError(f"unknown parameters {sorted(unknown)}")
    p.update(kw)
    s = Params()
    s.nx, s.ny, s.nz = (int(v) for v in shape)
    for k, v in p.items():
        if k in ("body_force", "f_ext"):
            setattr(s, k, (C.c_double * 3)(*[float(t) for t in v]))
        else:
            setattr(s, k, v)
    return s


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check(rc, what):
    if rc != OK:
        raise LbmdError(rc, what)
    return rc


class _System:
    """Common part of a single system and a batch of replicas."""

    def _create(self, params_array, nrep, device, stream, batch):
        self.device = torch.device(device)
        L = lib()
        if batch:
            nbytes = L.lbmd_batch_workspace_bytes(params_array, nrep)
        else:
            nbytes = L.lbmd_workspace_bytes(params_array)
        if nbytes == 0:
            raise LbmdError(EINVAL, "workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        sp = C.c_void_p(self.stream.cuda_stream)
        if batch:
            rc = L.lb_create_batch(params_array, nrep, _ptr(self.ws), nbytes, sp, C.byref(h))
        else:
            rc = L.lb_create(params_array, _ptr(self.ws), nbytes, sp, C.byref(h))
        _check(rc, "lb_create")
        self._h = h
        self.x = self.v = self.img = None

    def close(self):
        if getattr(self, "_h", None):
            lib().lb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def counters(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().lbmd_get_counters(self._h, C.byref(a), C.byref(b), C.byref(c)), "counters")
        return dict(t_lb=a.value, t_md=b.value, subs=c.value)

    def set_counters(self, t_lb, t_md, subs):
        _check(lib().lbmd_set_counters(self._h, t_lb, t_md, subs), "set_counters")

    def md_couple_substep(self):
        return _check(lib().md_couple_substep(self._h), "md_couple_substep")

    def lb_step(self):
        return _check(lib().lb_step(self._h), "lb_step")

    def cycle(self, ncycles=1):
        """Step-by-step cycles: n_sub MD steps, then one LB step."""
        L = lib()
        for _ in range(ncycles):
            if self.N > 0:
                for _ in range(self.n_sub):
                    rc = L.md_couple_substep(self._h)
                    if rc != OK:
                        raise LbmdError(rc, "md_couple_substep")
            rc = L.lb_step(self._h)
            if rc != OK:
                raise LbmdError(rc, "lb_step")

    def sort_particles(self):
        """Reorder the bound particles spatially (Morton order of 4^3-site
        tiles, per replica) in place; returns the permutation (new index t
        holds old particle perm[t])."""
        perm = torch.empty(max(self.N, 1), dtype=torch.int32, device=self.device)
        _check(lib().lbmd_sort_particles(self._h, _ptr(perm)), "lbmd_sort_particles")
        return perm[: self.N]

    def run_cycles(self, ncycles=1):
        """The same cycles replayed from one captured HIP graph."""
        return _check(lib().lbmd_run_cycles(self._h, int(ncycles)), "lbmd_run_cycles")

    def save_state(self, out=None):
        """Checkpoint at an LB-step boundary into a device byte tensor."""
        n = lib().lbmd_state_bytes(self._h)
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=self.device)
        elif out.numel() < n:
            raise LbmdError(ENOSPACE, "lbmd_save_state")
        _check(lib().lbmd_save_state(self._h, _ptr(out)), "lbmd_save_state")
        return out

    def load_state(self, state):
        _check(lib().lbmd_load_state(self._h, _ptr(state)), "lbmd_load_state")

    def set_launch_shape(self, lb_blocks=0, part_blocks=0, couple_lanes=0):
        _check(lib().lbmd_set_launch_shape(self._h, lb_blocks, part_blocks, couple_lanes),
               "lbmd_set_launch_shape")

    def autotune(self, cache_path=None):
        """Time the launch shapes of the hot kernels on this system and keep
        the fastest (grids: 0 = one block per work item; lanes: 0 = the
        built-in default)."""
        a, b, l = C.c_int32(), C.c_int32(), C.c_int32()
        path = cache_path.encode() if cache_path else None
        _check(lib().lbmd_autotune(self._h, path, C.byref(a), C.byref(b), C.byref(l)),
               "lbmd_autotune")
        return dict(lb_blocks=a.value, part_blocks=b.value, couple_lanes=l.value)


class Lattice(_System):
    """One LB/MD system on one GPU: a periodic lattice plus N particles.

    >>> sim = Lattice((64, 64, 64), precision=32, n_sub=5, kT=1e-4, ...)
    >>> sim.bind_particles(x, v)          # [3, N] arrays (FP64 on the device)
    >>> sim.run_cycles(100)               # 100 x (n_sub MD steps + one LB step)
    """

    def __init__(self, shape, device="cuda", stream=None, **kw):
        self.shape = tuple(int(v) for v in shape)
        self.nsites = int(np.prod(self.shape))
        self.params = make_params(self.shape, **kw)
        self.kw = dict(DEFAULTS, **kw)
        self.dtype = torch.float32 if self.params.precision == 32 else torch.float64
        self.N = self.params.n_particles
        self.n_sub = self.params.n_sub
        self._create(C.byref(self.params), 1, device, stream, batch=False)

    def bind_particles(self, x, v, img=None):
        """Copies x, v (and img) into arrays owned by this object, which the
        library then advances in place (self.x, self.v, self.img)."""
        N = self.N
        f64 = torch.float64  # particle state is FP64 in both lattice precisions
        # the arrays bound so far stay alive until the library is done with
        # them: binding in mid-interval reads them (lbmd_bind_particles)
        previous = (getattr(self, "x", None), getattr(self, "v", None), getattr(self, "img", None))
        self.x = torch.as_tensor(x, dtype=f64, device=self.device).reshape(3, N).clone()
        self.v = torch.as_tensor(v, dtype=f64, device=self.device).reshape(3, N).clone()
        if img is None:
            self.img = torch.zeros((3, N), dtype=torch.int32, device=self.device)
        else:
            self.img = torch.as_tensor(img, dtype=torch.int32, device=self.device).reshape(3, N).clone()
        _check(lib().lbmd_bind_particles(self._h, _ptr(self.x), _ptr(self.v), _ptr(self.img)),
               "lbmd_bind_particles")
        self.stream.synchronize()
        del previous

    def populations(self):
        out = torch.empty((19, self.nsites), dtype=self.dtype, device=self.device)
        _check(lib().lbmd_get_populations(self._h, _ptr(out)), "lbmd_get_populations")
        return out

    def set_populations(self, dev):
        t = torch.as_tensor(dev, dtype=self.dtype, device=self.device).reshape(19, self.nsites).contiguous()
        _check(lib().lbmd_set_populations(self._h, _ptr(t)), "lbmd_set_populations")
        torch.cuda.current_stream(self.device).synchronize()

    def transfer(self):
        out = torch.empty((3, self.nsites), dtype=self.dtype, device=self.device)
        _check(lib().lbmd_get_transfer(self._h, _ptr(out)), "lbmd_get_transfer")
        return out

    def moments(self, fields=False, allow_nonfinite=False, noalloc=False):
        """Totals (LBMD_TOT_* layout) and optionally the density and velocity
        fields; noalloc=True calls lb_moments_noalloc (reduction scratch in
        the library's fixed device array instead of the workspace)."""
        tot = np.zeros(NTOTALS)
        rho = u = None
        if fields:
            rho = torch.empty(self.nsites, dtype=self.dtype, device=self.device)
            u = torch.empty((3, self.nsites), dtype=self.dtype, device=self.device)
        fn = lib().lb_moments_noalloc if noalloc else lib().lb_moments
        rc = fn(self._h, _ptr(rho), _ptr(u), tot.ctypes.data_as(C.c_void_p))
        if rc != OK and not (allow_nonfinite and rc == ENONFINITE):
            raise LbmdError(rc, "lb_moments_noalloc" if noalloc else "lb_moments")
        return (tot, rho, u) if fields else tot


    # -- reverse mode ---------------------------------------------------------
    def adjoint_attach(self, seg_cycles):
        n = lib().lbmd_adjoint_workspace_bytes(self._h, int(seg_cycles))
        if n == 0:
            raise LbmdError(EINVAL, "lbmd_adjoint_workspace_bytes")
        self.adj_ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().lbmd_adjoint_attach(self._h, _ptr(self.adj_ws), n, int(seg_cycles)),
               "lbmd_adjoint_attach")

    def adjoint_seed(self, xbar=None, vbar=None):
        f64 = torch.float64
        xb = None if xbar is None else torch.as_tensor(xbar, dtype=f64, device=self.device).reshape(3, self.N).contiguous()
        vb = None if vbar is None else torch.as_tensor(vbar, dtype=f64, device=self.device).reshape(3, self.N).contiguous()
        _check(lib().lbmd_adjoint_seed(self._h, _ptr(xb), _ptr(vb)), "lbmd_adjoint_seed")
        torch.cuda.current_stream(self.device).synchronize()  # xb, vb may be freed

    def adjoint_record(self, state, ncycles):
        _check(lib().lbmd_adjoint_record(self._h, _ptr(state), int(ncycles)), "lbmd_adjoint_record")

    def lb_step_adjoint(self):
        return _check(lib().lb_step_adjoint(self._h), "lb_step_adjoint")

    def md_couple_substep_adjoint(self):
        return _check(lib().md_couple_substep_adjoint(self._h), "md_couple_substep_adjoint")

    def adjoint_sweep(self, ncycles):
        """Reverse of the last `ncycles` recorded cycles."""
        L = lib()
        for _ in range(ncycles):
            rc = L.lb_step_adjoint(self._h)
            if rc != OK:
                raise LbmdError(rc, "lb_step_adjoint")
            if self.N > 0:
                for _ in range(self.n_sub):
                    rc = L.md_couple_substep_adjoint(self._h)
                    if rc != OK:
                        raise LbmdError(rc, "md_couple_substep_adjoint")

    def adjoint_result(self):
        """(dL/dx0 [3, N], dL/dv0 [3, N], grads) with grads = dict(gamma, nu, f_ext[3])."""
        xb = torch.empty((3, self.N), dtype=torch.float64, device=self.device)
        vb = torch.empty((3, self.N), dtype=torch.float64, device=self.device)
        g = np.zeros(5)
        _check(lib().lbmd_adjoint_result(self._h, _ptr(xb), _ptr(vb), g.ctypes.data_as(C.c_void_p)),
               "lbmd_adjoint_result")
        return xb, vb, dict(gamma=g[0], nu=g[1], f_ext=g[2:5].copy())


class Batch(_System):
    """Independent replicas of uneven box and particle counts advanced in
    lockstep by one launch per phase.  per_rep: list of (shape, kwargs)."""

    def __init__(self, per_rep, device="cuda", stream=None):
        self.R = len(per_rep)
        arr = (Params * self.R)()
        self.shapes, self.Ns = [], []
        for r, (shape, kw) in enumerate(per_rep):
            arr[r] = make_params(shape, **kw)
            self.shapes.append(tuple(int(v) for v in shape))
            self.Ns.append(arr[r].n_particles)
        self.params = arr
        self.dtype = torch.float32 if arr[0].precision == 32 else torch.float64
        self.N = int(sum(self.Ns))
        self.n_sub = arr[0].n_sub
        self.offsets = np.concatenate([[0], np.cumsum(self.Ns)]).astype(int)
        self._create(arr, self.R, device, stream, batch=True)

    def bind_particles(self, xs, vs):
        """xs, vs: lists of [3, N_r] arrays (replica order)."""
        f64 = torch.float64
        x = np.concatenate([np.asarray(a, np.float64).reshape(3, -1) for a in xs], 1)
        v = np.concatenate([np.asarray(a, np.float64).reshape(3, -1) for a in vs], 1)
        previous = (getattr(self, "x", None), getattr(self, "v", None), getattr(self, "img", None))
        self.x = torch.as_tensor(x, dtype=f64, device=self.device).clone()
        self.v = torch.as_tensor(v, dtype=f64, device=self.device).clone()
        self.img = torch.zeros((3, self.N), dtype=torch.int32, device=self.device)
        _check(lib().lbmd_bind_particles(self._h, _ptr(self.x), _ptr(self.v), _ptr(self.img)),
               "lbmd_bind_particles")
        self.stream.synchronize()  # (the arrays bound so far: lbmd_bind_particles)
        del previous

    def particles(self, rep):
        a, b = self.offsets[rep], self.offsets[rep + 1]
        return self.x[:, a:b], self.v[:, a:b], self.img[:, a:b]

    def populations(self, rep):
        S = int(np.prod(self.shapes[rep]))
        out = torch.empty((19, S), dtype=self.dtype, device=self.device)
        _check(lib().lbmd_batch_get_populations(self._h, rep, _ptr(out)), "batch_get_populations")
        return out

    def temperatures(self):
        """Particle temperature T_p of every replica (the library's
        LBMD_TOT_TPART) in units of its kT; NaN for a replica without
        particles, with kT = 0, or whose particles went non-finite."""
        tp = self.moments()[:, TOT["tpart"]]
        kT = np.array([self.params[r].kT for r in range(self.R)])
        ok = (np.asarray(self.Ns) > 0) & (kT > 0)
        return np.where(ok, tp / np.where(ok, kT, 1.0), np.nan)

    def moments(self, allow_nonfinite=True):
        tot = np.zeros((self.R, NTOTALS))
        rc = lib().lbmd_batch_moments(self._h, tot.ctypes.data_as(C.c_void_p))
        if rc != OK and not (allow_nonfinite and rc == ENONFINITE):
            raise LbmdError(rc, "lbmd_batch_moments")
        return tot
