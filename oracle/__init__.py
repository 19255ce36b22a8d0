"""FP64 CPU oracle of the fluctuating D3Q19 LB fluid with dissipative particle
coupling (Tretyakov & Duenweg, arXiv:1610.02733, Sec. 2-3).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP implementation in ``paper_1610_02733_amd``; both are fed the
same seeded inputs by the tests.

The arithmetic lives in ``lbmd_oracle.c`` (plain C, FP64; its site and
particle loops run on OpenMP threads with results independent of the thread
count); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbmd_oracle.c")
_LIB = os.path.join(_HERE, "liblbmd_oracle.so")

Q = 19
NTOTALS = 15


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction,
    OpenMP for the parallel loops)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("n_sub", C.c_int32), ("variant", C.c_int32), ("n_particles", C.c_int32),
        ("force_model", C.c_int32), ("chain_len", C.c_int32),
        ("replica", C.c_uint32), ("stencil", C.c_int32),
        ("seed", C.c_uint64),
        ("rho0", C.c_double), ("nu", C.c_double), ("nu_bulk", C.c_double),
        ("gamma_ghost", C.c_double), ("kT", C.c_double), ("friction", C.c_double),
        ("particle_mass", C.c_double),
        ("body_force", C.c_double * 3), ("f_ext", C.c_double * 3),
        ("k_bond", C.c_double), ("r0_bond", C.c_double),
        ("wca_eps", C.c_double), ("wca_sigma", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        lp = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        up = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.orc_tables.argtypes = [ip, dp, dp, dp]
        L.orc_philox4x32_10.argtypes = [up, up, up]
        L.orc_fluid_variates.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, dp]
        L.orc_particle_variates.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, dp]
        L.orc_create.argtypes = [C.POINTER(OrcParams), C.POINTER(P)]
        L.orc_destroy.argtypes = [P]
        L.orc_set_particles.argtypes = [P, dp, dp, C.c_void_p]
        L.orc_get_particles.argtypes = [P, dp, dp, ip]
        L.orc_set_populations.argtypes = [P, dp]
        L.orc_get_populations.argtypes = [P, dp]
        L.orc_get_J.argtypes = [P, dp]
        L.orc_set_J.argtypes = [P, dp]
        L.orc_counters.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.orc_set_counters.argtypes = [P, C.c_int64, C.c_int64, C.c_int32]
        L.orc_lb_step.argtypes = [P]
        L.orc_md_couple_substep.argtypes = [P]
        L.orc_lb_step_sampled.argtypes = [P, C.c_int64, lp, dp]
        L.orc_collide_site.argtypes = [P, C.c_int64, C.c_int64, dp, dp, dp]
        L.orc_cube_weights.argtypes = [P, dp, lp, dp]
        L.orc_stencil3_weights.argtypes = [P, dp, lp, dp]
        L.orc_moments.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_max_threads.restype = C.c_int32
        for name in ("orc_create", "orc_set_particles", "orc_get_particles",
                     "orc_set_populations", "orc_get_populations", "orc_get_J",
                     "orc_set_J", "orc_lb_step", "orc_md_couple_substep",
                     "orc_lb_step_sampled", "orc_collide_site", "orc_moments"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def tables():
    """D3Q19 velocities c[19,3], weights w[19], mode matrix e[19,19] (e[k,i] =
    e_k(c_i)) and norms b[19] exactly as the oracle uses them."""
    c = np.zeros(57, np.int32)
    w = np.zeros(19)
    e = np.zeros(361)
    b = np.zeros(19)
    lib().orc_tables(c, w, e, b)
    return c.reshape(19, 3), w, e.reshape(19, 19), b


def set_threads(n):
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def max_threads():
    return int(lib().orc_max_threads())


def philox4x32_10(counter, key):
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.asarray(counter, np.uint32), np.asarray(key, np.uint32), out)
    return out


def fluid_variates(seed, replica, site, step):
    out = np.zeros(15)
    lib().orc_fluid_variates(seed, replica, site, step, out)
    return out


def particle_variates(seed, replica, particle, step):
    out = np.zeros(3)
    lib().orc_particle_variates(seed, replica, particle, step, out)
    return out


_PARAM_DEFAULTS = dict(nu_bulk=-1.0, gamma_ghost=0.0, kT=0.0, friction=0.0,
                       particle_mass=1.0, body_force=(0.0, 0.0, 0.0),
                       f_ext=(0.0, 0.0, 0.0), k_bond=0.0, r0_bond=1.0,
                       wca_eps=0.0, wca_sigma=1.0, force_model=0, chain_len=1,
                       replica=0, seed=0, n_particles=0, variant=2, n_sub=1, stencil=0,
                       rho0=1.0, nu=1.0 / 6.0)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} returned {rc}")


class Oracle:
    """One oracle system: a periodic nx*ny*nz lattice plus N point particles.

    Call pattern (the paper's schedule, Sec. 3): repeat { n x
    md_couple_substep(); lb_step() }.
    """

    def __init__(self, nx, ny, nz, **kw):
        p = dict(_PARAM_DEFAULTS)
        p.update(kw)
        self.prm = p
        self.shape = (nx, ny, nz)
        self.nsites = nx * ny * nz
        s = OrcParams()
        s.nx, s.ny, s.nz = nx, ny, nz
        for k, v in p.items():
            if k in ("body_force", "f_ext"):
                setattr(s, k, (C.c_double * 3)(*v))
            else:
                setattr(s, k, v)
        self._p = s
        h = C.c_void_p()
        _check(lib().orc_create(C.byref(s), C.byref(h)), "orc_create")
        self._h = h
        self.N = p["n_particles"]

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # state ---------------------------------------------------------------
    def set_particles(self, x, v, img=None):
        x = np.ascontiguousarray(x, np.float64).reshape(3, self.N)
        v = np.ascontiguousarray(v, np.float64).reshape(3, self.N)
        ip = None
        if img is not None:
            img = np.ascontiguousarray(img, np.int32).reshape(3, self.N)
            ip = img.ctypes.data_as(C.c_void_p)
        _check(lib().orc_set_particles(self._h, x, v, ip), "orc_set_particles")

    def particles(self):
        x = np.zeros((3, max(self.N, 1)))
        v = np.zeros((3, max(self.N, 1)))
        img = np.zeros((3, max(self.N, 1)), np.int32)
        lib().orc_get_particles(self._h, x, v, img)
        return x[:, :self.N], v[:, :self.N], img[:, :self.N]

    def set_populations(self, f):
        f = np.ascontiguousarray(f, np.float64).reshape(19, self.nsites)
        lib().orc_set_populations(self._h, f)

    def populations(self):
        f = np.zeros((19, self.nsites))
        lib().orc_get_populations(self._h, f)
        return f

    def J(self):
        J = np.zeros((3, self.nsites))
        lib().orc_get_J(self._h, J)
        return J

    def set_J(self, J):
        lib().orc_set_J(self._h, np.ascontiguousarray(J, np.float64).reshape(3, self.nsites))

    def counters(self):
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32()
        lib().orc_counters(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d))
        return dict(t_lb=a.value, t_md=b.value, subs=c.value, nonfinite=d.value)

    def set_counters(self, t_lb, t_md, subs):
        lib().orc_set_counters(self._h, t_lb, t_md, subs)

    # steps ---------------------------------------------------------------
    def lb_step(self):
        return lib().orc_lb_step(self._h)

    def md_couple_substep(self):
        return lib().orc_md_couple_substep(self._h)

    def cycle(self, ncycles=1):
        for _ in range(ncycles):
            if self.N > 0:
                for _ in range(self.prm["n_sub"]):
                    rc = self.md_couple_substep()
                    if rc not in (0, -5):
                        raise OracleError(f"md_couple_substep returned {rc}")
            _check(self.lb_step(), "orc_lb_step")

    def lb_step_sampled(self, sites):
        sites = np.ascontiguousarray(sites, np.int64)
        out = np.zeros((len(sites), 19))
        _check(lib().orc_lb_step_sampled(self._h, len(sites), sites, out), "sampled")
        return out

    def collide_site(self, f, J, site=0, step=0):
        out = np.zeros(19)
        lib().orc_collide_site(self._h, site, step, np.ascontiguousarray(f, np.float64),
                               np.ascontiguousarray(J, np.float64), out)
        return out

    def cube_weights(self, R):
        sites = np.zeros(8, np.int64)
        w = np.zeros(8)
        lib().orc_cube_weights(self._h, np.ascontiguousarray(R, np.float64), sites, w)
        return sites, w

    def stencil3_weights(self, R):
        sites = np.zeros(27, np.int64)
        w = np.zeros(27)
        lib().orc_stencil3_weights(self._h, np.ascontiguousarray(R, np.float64), sites, w)
        return sites, w

    def moments(self, fields=False):
        tot = np.zeros(NTOTALS)
        if fields:
            rho = np.zeros(self.nsites)
            u = np.zeros((3, self.nsites))
            lib().orc_moments(self._h, rho.ctypes.data_as(C.c_void_p),
                              u.ctypes.data_as(C.c_void_p), tot.ctypes.data_as(C.c_void_p))
            return tot, rho, u
        lib().orc_moments(self._h, None, None, tot.ctypes.data_as(C.c_void_p))
        return tot
