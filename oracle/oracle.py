"""ctypes binding of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports this module.

Arrays are numpy float64 in AoS layout, shape (n, 3).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

SURF = {"none": 0, "plane": 1, "sphere": 2, "ellipsoid": 3, "torus": 4, "cylinder": 5, "height": 6, "bridge": 7}
PAIR = {"none": 0, "lj": 1, "lj_smooth": 2}


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
        os.path.getmtime(SRC_PATH), os.path.getmtime(os.path.join(HERE, "mdo.h"))
    ):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-o", tmp, SRC_PATH, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


MAX_TYPES = 4


class _Model(C.Structure):
    _fields_ = [
        ("ntypes", C.c_int), ("bpm", C.c_int), ("sigma", C.c_double * MAX_TYPES),
        ("eps", (C.c_double * MAX_TYPES) * MAX_TYPES),
        ("rc", (C.c_double * MAX_TYPES) * MAX_TYPES), ("kb", C.c_double),
        ("r0", (C.c_double * MAX_TYPES) * MAX_TYPES), ("ka", C.c_double), ("theta0", C.c_double),
        ("wall_eps", C.c_double), ("wall_sigma", C.c_double), ("wall_radius", C.c_double),
    ]


@dataclass
class Model:
    """Bead model (capsid example of the SI): see mdo.h."""
    sigma: tuple = (1.0,)
    eps: float = 1.0                            # well depth of the pairs not in eps_pairs
    eps_pairs: dict = field(default_factory=dict)  # {(a, b): eps}
    rc: dict = field(default_factory=dict)      # {(a, b): rc}; absent: 2^(1/6) sigma_ab
    bpm: int = 0
    kb: float = 0.0
    r0: dict = field(default_factory=dict)      # {(a, b): r0}; absent: 2^(1/6) (sigma_a + sigma_b) / 4
    ka: float = 0.0
    theta0: float = math.pi
    wall_eps: float = 0.0
    wall_sigma: float = 1.0
    wall_radius: float = 0.0

    def to_c(self) -> _Model:
        m = _Model()
        m.ntypes = len(self.sigma)
        m.bpm = self.bpm
        for a, s in enumerate(self.sigma):
            m.sigma[a] = s
        for a in range(MAX_TYPES):
            for b in range(MAX_TYPES):
                m.eps[a][b] = self.eps
        for (a, b), v in self.eps_pairs.items():
            m.eps[a][b] = m.eps[b][a] = v
        for (a, b), v in self.rc.items():
            m.rc[a][b] = m.rc[b][a] = v
        m.kb = self.kb
        for (a, b), v in self.r0.items():
            m.r0[a][b] = m.r0[b][a] = v
        m.ka, m.theta0 = self.ka, self.theta0
        m.wall_eps, m.wall_sigma, m.wall_radius = self.wall_eps, self.wall_sigma, self.wall_radius
        return m


class _Params(C.Structure):
    _fields_ = [
        ("dt", C.c_double), ("kT", C.c_double), ("gamma", C.c_double),
        ("eps", C.c_double), ("sigma", C.c_double), ("rc", C.c_double),
        ("pair", C.c_int), ("surface", C.c_int),
        ("surf", C.c_double * 8), ("gscale", C.c_double),
        ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
        ("periodic", C.c_int * 3),
        ("seed", C.c_uint64), ("eta", C.c_double), ("max_iter", C.c_int),
        ("use_cells", C.c_int), ("frozen", C.c_int),
        ("model", _Model), ("types", C.POINTER(C.c_uint8)),
    ]


@dataclass
class Params:
    dt: float = 0.001
    kT: float = 1.0
    gamma: float = 1.0
    eps: float = 1.0
    sigma: float = 1.0
    rc: float = 2.0 ** (1.0 / 6.0)
    pair: str = "lj"
    surface: str = "sphere"
    surf: tuple = (0.0, 0.0, 0.0, 1.0)
    gscale: float = 1.0
    box_lo: tuple = (0.0, 0.0, 0.0)
    box_hi: tuple = (0.0, 0.0, 0.0)
    periodic: tuple = (0, 0, 0)
    seed: int = 0
    eta: float = 0.0
    max_iter: int = 32
    use_cells: int = 1
    frozen: int = 0
    model: Model | None = None
    types: np.ndarray | None = None

    def to_c(self) -> _Params:
        p = _Params()
        p.dt, p.kT, p.gamma = self.dt, self.kT, self.gamma
        p.eps, p.sigma, p.rc = self.eps, self.sigma, self.rc
        p.pair = PAIR[self.pair]
        p.surface = SURF[self.surface]
        s = list(self.surf) + [0.0] * (8 - len(self.surf))
        for k in range(8):
            p.surf[k] = float(s[k])
        p.gscale = self.gscale
        for k in range(3):
            p.box_lo[k] = float(self.box_lo[k])
            p.box_hi[k] = float(self.box_hi[k])
            p.periodic[k] = int(self.periodic[k])
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        p.eta = self.eta
        p.max_iter = self.max_iter
        p.use_cells = self.use_cells
        p.frozen = self.frozen
        if self.model is not None:
            p.model = self.model.to_c()
        if self.types is not None:
            self._types_c = np.ascontiguousarray(self.types, dtype=np.uint8)
            p.types = self._types_c.ctypes.data_as(C.POINTER(C.c_uint8))
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        u8p = C.POINTER(C.c_uint8)
        u32p = C.POINTER(C.c_uint32)
        i64p = C.POINTER(C.c_int64)
        pp = C.POINTER(_Params)
        L.mdo_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.mdo_threads.restype = C.c_int
        L.mdo_set_threads.argtypes = [C.c_int]
        L.mdo_set_threads.restype = None
        L.mdo_philox4x32_10.restype = None
        L.mdo_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, dp]
        L.mdo_normals.restype = None
        L.mdo_surface_g.argtypes = [pp, dp, dp]
        L.mdo_surface_g.restype = C.c_double
        L.mdo_forces.argtypes = [pp, C.c_int64, dp, dp, dp, dp]
        L.mdo_init_force.argtypes = [pp, C.c_int64, dp, dp, dp, u8p, C.c_int64, dp]
        L.mdo_position_stage.argtypes = [pp, dp, dp, dp, C.c_double, dp, dp, dp, C.POINTER(C.c_int)]
        L.mdo_momentum_stage.argtypes = [pp, dp, dp, dp, C.c_double, dp, dp, C.POINTER(C.c_int)]
        L.mdo_run.argtypes = [pp, C.c_int64, dp, dp, dp, dp, u8p, i64p, C.c_int64, C.POINTER(C.c_int)]
        L.mdo_diag.argtypes = [pp, C.c_int64, dp, dp, dp, u8p, dp]
        for name in ("mdo_forces", "mdo_init_force", "mdo_position_stage", "mdo_momentum_stage",
                     "mdo_run", "mdo_diag"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def threads() -> int:
    """OpenMP threads of the oracle's parallel loops."""
    return int(lib().mdo_threads())


def set_threads(n: int):
    lib().mdo_set_threads(int(n))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    out = (C.c_uint32 * 4)()
    lib().mdo_philox4x32_10(c, k, out)
    return [int(v) for v in out]


def normals(seed, pid, step):
    z = np.zeros(3)
    lib().mdo_normals(C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), C.c_uint32(pid), C.c_int64(step), _d(z))
    return z


def surface_g(P: Params, x):
    x = _f64(x, (3,))
    grad = np.zeros(3)
    cp = P.to_c()
    g = lib().mdo_surface_g(C.byref(cp), _d(x), _d(grad))
    return g, grad


def forces(P: Params, x):
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    F = np.zeros((n, 3))
    up = np.zeros(n)
    U = C.c_double(0.0)
    cp = P.to_c()
    _check(lib().mdo_forces(C.byref(cp), n, _d(x), _d(F), _d(up), C.byref(U)), "mdo_forces")
    return F, U.value, up


def _opt_mass(mass, n):
    if mass is None:
        return None, None
    m = _f64(mass, (n,))
    return m, _d(m)


def _opt_cons(cons, n):
    if cons is None:
        return None, None
    c = np.ascontiguousarray(cons, dtype=np.uint8).reshape(n)
    return c, c.ctypes.data_as(C.POINTER(C.c_uint8))


def init_force(P: Params, x, p, mass=None, cons=None, step0=0):
    x = _f64(x, (-1, 3))
    p = _f64(p, (-1, 3))
    n = x.shape[0]
    f = np.zeros((n, 3))
    m, mp = _opt_mass(mass, n)
    c, cp_ = _opt_cons(cons, n)
    cp = P.to_c()
    _check(lib().mdo_init_force(C.byref(cp), n, _d(x), _d(p), mp, cp_, step0, _d(f)), "mdo_init_force")
    return f


def position_stage(P: Params, xm, pm, fm, m=1.0):
    xm, pm, fm = _f64(xm, (3,)), _f64(pm, (3,)), _f64(fm, (3,))
    xn, ph = np.zeros(3), np.zeros(3)
    lam = C.c_double(0.0)
    it = C.c_int(0)
    cp = P.to_c()
    rc = lib().mdo_position_stage(C.byref(cp), _d(xm), _d(pm), _d(fm), m, _d(xn), _d(ph), C.byref(lam),
                                  C.byref(it))
    _check(rc, "mdo_position_stage")
    return xn, ph, lam.value, it.value


def momentum_stage(P: Params, xn, ph, fn, m=1.0):
    xn, ph, fn = _f64(xn, (3,)), _f64(ph, (3,)), _f64(fn, (3,))
    pn = np.zeros(3)
    mu = C.c_double(0.0)
    it = C.c_int(0)
    cp = P.to_c()
    rc = lib().mdo_momentum_stage(C.byref(cp), _d(xn), _d(ph), _d(fn), m, _d(pn), C.byref(mu), C.byref(it))
    _check(rc, "mdo_momentum_stage")
    return pn, mu.value, it.value


class State:
    """Oracle state (x^m, p^m, f^m, m) for one system."""

    def __init__(self, P: Params, x, p, mass=None, cons=None, step0=0, f=None):
        self.P = P
        self.x = _f64(x, (-1, 3)).copy()
        self.p = _f64(p, (-1, 3)).copy()
        self.n = self.x.shape[0]
        self.mass = None if mass is None else _f64(mass, (self.n,)).copy()
        self.cons = None if cons is None else np.ascontiguousarray(cons, dtype=np.uint8).reshape(self.n).copy()
        self.step = int(step0)
        self.f = (init_force(P, self.x, self.p, self.mass, self.cons, step0) if f is None
                  else _f64(f, (-1, 3)).copy())
        self.max_iter_seen = 0

    def run(self, nsteps):
        stepc = C.c_int64(self.step)
        it = C.c_int(0)
        cp = self.P.to_c()
        _, mp = _opt_mass(self.mass, self.n)
        _, cp_ = _opt_cons(self.cons, self.n)
        rc = lib().mdo_run(C.byref(cp), self.n, _d(self.x), _d(self.p), _d(self.f), mp, cp_,
                           C.byref(stepc), int(nsteps), C.byref(it))
        self.step = stepc.value
        self.max_iter_seen = max(self.max_iter_seen, it.value)
        _check(rc, "mdo_run")
        return self

    def diag(self):
        out = np.zeros(6)
        cp = self.P.to_c()
        _, mp = _opt_mass(self.mass, self.n)
        _, cp_ = _opt_cons(self.cons, self.n)
        _check(lib().mdo_diag(C.byref(cp), self.n, _d(self.x), _d(self.p), mp, cp_, _d(out)), "mdo_diag")
        return dict(K=out[0], U=out[1], ndof=out[2], kT=out[3], gdist=out[4], nv=out[5])
