"""Python binding of the C ABI in include/md.h (argument marshalling only).

Every step of the computation runs in the HIP library libmd.so; this module
converts numpy arrays to pointers and status codes to exceptions.  It fails
loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmd.so")

SURF = {"none": 0, "plane": 1, "sphere": 2, "ellipsoid": 3, "torus": 4, "cylinder": 5, "height": 6, "bridge": 7}
PAIR = {"none": 0, "lj": 1, "lj_smooth": 2}

MD_OK, MD_EINVAL, MD_ESTATE, MD_EOFFSURF, MD_ENEWTON, MD_ENAN, MD_ENOMEM, MD_EAGAIN, MD_EHIP, MD_ENOTFOUND = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
SYMBOLS = ["md_create", "md_set_surface", "md_set_particles", "md_step", "md_get_state", "md_destroy",
           "md_strerror", "md_job_footprint", "md_pool_create", "md_pool_admit", "md_pool_run", "md_pool_poll",
           "md_pool_fetch", "md_pool_release", "md_pool_usage", "md_pool_destroy", "md_get_stats",
           "md_pool_get_stats", "md_tune", "md_set_model", "md_set_particles_dev", "md_get_state_dev",
           "md_get_state_dev_noalloc", "md_pool_launch", "md_pool_fetch_many"]
MD_MAX_TYPES = 4


class MDError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class _Params(C.Structure):
    _fields_ = [
        ("dt", C.c_double), ("kT", C.c_double), ("gamma", C.c_double),
        ("eps", C.c_double), ("sigma", C.c_double), ("rc", C.c_double),
        ("pair_kind", C.c_int), ("force_fp64", C.c_int), ("skin", C.c_double),
        ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3), ("periodic", C.c_int * 3),
        ("seed", C.c_uint64), ("newton_tol", C.c_double), ("newton_max_iter", C.c_int), ("newton_frozen", C.c_int),
        ("device", C.c_int), ("stream", C.c_void_p),
    ]


class _Diag(C.Structure):
    _fields_ = [
        ("K", C.c_double), ("U", C.c_double), ("ndof", C.c_double), ("kT", C.c_double),
        ("gdist_max", C.c_double), ("nv_max", C.c_double), ("step", C.c_int64), ("rebuilds", C.c_int64),
        ("newton_iter_max", C.c_int), ("nlist_max", C.c_int), ("error_index", C.c_int),
        ("exact_sum_breaches", C.c_int), ("error_step", C.c_int64),
    ]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class _Stats(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("particle_steps", C.c_int64), ("step_launches", C.c_int64),
        ("chunks", C.c_int64), ("builds", C.c_int64), ("step_kernel_ms", C.c_double),
        ("rebuild_ms", C.c_double), ("nl_mean", C.c_double), ("step_variant", C.c_int), ("step_waves", C.c_int),
        ("step_halo_lds", C.c_int), ("list_capacity", C.c_int), ("skin", C.c_double), ("reserved", C.c_double),
    ]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class _Model(C.Structure):
    _fields_ = [
        ("ntypes", C.c_int), ("beads_per_molecule", C.c_int), ("sigma", C.c_double * MD_MAX_TYPES),
        ("eps", (C.c_double * MD_MAX_TYPES) * MD_MAX_TYPES), ("rc", (C.c_double * MD_MAX_TYPES) * MD_MAX_TYPES),
        ("kb", C.c_double), ("r0", (C.c_double * MD_MAX_TYPES) * MD_MAX_TYPES), ("ka", C.c_double),
        ("theta0", C.c_double), ("wall_eps", C.c_double), ("wall_sigma", C.c_double), ("wall_radius", C.c_double),
    ]


@dataclass
class Model:
    """Bead model of md_set_model: bead sizes by type, LJ well depth (eps for
    every type pair, eps_pairs overriding pairs), per-pair cut-offs rc (absent:
    purely repulsive), linear molecules of beads_per_molecule consecutive
    particles with bond stiffness kb, rest lengths r0 (absent: the default of
    the header), bend stiffness ka about theta0, and the repulsive wall."""
    sigma: tuple = (1.0,)
    eps: float = 1.0
    eps_pairs: dict = field(default_factory=dict)
    rc: dict = field(default_factory=dict)
    beads_per_molecule: int = 0
    kb: float = 0.0
    r0: dict = field(default_factory=dict)
    ka: float = 0.0
    theta0: float = 3.141592653589793
    wall_eps: float = 0.0
    wall_sigma: float = 1.0
    wall_radius: float = 0.0

    def to_c(self) -> _Model:
        m = _Model()
        m.ntypes = len(self.sigma)
        m.beads_per_molecule = int(self.beads_per_molecule)
        for a, v in enumerate(self.sigma):
            m.sigma[a] = float(v)
        for a in range(MD_MAX_TYPES):
            for b in range(MD_MAX_TYPES):
                m.eps[a][b] = float(self.eps)
        for table, src in ((m.eps, self.eps_pairs), (m.rc, self.rc), (m.r0, self.r0)):
            for (a, b), v in src.items():
                table[a][b] = table[b][a] = float(v)
        m.kb, m.ka, m.theta0 = float(self.kb), float(self.ka), float(self.theta0)
        m.wall_eps, m.wall_sigma, m.wall_radius = float(self.wall_eps), float(self.wall_sigma), float(self.wall_radius)
        return m


class _JobDesc(C.Structure):
    _fields_ = [
        ("params", _Params), ("surface_kind", C.c_int), ("surface_prm", C.c_double * 8),
        ("n", C.c_int64), ("x", C.POINTER(C.c_double)), ("p", C.POINTER(C.c_double)),
        ("mass", C.POINTER(C.c_double)), ("constrained", C.POINTER(C.c_uint8)),
        ("step0", C.c_int64), ("nsteps", C.c_int64),
        ("model", C.c_void_p), ("types", C.POINTER(C.c_uint8)),
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
    force_fp64: int = 1
    skin: float = 0.3
    box_lo: tuple = (0.0, 0.0, 0.0)
    box_hi: tuple = (0.0, 0.0, 0.0)
    periodic: tuple = (0, 0, 0)
    seed: int = 0
    newton_tol: float = 0.0
    newton_max_iter: int = 32
    newton_frozen: int = 0
    device: int = 0
    stream: int | None = None

    def to_c(self) -> _Params:
        p = _Params()
        p.dt, p.kT, p.gamma = self.dt, self.kT, self.gamma
        p.eps, p.sigma, p.rc = self.eps, self.sigma, self.rc
        p.pair_kind = PAIR[self.pair]
        p.force_fp64 = int(self.force_fp64)
        p.skin = self.skin
        for k in range(3):
            p.box_lo[k] = float(self.box_lo[k])
            p.box_hi[k] = float(self.box_hi[k])
            p.periodic[k] = int(self.periodic[k])
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        p.newton_tol = self.newton_tol
        p.newton_max_iter = self.newton_max_iter
        p.newton_frozen = int(self.newton_frozen)
        p.device = self.device
        p.stream = self.stream
        return p


_lib = None


def lib():
    """Load libmd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH}; build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        u8 = C.POINTER(C.c_uint8)
        vp = C.c_void_p
        L.md_strerror.argtypes = [C.c_int]
        L.md_strerror.restype = C.c_char_p
        L.md_create.argtypes = [C.POINTER(_Params), C.POINTER(vp)]
        L.md_set_surface.argtypes = [vp, C.c_int, dp, C.c_int]
        L.md_set_particles.argtypes = [vp, C.c_int64, dp, dp, dp, u8, dp, C.c_int64]
        L.md_set_model.argtypes = [vp, C.POINTER(_Model), u8, C.c_int64]
        L.md_set_particles_dev.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, C.c_int64]
        L.md_get_state_dev.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_int64), C.POINTER(_Diag)]
        L.md_get_state_dev_noalloc.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_int64), C.POINTER(_Diag)]
        L.md_step.argtypes = [vp, C.c_int64]
        L.md_get_state.argtypes = [vp, dp, dp, dp, C.POINTER(C.c_int64), C.POINTER(_Diag)]
        L.md_destroy.argtypes = [vp]
        L.md_destroy.restype = None
        L.md_job_footprint.argtypes = [C.c_int64, C.c_int, dp, C.POINTER(_Params)]
        L.md_job_footprint.restype = C.c_size_t
        L.md_pool_create.argtypes = [C.c_size_t, C.c_int, C.c_int, vp, C.POINTER(vp)]
        L.md_pool_admit.argtypes = [vp, C.POINTER(_JobDesc), C.POINTER(C.c_int)]
        L.md_pool_run.argtypes = [vp, C.c_int]
        L.md_pool_launch.argtypes = [vp, C.c_int]
        L.md_pool_fetch_many.argtypes = [vp, C.POINTER(C.c_int), C.c_int, C.POINTER(dp), C.POINTER(dp),
                                         C.POINTER(_Diag), C.POINTER(C.c_int)]
        L.md_pool_poll.argtypes = [vp, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int)]
        L.md_pool_fetch.argtypes = [vp, C.c_int, dp, dp, C.POINTER(_Diag)]
        L.md_pool_release.argtypes = [vp, C.c_int]
        L.md_pool_usage.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]
        L.md_get_stats.argtypes = [vp, C.POINTER(_Stats)]
        L.md_tune.argtypes = [vp, C.c_int, dp, C.c_int, dp, dp]
        L.md_pool_get_stats.argtypes = [vp, C.POINTER(_Stats)]
        L.md_pool_destroy.argtypes = [vp]
        L.md_pool_destroy.restype = None
        for name in ("md_create", "md_set_surface", "md_set_particles", "md_set_model", "md_step", "md_get_state",
                     "md_set_particles_dev", "md_get_state_dev", "md_get_state_dev_noalloc",
                     "md_pool_create", "md_pool_admit", "md_pool_run", "md_pool_launch", "md_pool_poll",
                     "md_pool_fetch", "md_pool_fetch_many",
                     "md_pool_release", "md_pool_usage", "md_get_stats", "md_pool_get_stats", "md_tune"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def hip_runtime():
    """The HIP runtime libmd.so runs on (the already loaded library of that
    soname), for device buffers and synchronisation that must share it."""
    lib()
    return C.CDLL("libamdhip64.so.7")


def strerror(code: int) -> str:
    return lib().md_strerror(code).decode()


def _check(rc: int, what: str):
    if rc != MD_OK:
        raise MDError(rc, what)


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_uint8))


def _vec(a, n):
    return np.ascontiguousarray(a, dtype=np.float64).reshape(n, 3)


def _surf_prm(surf):
    q = (C.c_double * 8)()
    for k, v in enumerate(list(surf)[:8]):
        q[k] = float(v)
    return q


class System:
    """One system: md_create / md_set_surface / md_set_particles / md_step / md_get_state."""

    def __init__(self, params: Params, surface: str = "none", surf=()):
        self._h = C.c_void_p()
        self._cp = params.to_c()
        _check(lib().md_create(C.byref(self._cp), C.byref(self._h)), "md_create")
        self.n = 0
        if surface != "none" or surf:
            self.set_surface(surface, surf)

    def set_surface(self, surface: str, surf):
        q = np.ascontiguousarray(list(surf) + [0.0] * (8 - len(surf)), dtype=np.float64)
        _check(lib().md_set_surface(self._h, SURF[surface], _dp(q), len(surf)), "md_set_surface")

    def set_model(self, model: Model | None, types=None):
        """Bead model and per-particle types for the next set_particles."""
        if model is None:
            _check(lib().md_set_model(self._h, None, None, 0), "md_set_model")
            return
        t = np.ascontiguousarray(types, dtype=np.uint8).reshape(-1)
        self._model = model.to_c()
        _check(lib().md_set_model(self._h, C.byref(self._model), _u8(t), t.shape[0]), "md_set_model")

    def set_particles(self, x, p, mass=None, cons=None, fcomb=None, step0=0):
        x = np.asarray(x)
        n = x.shape[0]
        x = _vec(x, n)
        p = _vec(p, n)
        m = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64).reshape(n)
        c = None if cons is None else np.ascontiguousarray(cons, dtype=np.uint8).reshape(n)
        f = None if fcomb is None else _vec(fcomb, n)
        _check(lib().md_set_particles(self._h, n, _dp(x), _dp(p), _dp(m), _u8(c), _dp(f), int(step0)),
               "md_set_particles")
        self.n = n

    def set_particles_dev(self, n: int, x_ptr: int, p_ptr: int, mass_ptr: int | None = None,
                          cons_ptr: int | None = None, fcomb_ptr: int | None = None, step0: int = 0):
        """md_set_particles_dev: device addresses (e.g. tensor.data_ptr()) of
        contiguous arrays with the host layouts (x, p, fcomb: n*3 float64;
        mass: n float64; cons: n uint8)."""
        _check(lib().md_set_particles_dev(self._h, int(n), x_ptr, p_ptr, mass_ptr, cons_ptr, fcomb_ptr, int(step0)),
               "md_set_particles_dev")
        self.n = int(n)

    def get_state_dev(self, x_ptr: int | None, p_ptr: int | None, fcomb_ptr: int | None = None):
        """md_get_state_dev into device addresses; returns step and diagnostics."""
        step = C.c_int64(0)
        d = _Diag()
        _check(lib().md_get_state_dev(self._h, x_ptr, p_ptr, fcomb_ptr, C.byref(step), C.byref(d)), "md_get_state_dev")
        return dict(step=step.value, diag=d.to_dict())

    def get_state_dev_noalloc(self, x_ptr: int | None, p_ptr: int | None, fcomb_ptr: int | None = None):
        """md_get_state_dev_noalloc into device addresses (allocates no device
        memory); returns step and diagnostics."""
        step = C.c_int64(0)
        d = _Diag()
        _check(lib().md_get_state_dev_noalloc(self._h, x_ptr, p_ptr, fcomb_ptr, C.byref(step), C.byref(d)),
               "md_get_state_dev_noalloc")
        return dict(step=step.value, diag=d.to_dict())

    def step(self, nsteps: int):
        _check(lib().md_step(self._h, int(nsteps)), "md_step")

    def get_state(self, want_force: bool = True):
        n = self.n
        x = np.zeros((n, 3))
        p = np.zeros((n, 3))
        f = np.zeros((n, 3)) if want_force else None
        step = C.c_int64(0)
        d = _Diag()
        rc = lib().md_get_state(self._h, _dp(x), _dp(p), _dp(f), C.byref(step), C.byref(d))
        # after a device error (Newton cap, non-finite state) the state and the
        # diagnostics naming the failing step and particle are still returned
        if rc not in (MD_OK, MD_ENEWTON, MD_ENAN):
            _check(rc, "md_get_state")
        return dict(x=x, p=p, f=f, step=step.value, diag=d.to_dict(), status=rc)

    def stats(self):
        st = _Stats()
        _check(lib().md_get_stats(self._h, C.byref(st)), "md_get_stats")
        return st.to_dict()

    def tune(self, trial_steps: int, skins=None):
        """md_tune: the FP32-class step-kernel instance, then the list skin, on the
        live system; returns (best skin, GPU microseconds per step)."""
        arr = None if skins is None else np.ascontiguousarray(skins, dtype=np.float64)
        best = C.c_double(0.0)
        us = C.c_double(0.0)
        _check(lib().md_tune(self._h, int(trial_steps), _dp(arr), 0 if arr is None else len(arr), C.byref(best),
                             C.byref(us)), "md_tune")
        return best.value, us.value

    def close(self):
        if self._h:
            lib().md_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(n: int, surface: str, surf, params: Params) -> int:
    q = _surf_prm(surf)
    cp = params.to_c()
    return int(lib().md_job_footprint(int(n), SURF[surface], q, C.byref(cp)))


class Pool:
    """Many jobs resident on one device, advanced together (md_pool_*)."""

    def __init__(self, budget_bytes: int, max_jobs: int, device: int = 0, stream: int | None = None):
        self._h = C.c_void_p()
        _check(lib().md_pool_create(int(budget_bytes), int(max_jobs), int(device), stream, C.byref(self._h)),
               "md_pool_create")
        self._keep = {}

    def admit(self, params: Params, surface: str, surf, x, p, nsteps: int, step0: int = 0, mass=None, cons=None,
              model: "Model | None" = None, types=None):
        """Returns the job id, or None when the pool has no room (MD_EAGAIN)."""
        x = np.asarray(x)
        n = x.shape[0]
        d = _JobDesc()
        d.params = params.to_c()
        d.surface_kind = SURF[surface]
        d.surface_prm = _surf_prm(surf)
        xs, ps = _vec(x, n), _vec(p, n)
        m = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64).reshape(n)
        c = None if cons is None else np.ascontiguousarray(cons, dtype=np.uint8).reshape(n)
        d.n = n
        d.x, d.p, d.mass, d.constrained = _dp(xs), _dp(ps), _dp(m), _u8(c)
        d.step0, d.nsteps = int(step0), int(nsteps)
        keep = None
        if model is not None:
            mc = model.to_c()
            t = np.ascontiguousarray(types, dtype=np.uint8).reshape(n)
            d.model = C.cast(C.pointer(mc), C.c_void_p)
            d.types = _u8(t)
            keep = (mc, t)  # alive until md_pool_admit has copied them
        jid = C.c_int(-1)
        rc = lib().md_pool_admit(self._h, C.byref(d), C.byref(jid))
        del keep
        if rc == MD_EAGAIN:
            return None
        _check(rc, "md_pool_admit")
        self._keep[jid.value] = n
        return jid.value

    def run(self, steps: int):
        _check(lib().md_pool_run(self._h, int(steps)), "md_pool_run")

    def launch(self, steps: int):
        """md_pool_launch: enqueue one chunk and return without waiting (the next
        poll, fetch, release or run completes it)."""
        _check(lib().md_pool_launch(self._h, int(steps)), "md_pool_launch")

    def poll(self, cap: int = 4096):
        ids = (C.c_int * cap)()
        nd = C.c_int(0)
        _check(lib().md_pool_poll(self._h, ids, cap, C.byref(nd)), "md_pool_poll")
        return [ids[k] for k in range(nd.value)]

    def fetch(self, job: int):
        n = self._keep[job]
        x = np.zeros((n, 3))
        p = np.zeros((n, 3))
        d = _Diag()
        rc = lib().md_pool_fetch(self._h, int(job), _dp(x), _dp(p), C.byref(d))
        return rc, dict(x=x, p=p, diag=d.to_dict())

    def fetch_many(self, jobs):
        """md_pool_fetch_many: [(status, dict(x, p, diag))] for the given job ids,
        with one wait for all of them."""
        jobs = [int(j) for j in jobs]
        n = len(jobs)
        if n == 0:
            return []
        xs = [np.zeros((self._keep.get(j, 0), 3)) for j in jobs]
        ps = [np.zeros((self._keep.get(j, 0), 3)) for j in jobs]
        ids = (C.c_int * n)(*jobs)
        DP = C.POINTER(C.c_double)
        xa = (DP * n)(*[_dp(a) for a in xs])
        pa = (DP * n)(*[_dp(a) for a in ps])
        ds = (_Diag * n)()
        st = (C.c_int * n)()
        _check(lib().md_pool_fetch_many(self._h, ids, n, xa, pa, ds, st), "md_pool_fetch_many")
        return [(st[q], dict(x=xs[q], p=ps[q], diag=ds[q].to_dict())) for q in range(n)]

    def release(self, job: int):
        _check(lib().md_pool_release(self._h, int(job)), "md_pool_release")
        self._keep.pop(job, None)

    def usage(self):
        j = C.c_int(0)
        n = C.c_int64(0)
        b = C.c_size_t(0)
        _check(lib().md_pool_usage(self._h, C.byref(j), C.byref(n), C.byref(b)), "md_pool_usage")
        return dict(jobs=j.value, particles=n.value, bytes=b.value)

    def stats(self):
        st = _Stats()
        _check(lib().md_pool_get_stats(self._h, C.byref(st)), "md_pool_get_stats")
        return st.to_dict()

    def close(self):
        if self._h:
            lib().md_pool_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
